"""FP64 CPU oracle for lattice ITC (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package; the product path must never route through it.
"""
from .itc_oracle import *  # noqa: F401,F403
from .itc_oracle import __all__  # noqa: F401
from .chamfer import chamfer_transform  # noqa: F401
from .labels import label_pixels  # noqa: F401
from .volume import (volume_maps, read_trilinear, volume_codebook_terms, volume_step,  # noqa: F401
                     volume_divergence, fit_volume)
from .recursive import yvv_coefficients, yvv_filter_1d, recursive_density, recursive_maps  # noqa: F401
from .literal import (paper_widths, literal_q, literal_terms, literal_step, literal_divergence,  # noqa: F401
                      fit_literal, fit_literal_density)
