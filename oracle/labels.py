"""Pixel-to-codevector labelling of a lattice image (the segments the paper
shows for k = 5 codevectors in Section 4).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it, and it
imports nothing from the product.

Readings (listed with the design notes): a pixel with weight > 0 belongs to
the codevector nearest to it in the Euclidean norm (the Voronoi cell of the
codebook, as in vector quantisation); equal distances go to the smaller
index; pixels of weight 0 get -1. Distances are (u - w_u)^2 + (v - w_v)^2 in
FP64 with two rounded products and a rounded sum (exact whenever the
coordinates stay below 2048 and the codebook is FP32), the order the GPU
kernel uses too, so both sides take the same decisions.
"""
from __future__ import annotations

import numpy as np

__all__ = ["label_pixels"]


def label_pixels(I: np.ndarray, W: np.ndarray) -> np.ndarray:
    """int32 (H, W) labels: argmin_k ||x - w_k|| for I(x) > 0 (first k on ties), else -1."""
    I = np.asarray(I)
    Wc = np.asarray(W, np.float64)
    H, Wd = I.shape
    out = np.full((H, Wd), -1, np.int32)
    us, vs = np.nonzero(I > 0)
    for a in range(0, len(us), 4096):
        u = us[a:a + 4096].astype(np.float64)
        v = vs[a:a + 4096].astype(np.float64)
        d2 = (u[:, None] - Wc[None, :, 0]) ** 2 + (v[:, None] - Wc[None, :, 1]) ** 2
        out[us[a:a + 4096], vs[a:a + 4096]] = np.argmin(d2, axis=1)  # first minimum on ties
    return out
