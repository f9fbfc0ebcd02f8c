import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU check")


@pytest.fixture(scope="session")
def gpu_lib():
    """The HIP library's Python binding; fails loudly when the GPU or library is missing."""
    import torch
    if not torch.cuda.is_available():
        pytest.fail("gpu test selected but torch.cuda is not available")
    from paper_1310_7114_amd import itc
    itc.load()
    return itc
