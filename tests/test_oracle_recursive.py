"""Pins of the recursive-Gaussian maps oracle (large widths), CPU only.

The recursive filter approximates the Gaussian, so it is pinned against the
Gaussian itself: unit DC gain (B = 1 - (b1 + b2 + b3)/b0 makes the impulse
response sum to 1), zero phase (the causal/anticausal cascade is symmetric),
and closeness to the sampled normalised Gaussian within a few per cent of its
peak, tightening as sigma grows (the accuracy Young and van Vliet report for
their third-order filter). The maps are pinned against the untruncated direct
maps of the mask oracle (which fix the sign and axes of the moments), and by
transpose equivariance and linearity.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1310_7114_amd import synth as S


@pytest.mark.parametrize("sigma,max_err", [(2.0, 0.06), (4.0, 0.04), (8.0, 0.03), (16.0, 0.02), (32.0, 0.015)])
def test_impulse_response(sigma, max_err):
    n = int(30 * sigma) + 40
    x = np.zeros(n)
    c = n // 2
    x[c] = 1.0
    y = O.yvv_filter_1d(x, sigma) / (math.sqrt(2 * math.pi) * sigma)
    t = np.arange(n) - c
    g = np.exp(-t * t / (2 * sigma * sigma)) / (math.sqrt(2 * math.pi) * sigma)
    assert abs(y.sum() - 1.0) <= 1e-6
    k = min(c, n - 1 - c)
    assert np.abs(y[c - k:c + k + 1] - y[c - k:c + k + 1][::-1]).max() <= 1e-14
    assert np.abs(y - g).max() <= max_err * g.max()


@pytest.mark.parametrize("sigma,tol_a,tol_m", [(4.0, 0.02, 0.06), (8.0, 0.02, 0.05), (16.0, 0.02, 0.04),
                                               (32.0, 0.015, 0.03)])
def test_maps_near_the_gaussian_maps(sigma, tol_a, tol_m):
    img = S.config2_case(0).weights
    A, Mu, Mv, sx = O.recursive_maps(img, sigma)
    Ad = O.lattice_maps(img, sigma, int(math.ceil(7 * sigma)))
    Mu_d, Mv_d = O.moment_maps(*Ad)
    rel = lambda a, b: np.linalg.norm(a - b) / np.linalg.norm(b)  # noqa: E731
    assert rel(A, Ad[0]) <= tol_a
    assert rel(Mu, Mu_d) <= tol_m and rel(Mv, Mv_d) <= tol_m
    assert sx == pytest.approx(float(np.sum(img * A)), rel=1e-12)


def test_transpose_and_linearity():
    rng = np.random.default_rng(0)
    I = rng.uniform(size=(37, 52))
    J = rng.uniform(size=(37, 52))
    A, Mu, Mv, _ = O.recursive_maps(I, 3.3)
    At, Mut, Mvt, _ = O.recursive_maps(I.T, 3.3)
    assert np.allclose(At, A.T, rtol=1e-12, atol=1e-12)
    assert np.allclose(Mut, Mv.T, rtol=1e-12, atol=1e-11) and np.allclose(Mvt, Mu.T, rtol=1e-12, atol=1e-11)
    A2, _, _, _ = O.recursive_maps(2.0 * I + J, 3.3)
    AJ, _, _, _ = O.recursive_maps(J, 3.3)
    assert np.allclose(A2, 2.0 * A + AJ, rtol=1e-12, atol=1e-12)
