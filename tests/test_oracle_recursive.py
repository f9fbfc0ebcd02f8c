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
import oracle.recursive as OR
from paper_1310_7114_amd import synth as S

# The filter's three poles as Young and van Vliet give them (their m0, m1, m2;
# Signal Processing 44 (1995)): the recursion's denominator is, with z the
# one-sample delay, (m0 + q - q z)((m1 + q)^2 + m2^2 - 2 (m1 + q) q z + q^2 z^2),
# scaled by 0.422205 (= the q^3 coefficient of b0). Expanding it gives the
# b0..b3 polynomials independently of how the oracle writes them.
POLES = (1.16680, 1.10783, 1.40586)
B_SCALE = 0.422205


def b_from_poles(q):
    m0, m1, m2 = POLES
    a, c, d = m0 + q, (m1 + q) ** 2 + m2 * m2, 2.0 * (m1 + q)
    return (B_SCALE * a * c, B_SCALE * q * (a * d + c), -B_SCALE * q * q * (a + d), B_SCALE * q ** 3)


def poly_matches_poles(b_of_q, tol=1e-5):
    for q in (0.1, 0.5, 1.0, 2.0, 5.0, 10.0, 40.0):
        got, ref = np.array(b_of_q(q)), np.array(b_from_poles(q))
        if np.abs(got - ref).max() > tol * np.abs(ref).max():
            return False
    return True


def test_polynomials_equal_the_pole_form():
    """b0..b3(q) equal the expansion of the factored pole form to the printed precision (5-6 digits)."""
    assert poly_matches_poles(OR.yvv_b)


@pytest.mark.parametrize("k", range(6))
@pytest.mark.parametrize("rel", [1e-4, -1e-4, 1e-3])
def test_pole_pin_catches_a_mistyped_constant(monkeypatch, k, rel):
    """A single polynomial constant off by 1e-4 (a digit beyond the fourth) fails the pole-form pin."""
    bad = list(OR.B_POLY)
    bad[k] *= 1.0 + rel
    monkeypatch.setattr(OR, "B_POLY", tuple(bad))
    assert not poly_matches_poles(OR.yvv_b)


def test_width_relation_near_a_least_squares_fit():
    """q(sigma) is an empirical fit: it lies within 3.5 % of the q that best fits the sampled Gaussian
    (least squares over the impulse response) for sigma from 1 to 32, and continues linearly."""
    from scipy.optimize import minimize_scalar

    def response(q, n, c):
        b0, b1, b2, b3 = b_from_poles(q)
        B, a = 1.0 - (b1 + b2 + b3) / b0, (b1 / b0, b2 / b0, b3 / b0)
        x = np.zeros(n)
        x[c] = 1.0
        w = np.zeros(n)
        for i in range(n):
            w[i] = B * x[i] + sum(a[k] * w[i - 1 - k] for k in range(3) if i - 1 - k >= 0)
        y = np.zeros(n)
        for i in range(n - 1, -1, -1):
            y[i] = B * w[i] + sum(a[k] * y[i + 1 + k] for k in range(3) if i + 1 + k < n)
        return y

    for sigma in (1.0, 2.0, 3.0, 6.0, 12.0, 32.0):
        n = int(20 * sigma) + 60
        c = n // 2
        t = np.arange(n) - c
        g = np.exp(-t * t / (2 * sigma * sigma))
        g /= g.sum()
        fit = minimize_scalar(lambda q: float(((response(q, n, c) - g) ** 2).sum()), bounds=(0.05, 3 * sigma + 3),
                              method="bounded", options={"xatol": 1e-7}).x
        assert abs(OR.yvv_q(sigma) / fit - 1.0) <= 0.035, sigma
    assert OR.yvv_q(40.0) - OR.yvv_q(20.0) == pytest.approx(20 * OR.Q_FIT[0], rel=1e-12)


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
