"""Large-width maps by recursive filtering (Section 3.1: for large kernel
widths, recursive filters replace the finite masks; the paper cites Deriche
and van Vliet).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it, and it
imports nothing from the product.

The filter is Young and van Vliet's third-order recursive Gaussian (1995): a
causal pass w[n] = B x[n] + a1 w[n-1] + a2 w[n-2] + a3 w[n-3] followed by the
anticausal pass y[n] = B w[n] + a1 y[n+1] + a2 y[n+2] + a3 y[n+3], with
coefficients from q(sigma) (their eqs. for q and b0..b3) and unit DC gain.
It approximates the normalised Gaussian; it is a different kernel from the
sampled masks, so the recursive maps have their own oracle here.

Readings (listed with the design notes):
* boundaries: the signal is zero outside the lattice; each line is extended by
  m = ceil(6 sigma) zeros at its end so that the causal response has decayed
  before the anticausal pass starts (zero state at both ends);
* scale: outputs are multiplied by sqrt(2 pi) sigma per axis, the mass of the
  unnormalised sampled Gaussian used by the direct maps (the update and D do
  not depend on it);
* moments: M = -sigma^2 grad A (exact for a Gaussian kernel), with the
  gradient by central differences; A is filtered on the lattice grown by a
  one-pixel ring of zero weights, so the differences at the border use the
  smoothed density just outside it;
* S_X = sum h A as for the direct maps.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["yvv_q", "yvv_b", "yvv_coefficients", "yvv_filter_1d", "recursive_density", "recursive_maps"]

# Young and van Vliet's published constants. Q_FIT: the two branches of
# their empirical width relation q(sigma). B_POLY: b0..b3 as polynomials in q.
# The polynomials are pinned exactly against the filter's factored pole form
# (tests/test_oracle_recursive.py). The q(sigma) relation is an empirical fit;
# it is pinned only to within a few per cent of an independent least-squares
# fit of q, so its constants are parity unpinned beyond that band.
Q_FIT = (0.98711, 0.96330, 3.97156, 4.14554, 0.26891)
B_POLY = (1.57825, 2.44413, 1.4281, 0.422205, 2.85619, 1.26661)


def yvv_q(sigma: float) -> float:
    """q(sigma): q = 0.98711 sigma - 0.96330 for sigma >= 2.5, else 3.97156 - 4.14554 sqrt(1 - 0.26891 sigma)."""
    k1, k0, c0, c1, c2 = Q_FIT
    if sigma >= 2.5:
        return k1 * sigma - k0
    return c0 - c1 * math.sqrt(1.0 - c2 * sigma)


def yvv_b(q: float):
    """(b0, b1, b2, b3) of the recursion for parameter q."""
    p0, p1, p2, p3, p4, p5 = B_POLY
    b0 = p0 + p1 * q + p2 * q * q + p3 * q ** 3
    b1 = p1 * q + p4 * q * q + p5 * q ** 3
    b2 = -(p2 * q * q + p5 * q ** 3)
    b3 = p3 * q ** 3
    return b0, b1, b2, b3


def yvv_coefficients(sigma: float):
    """(B, a1, a2, a3) of the Young-van Vliet recursive Gaussian for width sigma >= 0.5."""
    b0, b1, b2, b3 = yvv_b(yvv_q(sigma))
    B = 1.0 - (b1 + b2 + b3) / b0
    return B, b1 / b0, b2 / b0, b3 / b0


def yvv_filter_1d(x: np.ndarray, sigma: float) -> np.ndarray:
    """Causal then anticausal pass along the last axis, on the line extended by ceil(6 sigma) zeros."""
    B, a1, a2, a3 = yvv_coefficients(sigma)
    x = np.asarray(x, np.float64)
    n = x.shape[-1]
    m = int(math.ceil(6.0 * sigma))
    xp = np.zeros(x.shape[:-1] + (n + m,))
    xp[..., :n] = x
    w = np.zeros_like(xp)
    for i in range(n + m):
        acc = B * xp[..., i]
        if i >= 1:
            acc = acc + a1 * w[..., i - 1]
        if i >= 2:
            acc = acc + a2 * w[..., i - 2]
        if i >= 3:
            acc = acc + a3 * w[..., i - 3]
        w[..., i] = acc
    y = np.zeros_like(xp)
    for i in range(n + m - 1, -1, -1):
        acc = B * w[..., i]
        if i + 1 < n + m:
            acc = acc + a1 * y[..., i + 1]
        if i + 2 < n + m:
            acc = acc + a2 * y[..., i + 2]
        if i + 3 < n + m:
            acc = acc + a3 * y[..., i + 3]
        y[..., i] = acc
    return y[..., :n] * (math.sqrt(2.0 * math.pi) * sigma)


def recursive_density(I: np.ndarray, sigma: float) -> np.ndarray:
    """A = the recursive Gaussian of I along v (rows), then along u (columns)."""
    A = yvv_filter_1d(np.asarray(I, np.float64), sigma)
    return yvv_filter_1d(A.T, sigma).T


def recursive_maps(I: np.ndarray, sigma: float):
    """(A, M_u, M_v, S_X): A filtered on the lattice grown by a one-pixel ring,
    M = -sigma^2 grad A by central differences on that ring."""
    I = np.asarray(I, np.float64)
    H, W = I.shape
    Ie = np.zeros((H + 2, W + 2))
    Ie[1:-1, 1:-1] = I
    Ae = recursive_density(Ie, sigma)
    A = Ae[1:-1, 1:-1]
    Mu = -sigma * sigma * 0.5 * (Ae[2:, 1:-1] - Ae[:-2, 1:-1])
    Mv = -sigma * sigma * 0.5 * (Ae[1:-1, 2:] - Ae[1:-1, :-2])
    return A, Mu, Mv, float(np.sum(I * A))
