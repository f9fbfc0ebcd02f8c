"""The paper's own accelerated ITC (Algorithm 1 with the update eq. (6)).

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it, and it
imports nothing from the product.

Algorithm 1 works on the lattice throughout: P = X * G_xi once; then per
iteration Q = W * G_omega with the codebook as an image of M impulses, the
entropies V(X;W) and V(W) as sums over the lattice of P Q and Q^2, and eq. (6)
for every codevector with the Gaussian G_omega(x - w_k) replaced by a discrete
mask F over a neighbourhood N of w_k (Section 3.1).

Readings (each listed with the design notes):
* codevectors are lattice points, as the paper places them ("on a discrete
  grid"): the continuous value eq. (6) produces is rounded to the nearest
  lattice point (halves upward) and clamped into the H x W lattice;
* F and the masks of P and Q are the sampled unnormalised Gaussians
  g(t) = exp(-t^2/(2 s^2)) on |du|, |dv| <= R, R = ceil(3 s) by default;
  the normalisations of p and q cancel in eq. (6) and in D;
* c = V(X;W) / V(W) from the same lattice sums; D = log V(W) + log V(X)
  - 2 log V(X;W) with V(X) = sum P^2;
* several codevectors on one pixel add their impulses; a codevector whose
  data sum sum_N P F is 0 keeps its place; updates are Jacobi;
* widths are the caller's; the paper's experiments use omega = sqrt(N/M)/2
  and xi = omega/2 (``paper_widths``).
"""
from __future__ import annotations

import math

import numpy as np

from .itc_oracle import density_map, taps

__all__ = ["paper_widths", "literal_q", "literal_terms", "literal_step", "literal_divergence", "fit_literal",
           "fit_literal_density"]


def paper_widths(N: float, M: int):
    """(xi, omega) of the paper's runtime experiments: omega = sqrt(N/M)/2, xi = omega/2."""
    omega = math.sqrt(N / M) / 2.0
    return omega / 2.0, omega


def _window(H, W, w, R):
    """Lattice rows/columns of the window |x - w| <= R around the lattice point w, clipped."""
    u, v = int(w[0]), int(w[1])
    u0, u1 = max(u - R, 0), min(u + R, H - 1)
    v0, v1 = max(v - R, 0), min(v + R, W - 1)
    return u0, u1, v0, v1


def literal_q(shape, Wc, omega, R):
    """Q = W * G_omega: the mask g x g placed at every codevector (an impulse each), on the lattice."""
    H, W = shape
    g = taps(omega, R)
    Q = np.zeros((H, W))
    for w in Wc:
        u0, u1, v0, v1 = _window(H, W, w, R)
        u, v = int(w[0]), int(w[1])
        if u0 > u1 or v0 > v1:
            continue
        Q[u0:u1 + 1, v0:v1 + 1] += np.outer(g[u0 - u + R:u1 - u + R + 1], g[v0 - v + R:v1 - v + R + 1])
    return Q


def literal_terms(P, Q, Wc, omega, R):
    """Per codevector the four window sums of eq. (6):
    a_k = sum P F, b_k = sum P F x, e_k = sum Q F, d_k = sum Q F x over N(w_k)."""
    H, W = P.shape
    g = taps(omega, R)
    M = len(Wc)
    a = np.zeros(M); b = np.zeros((M, 2)); e = np.zeros(M); d = np.zeros((M, 2))
    for k, w in enumerate(Wc):
        u0, u1, v0, v1 = _window(H, W, w, R)
        if u0 > u1 or v0 > v1:
            continue
        u, v = int(w[0]), int(w[1])
        F = np.outer(g[u0 - u + R:u1 - u + R + 1], g[v0 - v + R:v1 - v + R + 1])
        U, V = np.meshgrid(np.arange(u0, u1 + 1, dtype=np.float64), np.arange(v0, v1 + 1, dtype=np.float64),
                           indexing="ij")
        Pw, Qw = P[u0:u1 + 1, v0:v1 + 1], Q[u0:u1 + 1, v0:v1 + 1]
        a[k] = np.sum(Pw * F)
        b[k] = (np.sum(Pw * F * U), np.sum(Pw * F * V))
        e[k] = np.sum(Qw * F)
        d[k] = (np.sum(Qw * F * U), np.sum(Qw * F * V))
    return a, b, e, d


def literal_step(P, Wc, omega, R):
    """One sweep of eq. (6) from the lattice codebook Wc.

    Returns (unrounded w^new [M, 2], c, V(X;W), V(W)); a codevector with
    a_k = 0 keeps its place."""
    Wc = np.asarray(Wc, np.float64)
    Q = literal_q(P.shape, Wc, omega, R)
    v_xw = float(np.sum(P * Q))
    v_w = float(np.sum(Q * Q))
    c = v_xw / v_w
    a, b, e, d = literal_terms(P, Q, Wc, omega, R)
    out = Wc.copy()
    ok = a > 0
    out[ok] = (b[ok] - c * d[ok] + c * e[ok, None] * Wc[ok]) / a[ok, None]
    return out, c, v_xw, v_w


def literal_divergence(P, Wc, omega, R, v_x=None):
    """D of eq. (1) with the lattice sums of Algorithm 1."""
    Q = literal_q(P.shape, Wc, omega, R)
    if v_x is None:
        v_x = float(np.sum(P * P))
    return -2.0 * math.log(float(np.sum(P * Q))) + math.log(float(np.sum(Q * Q))) + math.log(v_x)


def _to_lattice(w, shape):
    H, W = shape
    r = np.floor(w + 0.5)
    r[:, 0] = np.clip(r[:, 0], 0, H - 1)
    r[:, 1] = np.clip(r[:, 1], 0, W - 1)
    return r


def fit_literal(I, W0, xi, omega, iters, R_xi=None, R_omega=None, theta=None):
    """Algorithm 1: returns (lattice codebook, D trace over W_0..W_T, sweeps done, P).

    W0 must hold lattice points. Stops early when max_k ||w_k^new - w_k|| <= theta."""
    I = np.asarray(I, np.float64)
    R_xi = int(math.ceil(3.0 * xi - 1e-12)) if R_xi is None else int(R_xi)
    P = density_map(I, xi, R_xi)
    return fit_literal_density(P, W0, omega, iters, R_omega, theta)


def fit_literal_density(P, W0, omega, iters, R_omega=None, theta=None):
    """Algorithm 1's loop from a given density P (computed once, by the masks or by the recursive
    filter of Section 3.1): returns (lattice codebook, D trace over W_0..W_T, sweeps done, P)."""
    P = np.asarray(P, np.float64)
    R_om = int(math.ceil(3.0 * omega - 1e-12)) if R_omega is None else int(R_omega)
    v_x = float(np.sum(P * P))
    Wc = np.array(W0, dtype=np.float64)
    if not np.array_equal(Wc, np.floor(Wc)):
        raise ValueError("Algorithm 1 starts from lattice points")
    trace = [literal_divergence(P, Wc, omega, R_om, v_x)]
    done = 0
    for _ in range(iters):
        wn, _, _, _ = literal_step(P, Wc, omega, R_om)
        wn = _to_lattice(wn, P.shape)
        step = float(np.max(np.linalg.norm(wn - Wc, axis=1)))
        Wc = wn
        done += 1
        trace.append(literal_divergence(P, Wc, omega, R_om, v_x))
        if theta is not None and theta >= 0 and step <= theta:
            break
    return Wc, np.array(trace), done, P
