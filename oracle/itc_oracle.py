"""Plain FP64 CPU oracle for information theoretic clustering (ITC) on lattices.

TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module. The product path (the HIP
library and its Python binding) never calls it, and this module imports
nothing from the product: the two share no code.

What it computes (Bauckhage & Kersting, "Efficient Information Theoretic
Clustering on Discrete Lattices"):

* the original ITC iteration over a weighted point set (Section 2, the
  Cauchy-Schwarz divergence eq. (1), the Parzen estimates eqs. (2)-(3), the
  overlap integrals of Section 2.1 and the fixed-point update eq. (4));
* the lattice variant (Section 3): the data terms of the same update are read
  from the Gaussian convolutions of the weight image I and of its
  coordinate-weighted copies u*I and v*I (Section 3.1, with per-pixel weights
  as in Section 5), truncated to a square window of radius R;
* the divergence of both variants and its analytic gradient with respect to
  the codevectors and the per-pixel weights.

Readings of the paper this oracle takes (each is listed in the design notes):

* one kernel width: xi = omega = sigma/sqrt(2), so that tau = rho = sigma and
  the data, codebook and data-data overlaps all use G_sigma. The printed
  constant c = (N/M) V(X;W) / V(W) of eq. (4) is then the exact stationarity
  condition of eq. (1);
* weighted data: p(x) = (1/N) sum_i h_i G_xi(x - x_i) with N = sum_i h_i
  (Section 5 with the density normalised); binary images have h = 1;
* lattice maps use the unnormalised sampled Gaussian g(t) = exp(-t^2/(2 s^2)):
  the Parzen normalisations cancel in every ratio of eq. (4) and in eq. (1);
* the window is |du|, |dv| <= R with R = ceil(3 sigma); the image is zero
  outside its H x W domain; maps are evaluated on that domain;
* codevectors are continuous; maps are read at them by bilinear interpolation
  (out-of-domain corners contribute 0); ``read='nearest'`` is available;
* Jacobi order: every w_k^new is computed from the previous codebook;
* a codevector whose data mass is exactly 0 keeps its position;
* lattice coordinates: u is the row, v the column, 0-based, pixel centres at
  integers; codebooks are (M, 2) arrays of (u, v).

Every function is pinned by tests against closed forms, brute force on tiny
inputs, finite differences and invariants; none is "parity unpinned".
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "parzen_gauss", "widths", "overlap_xw", "overlap_w", "overlap_x", "cs_divergence",
    "original_terms", "original_step", "original_divergence", "original_grad_w",
    "original_grad_h", "fit_original",
    "taps", "correlate_axis", "lattice_maps", "density_map", "lattice_maps_window", "moment_maps",
    "read_bilinear", "read_nearest", "read_bilinear_grad", "codebook_terms",
    "lattice_step", "lattice_divergence", "lattice_grad", "fit_lattice",
]


# ---------------------------------------------------------------------------
# Section 2: Parzen densities, overlap integrals, Cauchy-Schwarz divergence
# ---------------------------------------------------------------------------

def parzen_gauss(d: np.ndarray, s: float) -> np.ndarray:
    """Normalised isotropic 2-D Gaussian G_s evaluated at displacements d (..., 2)."""
    d2 = np.sum(np.asarray(d, dtype=np.float64) ** 2, axis=-1)
    return np.exp(-d2 / (2.0 * s * s)) / (2.0 * math.pi * s * s)


def widths(sigma: float):
    """Single-width reading: xi = omega = sigma/sqrt(2) -> (xi, omega)."""
    return sigma / math.sqrt(2.0), sigma / math.sqrt(2.0)


def _pairwise(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Displacements b_j - a_i, shape (len(a), len(b), 2)."""
    return b[None, :, :] - a[:, None, :]


def overlap_xw(X, h, W, xi, omega, truncate=None):
    """V(X;W) = int p q dx = (1/(MN)) sum_i sum_j h_i G_tau(x_i - w_j), tau^2 = xi^2 + omega^2.

    Gaussian product theorem, Section 2.1. ``truncate=R`` keeps only pairs with
    |du|, |dv| <= R (the lattice variant's finite mask).
    """
    X = np.asarray(X, np.float64); W = np.asarray(W, np.float64); h = np.asarray(h, np.float64)
    tau = math.sqrt(xi * xi + omega * omega)
    N, M = h.sum(), W.shape[0]
    tot = 0.0
    for s in range(0, X.shape[0], 4096):
        d = _pairwise(X[s:s + 4096], W)
        G = parzen_gauss(d, tau)
        if truncate is not None:
            G = G * (np.abs(d).max(axis=-1) <= truncate)
        tot += float(np.sum(h[s:s + 4096, None] * G))
    return tot / (M * N)


def overlap_w(W, omega):
    """V(W) = int q^2 dx = (1/M^2) sum_i sum_j G_rho(w_i - w_j), rho^2 = 2 omega^2 (Section 2.1)."""
    W = np.asarray(W, np.float64)
    rho = math.sqrt(2.0) * omega
    return float(np.sum(parzen_gauss(_pairwise(W, W), rho))) / W.shape[0] ** 2


def overlap_x(X, h, xi):
    """V(X) = int p^2 dx = (1/N^2) sum_i sum_j h_i h_j G_{sqrt2 xi}(x_i - x_j)."""
    X = np.asarray(X, np.float64); h = np.asarray(h, np.float64)
    s = math.sqrt(2.0) * xi
    tot = 0.0
    for a in range(0, X.shape[0], 2048):
        G = parzen_gauss(_pairwise(X[a:a + 2048], X), s)
        tot += float(h[a:a + 2048] @ G @ h)
    return tot / h.sum() ** 2


def cs_divergence(v_xw: float, v_w: float, v_x: float) -> float:
    """Eq. (1): D = 2 H(X;W) - H(W) - H(X) with Renyi entropies H = -log V."""
    return -2.0 * math.log(v_xw) + math.log(v_w) + math.log(v_x)


# ---------------------------------------------------------------------------
# Section 2: the original fixed-point iteration, eq. (4)
# ---------------------------------------------------------------------------

def original_terms(X, h, W, xi, omega, truncate=None):
    """Per-codevector sums of eq. (4) over all data points.

    Returns (den, num, GW, Gsum):
      den_k  = sum_j h_j G_tau(x_j - w_k)
      num_k  = sum_j h_j G_tau(x_j - w_k) x_j
      GW_k   = sum_j G_rho(w_j - w_k) w_j
      Gsum_k = sum_j G_rho(w_j - w_k)
    """
    X = np.asarray(X, np.float64); W = np.asarray(W, np.float64); h = np.asarray(h, np.float64)
    tau = math.sqrt(xi * xi + omega * omega)
    rho = math.sqrt(2.0) * omega
    M = W.shape[0]
    den = np.zeros(M); num = np.zeros((M, 2))
    for s in range(0, X.shape[0], 4096):
        Xs = X[s:s + 4096]
        d = _pairwise(W, Xs)                     # (M, n, 2): x_j - w_k
        G = parzen_gauss(d, tau) * h[None, s:s + 4096]
        if truncate is not None:
            G = G * (np.abs(d).max(axis=-1) <= truncate)
        den += G.sum(axis=1)
        num += G @ Xs
    Gww = parzen_gauss(_pairwise(W, W), rho)     # (M, M): G_rho(w_j - w_k), row k
    return den, num, Gww @ W, Gww.sum(axis=1)


def original_step(X, h, W, xi, omega, truncate=None):
    """One Jacobi sweep of eq. (4) with c = (N/M) V(X;W) / V(W).

    A codevector with den_k == 0 (no data under its window) keeps its place.
    """
    W = np.asarray(W, np.float64)
    N, M = float(np.sum(h)), W.shape[0]
    den, num, GW, Gsum = original_terms(X, h, W, xi, omega, truncate)
    c = (N / M) * overlap_xw(X, h, W, xi, omega, truncate) / overlap_w(W, omega)
    out = W.copy()
    ok = den > 0
    out[ok] = (num[ok] - c * GW[ok] + c * Gsum[ok, None] * W[ok]) / den[ok, None]
    return out


def original_divergence(X, h, W, xi, omega, truncate=None, v_x=None):
    """Eq. (1) for the point-set densities; V(X) is always untruncated.

    ``v_x`` may carry a precomputed V(X) (it does not depend on the codebook).
    """
    if v_x is None:
        v_x = overlap_x(X, h, xi)
    return cs_divergence(overlap_xw(X, h, W, xi, omega, truncate), overlap_w(W, omega), v_x)


def original_grad_w(X, h, W, sigma):
    """dD/dw_k of eq. (1) in the single-width reading (tau = rho = sigma).

    V(X;W) and V(W) differentiate through the Gaussians:
      d/dw_k sum_j h_j G(x_j - w_k) = sum_j h_j G(x_j - w_k) (x_j - w_k) / sigma^2
      d/dw_k sum_i sum_j G(w_i - w_j) = 2 sum_j G(w_j - w_k) (w_j - w_k) / sigma^2
    so dD/dw_k = -2 (dV_xw/dw_k)/V_xw + (dV_w/dw_k)/V_w.
    """
    xi, om = widths(sigma)
    W = np.asarray(W, np.float64)
    den, num, GW, Gsum = original_terms(X, h, W, xi, om)
    s_xw, s_w = den.sum(), Gsum.sum()
    dxw = (num - den[:, None] * W) / sigma ** 2
    dw = 2.0 * (GW - Gsum[:, None] * W) / sigma ** 2
    return -2.0 * dxw / s_xw + dw / s_w


def original_grad_h(X, h, W, sigma):
    """dD/dh_i (per-point weight) of eq. (1), single width, untruncated.

    V(X;W) is linear in h and V(X) quadratic; N = sum h cancels in D.
    """
    X = np.asarray(X, np.float64); W = np.asarray(W, np.float64); h = np.asarray(h, np.float64)
    Gxw = parzen_gauss(_pairwise(X, W), sigma).sum(axis=1)          # sum_k G(w_k - x_i)
    Gxx = np.zeros(X.shape[0])
    for a in range(0, X.shape[0], 2048):
        Gxx[a:a + 2048] = parzen_gauss(_pairwise(X[a:a + 2048], X), sigma) @ h
    s_xw = float(h @ Gxw)
    s_x = float(h @ Gxx)
    return -2.0 * Gxw / s_xw + 2.0 * Gxx / s_x


def fit_original(X, h, W0, sigma, iters, truncate=None, theta=None, xi=None, omega=None):
    """Iterate eq. (4); returns (W, D trace over W_0..W_T, iterations done).

    Stops early when max_k ||w_k^new - w_k|| <= theta (Algorithm 1's second
    stopping test with the Euclidean norm per codevector and max over k).
    """
    if xi is None or omega is None:
        xi, omega = widths(sigma)
    W = np.array(W0, dtype=np.float64)
    v_x = overlap_x(X, h, xi)
    trace = [original_divergence(X, h, W, xi, omega, truncate, v_x)]
    done = 0
    for _ in range(iters):
        Wn = original_step(X, h, W, xi, omega, truncate)
        step = float(np.max(np.linalg.norm(Wn - W, axis=1))) if W.size else 0.0
        W = Wn
        done += 1
        trace.append(original_divergence(X, h, W, xi, omega, truncate, v_x))
        if theta is not None and theta >= 0 and step <= theta:
            break
    return W, np.array(trace), done


# ---------------------------------------------------------------------------
# Section 3.1 (+ Section 5 weights): convolution maps on the lattice
# ---------------------------------------------------------------------------

def taps(sigma: float, R: int) -> np.ndarray:
    """Sampled unnormalised Gaussian g[t] = exp(-t^2 / (2 sigma^2)), t = -R..R."""
    t = np.arange(-R, R + 1, dtype=np.float64)
    return np.exp(-t * t / (2.0 * sigma * sigma))


def correlate_axis(f: np.ndarray, k: np.ndarray, axis: int) -> np.ndarray:
    """out[x] = sum_{t=-R}^{R} k[t] f[x - t] along ``axis``; f is zero off the domain."""
    R = (k.shape[0] - 1) // 2
    f = np.moveaxis(np.asarray(f, np.float64), axis, 0)
    n = f.shape[0]
    fp = np.zeros((n + 2 * R,) + f.shape[1:])
    fp[R:R + n] = f
    out = np.zeros_like(f)
    for i, t in enumerate(range(-R, R + 1)):
        out += k[i] * fp[R - t:R - t + n]
    return np.moveaxis(out, 0, axis)


def _coords(shape):
    H, W = shape
    return (np.arange(H, dtype=np.float64)[:, None] * np.ones((1, W)),
            np.ones((H, 1)) * np.arange(W, dtype=np.float64)[None, :])


def lattice_maps(I: np.ndarray, sigma: float, R: int):
    """Gaussian convolutions of I, u*I and v*I on the H x W lattice.

    A(x)   = sum_y I(y)       g(x - y)
    B_u(x) = sum_y I(y) y_u   g(x - y)
    B_v(x) = sum_y I(y) y_v   g(x - y)
    with the window |x_u - y_u|, |x_v - y_v| <= R. The 2-D Gaussian factorises,
    so each map is a correlation along v followed by one along u (Section 3.1:
    separable 1-D masks for small kernel width).
    """
    I = np.asarray(I, np.float64)
    g = taps(sigma, R)
    U, V = _coords(I.shape)
    out = []
    for f in (I, U * I, V * I):
        out.append(correlate_axis(correlate_axis(f, g, 1), g, 0))
    return tuple(out)


def density_map(I: np.ndarray, sigma: float, R: int) -> np.ndarray:
    """A(x) = sum_y I(y) g(x - y) alone (the P = X * G density of Algorithm 1)."""
    g = taps(sigma, R)
    return correlate_axis(correlate_axis(np.asarray(I, np.float64), g, 1), g, 0)


def lattice_maps_window(I: np.ndarray, sigma: float, R: int):
    """The same three maps as a direct 2-D window sum over all (du, dv) offsets."""
    I = np.asarray(I, np.float64)
    H, W = I.shape
    U, V = _coords(I.shape)
    src = [I, U * I, V * I]
    pad = [np.zeros((H + 2 * R, W + 2 * R)) for _ in src]
    for p, s in zip(pad, src):
        p[R:R + H, R:R + W] = s
    out = [np.zeros((H, W)) for _ in src]
    for du in range(-R, R + 1):
        for dv in range(-R, R + 1):
            gw = math.exp(-(du * du + dv * dv) / (2.0 * sigma * sigma))
            for o, p in zip(out, pad):
                o += gw * p[R - du:R - du + H, R - dv:R - dv + W]
    return tuple(out)


def moment_maps(A, Bu, Bv):
    """Pixel-centred moments M_u(x) = x_u A(x) - B_u(x), M_v(x) = x_v A(x) - B_v(x).

    Equivalently M(x) = sum_y I(y) (x - y) g(x - y).
    """
    U, V = _coords(A.shape)
    return U * A - Bu, V * A - Bv


# ---------------------------------------------------------------------------
# reading maps at continuous codevector positions
# ---------------------------------------------------------------------------

def _corners(F: np.ndarray, w: np.ndarray):
    """Yield (weight_u, weight_v, value) of the 4 bilinear corners of each w; off-domain -> 0."""
    H, W = F.shape
    u, v = w[:, 0], w[:, 1]
    i0, j0 = np.floor(u), np.floor(v)
    fu, fv = u - i0, v - j0
    for di, wu in ((0, 1.0 - fu), (1, fu)):
        for dj, wv in ((0, 1.0 - fv), (1, fv)):
            ii, jj = (i0 + di).astype(np.int64), (j0 + dj).astype(np.int64)
            ok = (ii >= 0) & (ii < H) & (jj >= 0) & (jj < W)
            val = np.zeros(w.shape[0])
            val[ok] = F[ii[ok], jj[ok]]
            yield di, dj, wu, wv, fu, fv, val


def read_bilinear(F: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Bilinear interpolation of lattice map F at points w (M, 2)."""
    w = np.asarray(w, np.float64)
    out = np.zeros(w.shape[0])
    for _, _, wu, wv, _, _, val in _corners(F, w):
        out += wu * wv * val
    return out


def read_bilinear_grad(F: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Gradient (d/du, d/dv) of the bilinear interpolant of F at w (M, 2)."""
    w = np.asarray(w, np.float64)
    out = np.zeros((w.shape[0], 2))
    for di, dj, wu, wv, fu, fv, val in _corners(F, w):
        su = 1.0 if di else -1.0      # d(weight_u)/du
        sv = 1.0 if dj else -1.0
        out[:, 0] += su * wv * val
        out[:, 1] += wu * sv * val
    return out


def read_nearest(F: np.ndarray, w: np.ndarray) -> np.ndarray:
    """Value of F at the lattice point nearest to each w (ties round half to even)."""
    w = np.asarray(w, np.float64)
    H, W = F.shape
    i, j = np.rint(w[:, 0]).astype(np.int64), np.rint(w[:, 1]).astype(np.int64)
    ok = (i >= 0) & (i < H) & (j >= 0) & (j < W)
    out = np.zeros(w.shape[0])
    out[ok] = F[i[ok], j[ok]]
    return out


def codebook_terms(W: np.ndarray, sigma: float):
    """Codebook sums with the unnormalised kernel, full M x M (no truncation).

    Returns (C, GW): C_k = sum_j g(w_j - w_k), GW_k = sum_j g(w_j - w_k) w_j.
    """
    W = np.asarray(W, np.float64)
    d = _pairwise(W, W)
    G = np.exp(-np.sum(d * d, axis=-1) / (2.0 * sigma * sigma))
    return G.sum(axis=1), G @ W


# ---------------------------------------------------------------------------
# Section 3: the lattice form of the update and the divergence
# ---------------------------------------------------------------------------

def _reads(maps, W, read):
    A, Bu, Bv = maps
    f = read_bilinear if read == "bilinear" else read_nearest
    return f(A, W), np.stack([f(Bu, W), f(Bv, W)], axis=1)


def lattice_step(maps, W, sigma, read="bilinear"):
    """Eq. (4) with its data sums read from the maps at each codevector.

    den_k = A(w_k), num_k = (B_u(w_k), B_v(w_k)); the codebook sums are direct.
    c = (N/M) V(X;W)/V(W) reduces to sum_k A(w_k) / sum_k sum_j g(w_j - w_k) once
    the common Parzen normalisation is cancelled.
    """
    W = np.asarray(W, np.float64)
    den, num = _reads(maps, W, read)
    C, GW = codebook_terms(W, sigma)
    c = den.sum() / C.sum()
    out = W.copy()
    ok = den != 0
    out[ok] = (num[ok] - c * GW[ok] + c * C[ok, None] * W[ok]) / den[ok, None]
    return out


def lattice_divergence(I, maps, W, sigma, read="bilinear", s_x=None):
    """Eq. (1) with lattice sums: V(X;W) from the map reads, V(X) = sum I A.

    Only the density map A = maps[0] is used. All three overlaps carry the same normalisation 1/(2 pi sigma^2) and the
    same 1/N, 1/M factors as in Section 2.1, written out here.
    """
    I = np.asarray(I, np.float64)
    A = maps[0]
    W = np.asarray(W, np.float64)
    N, M = float(I.sum()), W.shape[0]
    Z = 1.0 / (2.0 * math.pi * sigma * sigma)
    den = (read_bilinear if read == "bilinear" else read_nearest)(A, W)
    C, _ = codebook_terms(W, sigma)
    if s_x is None:
        s_x = float(np.sum(I * A))
    v_xw = Z * den.sum() / (M * N)
    v_w = Z * C.sum() / (M * M)
    v_x = Z * s_x / (N * N)
    return cs_divergence(v_xw, v_w, v_x)


def lattice_grad(I, maps, W, sigma, R):
    """Analytic gradient of lattice_divergence (bilinear reads).

    dD/dw_k = -(2/S_XW) grad A_bil(w_k) + (2/(sigma^2 S_W)) sum_j g(w_j - w_k)(w_j - w_k)
    dD/dI(y) = 2 A(y)/S_X - (2/S_XW) K(y),  K(y) = sum_k sum_c beta_kc g(c - y)
    where beta_kc are the bilinear corner weights of w_k (in-domain corners
    only) and g the truncated window. Raw sums: S_XW = sum_k A_bil(w_k),
    S_W = sum_{j,k} g(w_j - w_k), S_X = sum_x I(x) A(x).
    """
    I = np.asarray(I, np.float64)
    W = np.asarray(W, np.float64)
    A = maps[0]
    H, Wd = A.shape
    s_xw = float(read_bilinear(A, W).sum())
    C, GW = codebook_terms(W, sigma)
    s_w = float(C.sum())
    s_x = float(np.sum(I * A))
    gw = -2.0 / s_xw * read_bilinear_grad(A, W) + 2.0 / (sigma * sigma * s_w) * (GW - C[:, None] * W)
    # splat the bilinear weights, then correlate with the window Gaussian
    Z = np.zeros((H, Wd))
    u, v = W[:, 0], W[:, 1]
    i0, j0 = np.floor(u), np.floor(v)
    fu, fv = u - i0, v - j0
    for di, wu in ((0, 1.0 - fu), (1, fu)):
        for dj, wv in ((0, 1.0 - fv), (1, fv)):
            ii, jj = (i0 + di).astype(np.int64), (j0 + dj).astype(np.int64)
            ok = (ii >= 0) & (ii < H) & (jj >= 0) & (jj < Wd)
            np.add.at(Z, (ii[ok], jj[ok]), (wu * wv)[ok])
    g = taps(sigma, R)
    K = correlate_axis(correlate_axis(Z, g, 1), g, 0)
    gI = 2.0 * A / s_x - 2.0 / s_xw * K
    return gw, gI


def fit_lattice(I, W0, sigma, R, iters, read="bilinear", theta=None, maps=None):
    """Algorithm 1 with the maps computed once and eq. (4) read from them.

    Returns (W, D trace over W_0..W_T, iterations done, maps).
    """
    I = np.asarray(I, np.float64)
    if maps is None:
        maps = lattice_maps(I, sigma, R)
    s_x = float(np.sum(I * maps[0]))
    W = np.array(W0, dtype=np.float64)
    trace = [lattice_divergence(I, maps, W, sigma, read, s_x)]
    done = 0
    for _ in range(iters):
        Wn = lattice_step(maps, W, sigma, read)
        step = float(np.max(np.linalg.norm(Wn - W, axis=1))) if W.size else 0.0
        W = Wn
        done += 1
        trace.append(lattice_divergence(I, maps, W, sigma, read, s_x))
        if theta is not None and theta >= 0 and step <= theta:
            break
    return W, np.array(trace), done, maps
