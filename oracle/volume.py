"""Lattice ITC on 3-D lattices (volumes): the maps of Section 3.1 with a third
separable pass and the update eq. (4) in three dimensions.

TEST INFRASTRUCTURE ONLY, like the rest of this package: only the test suite,
the smoke check and the benchmark's CPU-baseline leg may import it, and it
imports nothing from the product.

The paper develops the method on 2-D lattices and states that it carries over
to higher-dimensional lattices; this module is that carry-over, in the same
readings as the 2-D oracle: one width sigma, unnormalised sampled Gaussian
taps g(t), a cubic window |d_axis| <= R, weights zero outside the D x H x W
lattice, coordinates x = (s, u, v) with s the slice, u the row, v the column
(0-based, voxel centres at integers), trilinear reads (corners off the lattice
contribute 0), Jacobi sweeps, a codevector with A_k = 0 kept in place.
Maps: A(x) = sum_y h(y) g(x - y) and B_a(x) = sum_y h(y) y_a g(x - y) for
each axis a; the update is w_k <- (B_k - c (GW_k - C_k w_k)) / A_k with
C_k = sum_j G(w_j - w_k), GW_k = sum_j G(w_j - w_k) w_j, c = S_XW / S_W.
"""
from __future__ import annotations

import math

import numpy as np

from .itc_oracle import correlate_axis, taps

__all__ = ["volume_maps", "read_trilinear", "volume_codebook_terms", "volume_step", "volume_divergence",
           "fit_volume"]


def volume_maps(I: np.ndarray, sigma: float, R: int):
    """(A, B_s, B_u, B_v): the Gaussian convolutions of I and of s*I, u*I, v*I on the
    lattice, each a correlation along v, then u, then s (the 3-D mask factorises)."""
    I = np.asarray(I, np.float64)
    g = taps(sigma, R)
    S, U, V = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in I.shape], indexing="ij")
    out = []
    for f in (I, S * I, U * I, V * I):
        out.append(correlate_axis(correlate_axis(correlate_axis(f, g, 2), g, 1), g, 0))
    return tuple(out)


def read_trilinear(F: np.ndarray, w: np.ndarray) -> np.ndarray:
    """F at continuous points w (M, 3): trilinear weights over the 8 lattice corners; corners
    off the lattice contribute 0."""
    w = np.asarray(w, np.float64)
    D, H, W = F.shape
    f = np.floor(w)
    fr = w - f
    out = np.zeros(len(w))
    for ds in (0, 1):
        for du in (0, 1):
            for dv in (0, 1):
                c = f + np.array([ds, du, dv])
                b = (np.where(ds, fr[:, 0], 1 - fr[:, 0]) * np.where(du, fr[:, 1], 1 - fr[:, 1])
                     * np.where(dv, fr[:, 2], 1 - fr[:, 2]))
                ok = (c[:, 0] >= 0) & (c[:, 0] < D) & (c[:, 1] >= 0) & (c[:, 1] < H) & (c[:, 2] >= 0) & (c[:, 2] < W)
                ci = c.astype(np.int64)
                val = np.zeros(len(w))
                val[ok] = F[ci[ok, 0], ci[ok, 1], ci[ok, 2]]
                out += b * val
    return out


def volume_codebook_terms(W: np.ndarray, sigma: float):
    """C_k = sum_j G(w_j - w_k) and GW_k = sum_j G(w_j - w_k) w_j, all j (untruncated)."""
    W = np.asarray(W, np.float64)
    d = W[None, :, :] - W[:, None, :]
    G = np.exp(-np.sum(d * d, axis=-1) / (2.0 * sigma * sigma))
    return G.sum(axis=1), G @ W


def volume_step(maps, W, sigma):
    """One Jacobi sweep of eq. (4) with the data sums read from the volume maps."""
    W = np.asarray(W, np.float64)
    A, Bs, Bu, Bv = maps
    den = read_trilinear(A, W)
    num = np.stack([read_trilinear(Bs, W), read_trilinear(Bu, W), read_trilinear(Bv, W)], axis=1)
    C, GW = volume_codebook_terms(W, sigma)
    c = den.sum() / C.sum()
    out = W.copy()
    ok = den != 0
    out[ok] = (num[ok] - c * GW[ok] + c * C[ok, None] * W[ok]) / den[ok, None]
    return out


def volume_divergence(I, maps, W, sigma, s_x=None):
    """D = log S_W + log S_X - 2 log S_XW with S_X = sum h A, S_XW = sum_k A(w_k), S_W = sum_k C_k."""
    if s_x is None:
        s_x = float(np.sum(np.asarray(I, np.float64) * maps[0]))
    s_xw = float(read_trilinear(maps[0], W).sum())
    s_w = float(volume_codebook_terms(W, sigma)[0].sum())
    return math.log(s_w) + math.log(s_x) - 2.0 * math.log(s_xw)


def fit_volume(I, W0, sigma, R, iters, theta=None):
    """Returns (W, D trace over W_0..W_T, sweeps done, maps)."""
    I = np.asarray(I, np.float64)
    maps = volume_maps(I, sigma, R)
    s_x = float(np.sum(I * maps[0]))
    W = np.array(W0, np.float64)
    trace = [volume_divergence(I, maps, W, sigma, s_x)]
    done = 0
    for _ in range(iters):
        Wn = volume_step(maps, W, sigma)
        step = float(np.max(np.linalg.norm(Wn - W, axis=1)))
        W = Wn
        done += 1
        trace.append(volume_divergence(I, maps, W, sigma, s_x))
        if theta is not None and theta >= 0 and step <= theta:
            break
    return W, np.array(trace), done, maps
