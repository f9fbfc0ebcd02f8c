"""Pins of the 3-D lattice oracle (volumes), CPU only: brute-force maps on a tiny
volume, the reduction to the pinned 2-D oracle at depth 1 (maps and the whole
fit), closed forms for an impulse, trilinear reads exact on trilinear
functions, axis-permutation equivariance and the M = 1 mean shift to the
centre of a symmetric ball."""
import math

import numpy as np

import oracle as O
from paper_1310_7114_amd import synth as S


def test_maps_brute_force():
    rng = np.random.default_rng(0)
    I = rng.uniform(size=(5, 6, 7)) * (rng.uniform(size=(5, 6, 7)) < 0.6)
    sigma, R = 1.3, 2
    A, Bs, Bu, Bv = O.volume_maps(I, sigma, R)
    D, H, W = I.shape
    for x in [(0, 0, 0), (2, 3, 4), (4, 5, 6), (1, 0, 6), (3, 2, 1)]:
        a = bs = bu = bv = 0.0
        for s in range(D):
            for u in range(H):
                for v in range(W):
                    if max(abs(x[0] - s), abs(x[1] - u), abs(x[2] - v)) <= R:
                        g = math.exp(-((x[0] - s) ** 2 + (x[1] - u) ** 2 + (x[2] - v) ** 2) / (2 * sigma ** 2))
                        a += I[s, u, v] * g
                        bs += I[s, u, v] * g * s
                        bu += I[s, u, v] * g * u
                        bv += I[s, u, v] * g * v
        assert np.allclose([A[x], Bs[x], Bu[x], Bv[x]], [a, bs, bu, bv], rtol=1e-12, atol=1e-14)


def test_depth_one_is_the_2d_method():
    c = S.config1_case(2)
    maps3 = O.volume_maps(c.weights[None], c.sigma, c.R)
    maps2 = O.lattice_maps(c.weights, c.sigma, c.R)
    assert np.allclose(maps3[0][0], maps2[0], rtol=1e-13, atol=0)
    assert np.all(maps3[1] == 0)
    assert np.allclose(maps3[2][0], maps2[1], rtol=1e-13, atol=0)
    assert np.allclose(maps3[3][0], maps2[2], rtol=1e-13, atol=0)
    W0 = np.concatenate([np.zeros((c.M, 1)), c.w0], axis=1)
    W3, tr3, _, _ = O.fit_volume(c.weights[None], W0, c.sigma, c.R, 20)
    W2, tr2, _, _ = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, 20)
    assert np.all(W3[:, 0] == 0)
    assert np.abs(W3[:, 1:] - W2).max() <= 1e-10
    assert np.allclose(tr3, tr2, rtol=1e-11)


def test_impulse_closed_form():
    I = np.zeros((9, 11, 10))
    I[4, 6, 3] = 2.5
    sigma, R = 1.7, 5
    A, Bs, Bu, Bv = O.volume_maps(I, sigma, R)
    s, u, v = np.meshgrid(np.arange(9.0), np.arange(11.0), np.arange(10.0), indexing="ij")
    d2 = (s - 4) ** 2 + (u - 6) ** 2 + (v - 3) ** 2
    inwin = (np.abs(s - 4) <= R) & (np.abs(u - 6) <= R) & (np.abs(v - 3) <= R)
    ref = 2.5 * np.exp(-d2 / (2 * sigma ** 2)) * inwin
    assert np.allclose(A, ref, rtol=1e-13, atol=1e-15)
    assert np.allclose(Bs, 4 * ref) and np.allclose(Bu, 6 * ref) and np.allclose(Bv, 3 * ref)


def test_trilinear_exact_and_off_lattice():
    s, u, v = np.meshgrid(np.arange(4.0), np.arange(5.0), np.arange(6.0), indexing="ij")
    F = 1.5 + 0.3 * s - 0.7 * u + 0.2 * v + 0.05 * s * u - 0.11 * u * v + 0.02 * s * v * u
    w = np.array([[0.3, 1.7, 2.2], [2.9, 3.1, 4.99], [1.0, 2.0, 3.0]])
    ref = 1.5 + 0.3 * w[:, 0] - 0.7 * w[:, 1] + 0.2 * w[:, 2] + 0.05 * w[:, 0] * w[:, 1] \
        - 0.11 * w[:, 1] * w[:, 2] + 0.02 * w[:, 0] * w[:, 2] * w[:, 1]
    assert np.allclose(O.read_trilinear(F, w), ref, rtol=1e-13)
    # a point half a voxel outside the first slice keeps half of the inside corners' weight
    assert np.isclose(O.read_trilinear(np.ones((4, 5, 6)), np.array([[-0.5, 2.0, 2.0]]))[0], 0.5)


def test_axis_permutation():
    c = S.volume_case(1, D=30, H=36, W=40, M=10, iters=10)
    W, tr, _, _ = O.fit_volume(c.weights, c.w0, c.sigma, c.R, 10)
    perm = (2, 0, 1)
    Wp, trp, _, _ = O.fit_volume(np.transpose(c.weights, perm), c.w0[:, list(perm)], c.sigma, c.R, 10)
    assert np.abs(Wp - W[:, list(perm)]).max() <= 1e-10
    assert np.allclose(trp, tr, rtol=1e-11)


def test_single_codevector_finds_the_ball_centre():
    s, u, v = np.meshgrid(np.arange(25.0), np.arange(25.0), np.arange(25.0), indexing="ij")
    I = (((s - 12) ** 2 + (u - 12) ** 2 + (v - 12) ** 2) <= 36).astype(float)
    W, tr, _, _ = O.fit_volume(I, np.array([[10.0, 14.0, 11.0]]), 2.0, 6, 200)
    assert np.abs(W[0] - 12.0).max() <= 1e-6
    assert np.all(np.diff(tr) <= 1e-12)
