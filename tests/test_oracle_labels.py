"""Pins of the labelling oracle (nearest codevector per foreground pixel), CPU only:
a pure-Python brute force over pixels and codevectors, scipy's k-d tree query
(an independent nearest-neighbour search), exact ties, and closed forms."""
import numpy as np
from scipy.spatial import cKDTree

import oracle as O
from paper_1310_7114_amd import synth as S


def brute(I, W):
    H, Wd = I.shape
    out = np.full((H, Wd), -1, np.int32)
    for u in range(H):
        for v in range(Wd):
            if I[u, v] > 0:
                best, bk = None, -1
                for k, w in enumerate(W):
                    d = (u - w[0]) ** 2 + (v - w[1]) ** 2
                    if best is None or d < best:
                        best, bk = d, k
                out[u, v] = bk
    return out


def test_brute_force_small():
    rng = np.random.default_rng(0)
    I = (rng.uniform(size=(13, 17)) < 0.6).astype(np.uint8)
    W = rng.uniform(-2, 18, size=(7, 2)).astype(np.float32).astype(np.float64)
    assert np.array_equal(O.label_pixels(I, W), brute(I, W))


def test_kdtree_on_a_silhouette():
    c = S.config3_cases(indices=[3])[0]
    W = c.w0 + np.random.default_rng(1).uniform(-0.5, 0.5, c.w0.shape)
    L = O.label_pixels(c.img, W)
    us, vs = np.nonzero(c.img > 0)
    _, k = cKDTree(W).query(np.stack([us, vs], 1).astype(np.float64))
    # the tree may break exact ties either way: compare distances, not indices
    d_or = np.hypot(us - W[L[us, vs], 0], vs - W[L[us, vs], 1])
    d_kd = np.hypot(us - W[k, 0], vs - W[k, 1])
    assert np.allclose(d_or, d_kd, rtol=0, atol=1e-12)
    assert np.all(L[c.img == 0] == -1)


def test_ties_go_to_the_smaller_index():
    I = np.ones((5, 5), np.uint8)
    W = np.array([[2.0, 4.0], [2.0, 0.0], [2.0, 0.0]])  # duplicate codevector 2 never wins
    L = O.label_pixels(I, W)
    assert not np.any(L == 2)
    assert np.all(L[:, 2] == 0)          # column 2 is equidistant from both: index 0
    assert np.all(L[:, :2] == 1) and np.all(L[:, 3:] == 0)


def test_single_codevector_and_background():
    I = np.zeros((6, 9), np.uint8)
    I[2:4, 3:7] = 7
    L = O.label_pixels(I, np.array([[100.0, -50.0]]))
    assert np.all(L[I > 0] == 0) and np.all(L[I == 0] == -1)
