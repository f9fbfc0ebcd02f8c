"""Pins of the chamfer distance-transform oracle (Section 5 weighting), CPU only.

The oracle runs Borgefors' sequential two-pass propagation. It is checked
against what fixes the result independently of that algorithm:
* the definition: the least path cost to the background, which on an
  unobstructed grid with orthogonal cost a and diagonal cost b (a <= b <= 2a)
  is min over background pixels q of a*max(|du|,|dv|) + (b-a)*min(|du|,|dv|),
  evaluated by brute force (the outside of the lattice is a background ring);
* scipy's chamfer transforms for the taxicab (a=1, b=2) and chessboard
  (a=1, b=1) masks;
* the Euclidean bound of the 3-4 chamfer: along a direction with
  t = min/max in [0, 1] the 3-4 cost over 3 is (1 + t/3) max while the
  Euclidean length is sqrt(1 + t^2) max, so T/3 lies within
  [2 sqrt(2)/3, sqrt(10)/3] = [0.9428, 1.0541] times the Euclidean
  distance transform;
* closed forms (all-foreground image: distance to the border), background
  zeros, and equivariance under transposes and flips.
"""
import numpy as np
import pytest
from scipy import ndimage

import oracle as O
from paper_1310_7114_amd import synth as S


def brute_force(X, a, b):
    H, W = X.shape
    pad = np.zeros((H + 2, W + 2), np.uint8)
    pad[1:-1, 1:-1] = X != 0
    bu, bv = np.nonzero(pad == 0)
    bu = bu - 1
    bv = bv - 1
    out = np.zeros((H, W), np.int64)
    for i in range(H):
        for j in range(W):
            if X[i, j]:
                du = np.abs(bu - i)
                dv = np.abs(bv - j)
                out[i, j] = int(np.min(a * np.maximum(du, dv) + (b - a) * np.minimum(du, dv)))
    return out


def rand_img(seed, H, W, p):
    return (np.random.default_rng(seed).uniform(size=(H, W)) < p).astype(np.uint8)


@pytest.mark.parametrize("a,b", [(3, 4), (1, 1), (1, 2), (5, 7), (2, 3)])
@pytest.mark.parametrize("seed,H,W,p", [(0, 7, 9, 0.8), (1, 12, 5, 0.9), (2, 1, 13, 0.7), (3, 10, 10, 0.95),
                                        (4, 6, 6, 1.0), (5, 8, 11, 0.3)])
def test_matches_definition(a, b, seed, H, W, p):
    X = rand_img(seed, H, W, p)
    assert np.array_equal(O.chamfer_transform(X, a, b), brute_force(X, a, b))


@pytest.mark.parametrize("metric,a,b", [("taxicab", 1, 2), ("chessboard", 1, 1)])
def test_matches_scipy(metric, a, b):
    X = rand_img(7, 40, 53, 0.85)
    pad = np.zeros((42, 55), np.uint8)
    pad[1:-1, 1:-1] = X
    ref = ndimage.distance_transform_cdt(pad, metric=metric)[1:-1, 1:-1]
    assert np.array_equal(O.chamfer_transform(X, a, b), ref)


def test_euclidean_bound():
    X = S.config1_case(1).img
    X2 = np.zeros((90, 90), np.uint8)
    uu, vv = np.mgrid[:90, :90]
    X2[(uu - 44.3) ** 2 + (vv - 45.1) ** 2 <= 40 ** 2] = 1
    for img in (X, X2):
        T = O.chamfer_transform(img, 3, 4) / 3.0
        pad = np.zeros((img.shape[0] + 2, img.shape[1] + 2), np.uint8)
        pad[1:-1, 1:-1] = img
        E = ndimage.distance_transform_edt(pad)[1:-1, 1:-1]
        assert np.all(T >= 2 * np.sqrt(2) / 3 * E - 1e-12)
        assert np.all(T <= np.sqrt(10) / 3 * E + 1e-12)
        if img is X2:  # inside a large disc the ratio approaches the upper bound
            assert (T / np.where(E > 0, E, 1))[E > 20].max() > 1.02


def test_all_foreground_is_distance_to_border():
    H, W = 9, 14
    T = O.chamfer_transform(np.ones((H, W), np.uint8), 3, 4)
    i, j = np.mgrid[:H, :W]
    assert np.array_equal(T, 3 * np.minimum.reduce([i + 1, j + 1, H - i, W - j]))


def test_background_and_boundary():
    X = rand_img(9, 30, 31, 0.7)
    T = O.chamfer_transform(X, 3, 4)
    assert np.all(T[X == 0] == 0)
    assert np.all(T[X != 0] >= 3)
    pad = np.zeros((32, 33), np.uint8)
    pad[1:-1, 1:-1] = X
    touch = np.zeros_like(X, bool)
    for du, dv in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        touch |= pad[1 + du:31 + du, 1 + dv:32 + dv] == 0
    assert np.all(T[(X != 0) & touch] == 3)
    assert np.all(O.chamfer_transform(np.zeros((5, 6), np.uint8)) == 0)


def test_equivariance():
    X = rand_img(11, 23, 17, 0.85)
    T = O.chamfer_transform(X, 3, 4)
    assert np.array_equal(O.chamfer_transform(X.T, 3, 4), T.T)
    assert np.array_equal(O.chamfer_transform(X[::-1], 3, 4), T[::-1])
    assert np.array_equal(O.chamfer_transform(X[:, ::-1], 3, 4), T[:, ::-1])
