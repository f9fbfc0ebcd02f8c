"""Pins of the Algorithm 1 oracle (eq. (6) on the lattice), CPU only.

The strongest pin is the Gaussian product theorem (Section 2.1): with masks
wide enough that truncation is negligible and the data far from the lattice
border, the lattice sums of eq. (6) are exact integrals (the lattice sum of a
Gaussian of width s >= 1 equals its integral to about exp(-2 pi^2 s^2)), and
the update becomes a closed form in the original point-set terms of eq. (4):
  w+ = (omega^2/tau^2) num/den + (xi^2/tau^2) w - (c_o/2)(GW - Gsum w)/den,
with den, num = sum_j h_j G_tau(x_j - w)(1, x_j), GW, Gsum = sum_j G_rho(w_j - w)(w_j, 1)
and c_o = (N/M) V(X;W)/V(W) of eq. (4). That is computed here by the
independent point-set code of the oracle. Further pins: the M = N fixed point,
brute-force Q and window sums on tiny inputs, D >= 0, equivariance, and the
lattice/clamping and theta behaviour of the fit.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_1310_7114_amd import synth as S


def point_set(shape, rng, n, margin):
    H, W = shape
    X = np.stack([rng.integers(margin, H - margin, n), rng.integers(margin, W - margin, n)], 1).astype(np.float64)
    X = np.unique(X, axis=0)
    h = rng.uniform(0.5, 2.0, len(X))
    I = np.zeros(shape)
    I[X[:, 0].astype(int), X[:, 1].astype(int)] = h
    return X, h, I


@pytest.mark.parametrize("xi,omega", [(1.5, 2.0), (2.0, 2.0), (1.6, 2.6)])
def test_gaussian_product_closed_form(xi, omega):
    # every Gaussian product summed over the lattice has width^2 >= xi^2 omega^2 / tau^2 >= 1.4
    assert xi * xi * omega * omega / (xi * xi + omega * omega) >= 1.4
    rng = np.random.default_rng(3)
    shape = (80, 90)
    Rx, Ro = int(math.ceil(8 * xi)), int(math.ceil(8 * omega))
    X, h, I = point_set(shape, rng, 40, Rx + Ro + 2)
    W = np.stack([rng.integers(Rx + Ro + 2, 80 - Rx - Ro - 2, 6), rng.integers(Rx + Ro + 2, 90 - Rx - Ro - 2, 6)],
                 1).astype(np.float64)
    P = O.density_map(I, xi, Rx)
    got, c, v_xw, v_w = O.literal_step(P, W, omega, Ro)
    tau2 = xi * xi + omega * omega
    den, num, GW, Gsum = O.original_terms(X, h, W, xi, omega)
    c_o = (h.sum() / len(W)) * O.overlap_xw(X, h, W, xi, omega) / O.overlap_w(W, omega)
    ref = (omega ** 2 / tau2) * num / den[:, None] + (xi ** 2 / tau2) * W \
        - 0.5 * c_o * (GW - Gsum[:, None] * W) / den[:, None]
    assert np.abs(got - ref).max() <= 1e-8
    # the lattice entropies are the Parzen overlaps up to the dropped normalisations
    assert v_xw == pytest.approx(O.overlap_xw(X, h, W, xi, omega) * h.sum() * len(W)
                                 * (2 * math.pi * xi * xi) * (2 * math.pi * omega * omega), rel=1e-10)
    assert v_w == pytest.approx(O.overlap_w(W, omega) * len(W) ** 2 * (2 * math.pi * omega * omega) ** 2,
                                rel=1e-10)


def test_equal_widths_is_the_damped_original():
    """xi = omega: one accelerated step is the original step damped by omega^2/tau^2 = 1/2."""
    rng = np.random.default_rng(5)
    xi = omega = 1.7
    R = int(math.ceil(8 * omega))
    X, h, I = point_set((70, 70), rng, 30, 2 * R + 2)
    W = np.stack([rng.integers(2 * R + 2, 70 - 2 * R - 2, 5)] * 2, 1).astype(np.float64)
    W[:, 1] = rng.integers(2 * R + 2, 70 - 2 * R - 2, 5)
    got, _, _, _ = O.literal_step(O.density_map(I, xi, R), W, omega, R)
    orig = O.original_step(X, h, W, xi, omega)
    assert np.abs(got - (0.5 * orig + 0.5 * W)).max() <= 1e-8


def test_fixed_point_when_the_codebook_is_the_data():
    img = S.config1_case(2).img
    W = np.argwhere(img > 0).astype(np.float64)
    P = O.density_map(img.astype(np.float64), 2.0, 6)
    got, c, _, _ = O.literal_step(P, W, 2.0, 6)
    assert c == pytest.approx(1.0, rel=1e-12)
    assert np.abs(got - W).max() <= 1e-9


def test_q_and_window_sums_brute_force():
    rng = np.random.default_rng(7)
    H, W_ = 9, 11
    P = rng.uniform(size=(H, W_))
    Wc = np.array([[0, 0], [4, 5], [8, 10], [4, 6], [4, 5]], np.float64)  # corners, a repeated pixel
    omega, R = 1.3, 3
    Q = O.literal_q((H, W_), Wc, omega, R)
    a, b, e, d = O.literal_terms(P, Q, Wc, omega, R)
    Qr = np.zeros((H, W_))
    for u in range(H):
        for v in range(W_):
            for w in Wc:
                if abs(u - w[0]) <= R and abs(v - w[1]) <= R:
                    Qr[u, v] += math.exp(-((u - w[0]) ** 2 + (v - w[1]) ** 2) / (2 * omega ** 2))
    assert np.allclose(Q, Qr, rtol=1e-14, atol=0)
    for k, w in enumerate(Wc):
        sa = sb0 = sb1 = se = sd0 = sd1 = 0.0
        for u in range(H):
            for v in range(W_):
                if abs(u - w[0]) <= R and abs(v - w[1]) <= R:
                    f = math.exp(-((u - w[0]) ** 2 + (v - w[1]) ** 2) / (2 * omega ** 2))
                    sa += P[u, v] * f; sb0 += P[u, v] * f * u; sb1 += P[u, v] * f * v
                    se += Qr[u, v] * f; sd0 += Qr[u, v] * f * u; sd1 += Qr[u, v] * f * v
        assert np.allclose([a[k], b[k, 0], b[k, 1], e[k], d[k, 0], d[k, 1]], [sa, sb0, sb1, se, sd0, sd1],
                           rtol=1e-12, atol=0)


def test_divergence_nonnegative_and_fit_on_lattice():
    for seed in (1, 3):
        c = S.config1_case(seed)
        xi, om = O.paper_widths(float(c.img.sum()), c.M)
        W, tr, done, _ = O.fit_literal(c.weights, c.w0, xi, om, 25)
        assert np.all(tr >= 0.0)
        assert np.array_equal(W, np.floor(W))
        assert W[:, 0].min() >= 0 and W[:, 0].max() <= 63 and W[:, 1].min() >= 0 and W[:, 1].max() <= 63
        assert tr[-1] < tr[0]


def test_theta_stops_when_nothing_moves():
    c = S.config1_case(1)
    xi, om = O.paper_widths(float(c.img.sum()), c.M)
    W, tr, done, _ = O.fit_literal(c.weights, c.w0, xi, om, 200, theta=0.5)
    assert done < 200
    W2, _, _, _ = O.fit_literal(c.weights, W, xi, om, 1)
    assert np.array_equal(W2, W)  # a fixed point on the lattice


def test_equivariance():
    """Integer translations and the transpose, with every window inside the lattice."""
    c = S.config1_case(3)
    xi, om = 1.8, 3.2

    def placed(du, dv):
        img = np.zeros((110, 100))
        img[du:du + 64, dv:dv + 64] = c.weights
        return img, c.w0 + np.array([du, dv], np.float64)

    img_a, W0_a = placed(20, 17)
    img_b, W0_b = placed(31, 24)
    Wa, tra, _, _ = O.fit_literal(img_a, W0_a, xi, om, 8)
    Wb, trb, _, _ = O.fit_literal(img_b, W0_b, xi, om, 8)
    assert np.array_equal(Wb, Wa + np.array([11.0, 7.0]))
    assert np.allclose(tra, trb, rtol=1e-12)
    WT, trT, _, _ = O.fit_literal(img_a.T, W0_a[:, ::-1], xi, om, 8)
    assert np.array_equal(WT, Wa[:, ::-1])
    assert np.allclose(trT, tra, rtol=1e-12)
