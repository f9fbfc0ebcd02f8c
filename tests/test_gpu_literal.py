"""Algorithm 1 with eq. (6) on the lattice: the HIP path against the oracle.

Codevectors are lattice points, so every sweep ends in a rounding decision.
The GPU computes P in FP32 (the convolution maps) and everything after in
FP64; the oracle is FP64 throughout, so a continuous update that lands within
about 1e-5 px of a half-integer can round the other way. Every GPU sweep is
checked against one oracle sweep taken from the GPU's own previous codebook:
the results must be equal except at near-ties of the oracle's continuous
update, where they may differ by one lattice step. So the whole GPU
trajectory is validated even after it has parted from the oracle's own. D at
every GPU codebook agrees to 1e-6 relative with the oracle's D at that
codebook; until the first near-tie the two trajectories are identical.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu

TIE = 1e-3  # px: a rounding decision this close to a half-integer may go either way


def gpu_run(itc, case, xi, omega, iters, theta=-1.0, w0=None):
    x = torch.from_numpy(case.img).cuda()
    w0 = case.w0 if w0 is None else w0
    w, tr, done = itc.fit_literal(x, torch.from_numpy(np.asarray(w0)).cuda().to(torch.int32), xi, omega, iters,
                                  theta=theta, scale=case.scale)
    torch.cuda.synchronize()
    return w.cpu().numpy().astype(np.float64), tr.cpu().numpy(), int(done.cpu()[0])


def oracle_trajectory(case, xi, omega, T):
    Rx = int(math.ceil(3 * xi - 1e-12))
    Ro = int(math.ceil(3 * omega - 1e-12))
    P = O.density_map(case.weights, xi, Rx)
    W = np.array(case.w0, np.float64)
    Ws, raw, D = [W], [], [O.literal_divergence(P, W, omega, Ro)]
    H, Wd = case.img.shape
    for _ in range(T):
        wn, _, _, _ = O.literal_step(P, W, omega, Ro)
        raw.append(wn)
        r = np.floor(wn + 0.5)
        r[:, 0] = np.clip(r[:, 0], 0, H - 1)
        r[:, 1] = np.clip(r[:, 1], 0, Wd - 1)
        W = r
        Ws.append(W)
        D.append(O.literal_divergence(P, W, omega, Ro))
    return Ws, raw, np.array(D)


def oracle_step(P, W, omega, Ro, shape):
    """One oracle sweep from codebook W: (continuous update, its lattice rounding)."""
    wn, _, _, _ = O.literal_step(P, W, omega, Ro)
    r = np.floor(wn + 0.5)
    r[:, 0] = np.clip(r[:, 0], 0, shape[0] - 1)
    r[:, 1] = np.clip(r[:, 1], 0, shape[1] - 1)
    return wn, r


def check_gpu_trajectory(itc, case, xi, omega, T, theta=-1.0, P=None, run=None):
    """Runs 1..T sweeps on the GPU and validates each against an oracle sweep from the GPU's previous
    codebook. Returns (GPU codebooks, sweeps during which the GPU equals the oracle's own run, sweeps done).
    P: the oracle's density (default: the masks of width xi); run(t, theta): the GPU call (default:
    itc.fit_literal on the case's weights)."""
    Ro = int(math.ceil(3 * omega - 1e-12))
    if P is None:
        P = O.density_map(case.weights, xi, int(math.ceil(3 * xi - 1e-12)))
    if run is None:
        run = lambda t, th: gpu_run(itc, case, xi, omega, t, theta=th)  # noqa: E731
    shape = case.img.shape
    w_full, trace, done_full = run(T, theta)
    prev = np.array(case.w0, np.float64)
    own = prev.copy()  # the oracle's own trajectory
    agreed, same = 0, True
    Ws = [prev]
    for t in range(1, done_full + 1):
        w, _, done = run(t, -1.0)
        assert done == t
        raw, ref = oracle_step(P, prev, omega, Ro, shape)
        for k, ax in np.argwhere(w != ref):
            frac = raw[k, ax] - np.floor(raw[k, ax])
            assert abs(frac - 0.5) < TIE, (t, k, ax, raw[k, ax], w[k, ax])
            assert abs(w[k, ax] - ref[k, ax]) == 1.0
        own = oracle_step(P, own, omega, Ro, shape)[1]
        same = same and np.array_equal(w, own)
        agreed = t if same else agreed
        # D at the GPU's codebook against the oracle's D at the same codebook
        assert trace[t] == pytest.approx(O.literal_divergence(P, w, omega, Ro), rel=1e-6), t
        prev = w
        Ws.append(w)
    assert trace[0] == pytest.approx(O.literal_divergence(P, np.array(case.w0, np.float64), omega, Ro), rel=1e-6)
    assert np.array_equal(w_full, Ws[-1])
    return Ws, agreed, done_full


def compare(itc, case, xi, omega, T):
    return check_gpu_trajectory(itc, case, xi, omega, T)[1]


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_literal_config1(gpu_lib, seed):
    """64 x 64 ellipses, M = 16, the paper's widths omega = sqrt(N/M)/2, xi = omega/2."""
    case = S.config1_case(seed)
    xi, om = O.paper_widths(float(case.img.sum()), case.M)
    agreed = compare(gpu_lib, case, xi, om, 20)
    assert agreed >= 10


def test_literal_config2(gpu_lib):
    """512 x 512 shapes, M = 100, paper widths (xi = 6.6, omega = 13.2: windows of 81 x 81 pixels)."""
    case = S.config2_case(0)
    xi, om = O.paper_widths(float(case.img.sum()), case.M)
    agreed = compare(gpu_lib, case, xi, om, 12)
    assert agreed >= 6


def test_literal_equal_widths_and_theta(gpu_lib):
    """xi = omega = 2 (R = 6) to convergence: theta = 0.5 stops after the first sweep that moves no
    codevector (moves are whole lattice steps), on a trajectory validated sweep by sweep."""
    case = S.config1_case(1)
    Ws, agreed, done = check_gpu_trajectory(gpu_lib, case, 2.0, 2.0, 100, theta=0.5)
    assert done < 100
    steps = [np.abs(Ws[t] - Ws[t - 1]).sum(axis=1).max() for t in range(1, done + 1)]
    assert all(s > 0 for s in steps[:-1]) and steps[-1] == 0  # the theta rule applied to the GPU's own steps
    # the oracle's own run stops by the same rule; where the runs never parted it stops at the same sweep
    Wo, tro, doneo, _ = O.fit_literal(case.weights, case.w0, 2.0, 2.0, 100, theta=0.5)
    if agreed == done:
        assert doneo == done and np.array_equal(Wo, Ws[-1])
    # converged on the lattice: one more sweep moves nothing
    w2, _, _ = gpu_run(gpu_lib, case, 2.0, 2.0, 1, w0=Ws[-1].astype(np.int32))
    assert np.array_equal(w2, Ws[-1])


def test_literal_zero_sweeps_and_clamp(gpu_lib):
    case = S.config1_case(2)
    xi, om = O.paper_widths(float(case.img.sum()), case.M)
    w, tr, done = gpu_run(gpu_lib, case, xi, om, 0)
    assert done == 0 and np.array_equal(w, case.w0)
    P = O.density_map(case.weights, xi, int(math.ceil(3 * xi - 1e-12)))
    assert tr[0] == pytest.approx(O.literal_divergence(P, case.w0, om, int(math.ceil(3 * om - 1e-12))), rel=1e-6)
    w0 = case.w0.astype(np.int32).copy()
    w0[0] = (-5, 3)
    w0[1] = (70, 200)
    w, _, _ = gpu_run(gpu_lib, case, xi, om, 0, w0=w0)
    assert tuple(w[0]) == (0, 3) and tuple(w[1]) == (63, 63)


def test_literal_rejects_bad_arguments(gpu_lib):
    x = torch.ones((8, 8), dtype=torch.uint8, device="cuda")
    w0 = torch.zeros((2, 2), dtype=torch.int32, device="cuda")
    for om, r in ((0.0, 0), (float("nan"), 0), (100.0, 0), (2.0, 257)):
        with pytest.raises(gpu_lib.ItcError):
            gpu_lib.fit_literal(x, w0, 1.0, om, 3, radius_omega=r)


# ---------------------------------------------------- P by recursive filtering
# The paper's widths on silhouettes whose xi exceeds the largest mask radius
# (xi > 32 / 3 px): P from the recursive Gaussian (Section 3.1), computed once
# on the GPU and handed to Algorithm 1; the oracle runs the same loop on its own
# FP64 recursive density.

def density_runner(itc, case, maps, omega):
    w0 = torch.from_numpy(np.asarray(case.w0)).cuda().to(torch.int32)

    def run(t, theta):
        w, tr, done = itc.fit_literal_density(maps, w0, omega, t, theta=theta)
        torch.cuda.synchronize()
        return w.cpu().numpy().astype(np.float64), tr.cpu().numpy(), int(done.cpu()[0])
    return run


@pytest.mark.parametrize("index", [14, 49])
def test_literal_recursive_density_paper_widths(gpu_lib, index):
    """Silhouettes 14 (M = 64, xi = 11.1, omega = 22.3) and 49 (M = 17, xi = 15.6, omega = 31.2) of the
    batch, with the paper's widths: beyond the masks, so P is the recursive density."""
    import oracle.recursive as OR
    case = S.config3_cases(indices=[index])[0]
    xi, om = O.paper_widths(float(case.img.sum()), case.M)
    assert xi > 32 / 3
    maps = gpu_lib.precompute_recursive(torch.from_numpy(case.img).cuda(), xi, scale=case.scale)
    P = OR.recursive_maps(case.weights, xi)[0]
    _, agreed, done = check_gpu_trajectory(gpu_lib, case, xi, om, 8, P=P,
                                           run=density_runner(gpu_lib, case, maps, om))
    assert done == 8 and agreed >= 4


def test_literal_recursive_density_wide_ellipse(gpu_lib):
    """One large ellipse (about 50,000 pixels), M = 4: xi = 28, omega = 56 (windows of 337 x 337), and
    the theta stop on a converged lattice codebook."""
    import oracle.recursive as OR
    m = np.zeros((300, 360), bool)
    S.fill_ellipse(m, 150.0, 175.0, 95.0, 160.0, 0.4)
    img = m.astype(np.uint8)
    rng = np.random.default_rng(7)
    on = np.argwhere(img > 0)
    w0 = on[rng.choice(len(on), size=4, replace=False)].astype(np.float64)
    case = S.LatticeCase(img, 1.0, w0, 1.0, 3, 40)
    xi, om = O.paper_widths(float(img.sum()), 4)
    assert 25 < xi < 35
    maps = gpu_lib.precompute_recursive(torch.from_numpy(img).cuda(), xi)
    P = OR.recursive_maps(img.astype(np.float64), xi)[0]
    Ws, agreed, done = check_gpu_trajectory(gpu_lib, case, xi, om, 40, theta=0.5, P=P,
                                            run=density_runner(gpu_lib, case, maps, om))
    assert done < 40 and np.array_equal(Ws[-1], Ws[-2])  # stopped on a sweep that moved nothing
    # the oracle's own run, where the two never parted, stops at the same sweep with the same codebook
    Wo, _, doneo, _ = O.fit_literal_density(P, w0, om, 40, theta=0.5)
    if agreed == done:
        assert doneo == done and np.array_equal(Wo, Ws[-1])
