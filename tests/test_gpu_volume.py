"""3-D lattices: the HIP volume maps and fit against the oracle."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def normwise(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def oracle_moments(maps):
    A, Bs, Bu, Bv = maps
    s, u, v = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in A.shape], indexing="ij")
    return A, s * A - Bs, u * A - Bu, v * A - Bv


def gpu_maps(itc, vol, sigma, scale=1.0, radius=0, pad=None):
    x = torch.from_numpy(vol).cuda()
    if pad is not None:
        D, H, W = vol.shape
        buf = torch.zeros((D, H + pad[0], W + pad[1]), dtype=x.dtype, device="cuda")
        buf[:, :H, :W] = x
        x = buf[:, :H, :W]
    m = itc.volume_precompute(x, sigma, scale=scale, radius=radius)
    torch.cuda.synchronize()
    return m, [p.cpu().double().numpy() for p in m.planes()], float(m.s_x.cpu()[0])


CASES = [
    ("ellipsoids48x56x64_s2", lambda: S.volume_case(0).vol, 2.0, 1.0, 0, None),
    ("ellipsoids_s3_r5_pitched", lambda: S.volume_case(1, D=30, H=36, W=40).vol, 3.0, 1.0, 5, (3, 7)),
    ("f32_random_20x17x23", lambda: np.random.default_rng(1).uniform(size=(20, 17, 23)).astype(np.float32), 1.5,
     0.5, 0, None),
    ("depth1_64x64", lambda: S.config1_case(1).img[None].copy(), 2.0, 1.0, 0, None),
    ("tiny1x1x1", lambda: np.ones((1, 1, 1), np.uint8), 1.0, 1.0, 0, None),
    # the wider in-plane staging classes (radius 9..16 and 17..32), ragged tiles
    ("ellipsoids_s4_r12", lambda: S.volume_case(4, D=30, H=40, W=72).vol, 4.0, 1.0, 0, (1, 3)),
    ("f64_s8_r32", lambda: np.random.default_rng(5).uniform(size=(19, 70, 90)), 8.0, 2.0, 32, None),
    # radius 2: the column passes take the zero-padded window instead of the ramps
    ("u8_s06_r2", lambda: S.volume_case(1, D=30, H=36, W=40).vol, 0.6, 1.0, 0, None),
]


@pytest.mark.parametrize("name,build,sigma,scale,radius,pad", CASES, ids=[c[0] for c in CASES])
def test_volume_maps(gpu_lib, name, build, sigma, scale, radius, pad):
    vol = build()
    R = radius or S.radius_for(sigma)
    _, got, sx = gpu_maps(gpu_lib, vol, sigma, scale, radius, pad)
    I = vol.astype(np.float64) * scale
    ref = oracle_moments(O.volume_maps(I, sigma, R))
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5
    assert sx == pytest.approx(float(np.sum(I * ref[0])), rel=1e-6)


def test_volume_fit(gpu_lib):
    case = S.volume_case(0)
    m, _, _ = gpu_maps(gpu_lib, case.vol, case.sigma)
    W_ref, tr_ref, _, _ = O.fit_volume(case.weights, case.w0, case.sigma, case.R, case.iters)
    w, tr, done = gpu_lib.volume_fit(m, torch.from_numpy(case.w0).cuda(), case.iters)
    torch.cuda.synchronize()
    assert int(done.cpu()[0]) == case.iters
    assert float(np.linalg.norm(w.cpu().double().numpy() - W_ref, axis=1).max()) <= 1e-3
    assert np.abs(tr.cpu().numpy() - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())
    w1, _, _ = gpu_lib.volume_fit(m, torch.from_numpy(case.w0).cuda(), 1)
    W1, _, _, _ = O.fit_volume(case.weights, case.w0, case.sigma, case.R, 1)
    assert float(np.linalg.norm(w1.cpu().double().numpy() - W1, axis=1).max()) <= 1e-4


def test_volume_fit_many_codevectors_and_theta(gpu_lib):
    """600 codevectors (three per thread) for 5 sweeps; then theta stops a small codebook."""
    case = S.volume_case(2, D=40, H=48, W=56, M=600, iters=5)
    m, _, _ = gpu_maps(gpu_lib, case.vol, case.sigma)
    W_ref, tr_ref, _, _ = O.fit_volume(case.weights, case.w0, case.sigma, case.R, case.iters)
    w, tr, _ = gpu_lib.volume_fit(m, torch.from_numpy(case.w0).cuda(), case.iters)
    torch.cuda.synchronize()
    assert float(np.linalg.norm(w.cpu().double().numpy() - W_ref, axis=1).max()) <= 1e-3
    assert np.abs(tr.cpu().numpy() - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())
    small = S.volume_case(3, D=30, H=36, W=40, M=6, iters=500)
    ms, _, _ = gpu_maps(gpu_lib, small.vol, small.sigma)
    w, tr, done = gpu_lib.volume_fit(ms, torch.from_numpy(small.w0).cuda(), 500, theta=1e-4)
    torch.cuda.synchronize()
    Wt, trt, dt, _ = O.fit_volume(small.weights, small.w0, small.sigma, small.R, 500, theta=1e-4)
    assert int(done.cpu()[0]) < 500
    assert abs(int(done.cpu()[0]) - dt) <= 2
    assert float(np.linalg.norm(w.cpu().double().numpy() - Wt, axis=1).max()) <= 1e-3


@pytest.mark.parametrize("M", [1, 3, 12, 64, 100, 200, 300])
def test_volume_fit_lane_layouts(gpu_lib, M):
    """Every layout of the fit: 64, 32, 16, 4, 2 and 1 lanes per codevector,
    and two codevectors per thread (M = 300), against the oracle for 3 sweeps."""
    case = S.volume_case(5, D=32, H=40, W=48, M=M, iters=3)
    m, _, _ = gpu_maps(gpu_lib, case.vol, case.sigma)
    W_ref, tr_ref, _, _ = O.fit_volume(case.weights, case.w0, case.sigma, case.R, case.iters)
    w, tr, done = gpu_lib.volume_fit(m, torch.from_numpy(case.w0).cuda(), case.iters)
    torch.cuda.synchronize()
    assert int(done.cpu()[0]) == case.iters
    assert float(np.linalg.norm(w.cpu().double().numpy() - W_ref, axis=1).max()) <= 1e-3
    assert np.abs(tr.cpu().numpy() - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


def test_volume_rejects(gpu_lib):
    x = torch.ones((4, 4, 4), dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu_lib.ItcError):
        gpu_lib.volume_precompute(x, 30.0)  # radius 90 > 32
