"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances:
  maps   normwise max|gpu - ref| / max|ref| <= 1e-5 per plane (FP32), 1e-12 (FP64)
  S_X    relative 1e-6 (FP32: map rounding, FP64 accumulation), 1e-12 (FP64)
  W      max_k ||w_gpu - w_ref|| <= 1e-3 px after the stated sweeps (FP32),
         1e-4 px after one sweep from the same codebook, 1e-9 px (FP64)
  D      |D_gpu - D_ref| <= 1e-5 * max(1, |D|)
"""
import functools

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu

DEV = "cuda"


def ref_maps(I, sigma, R):
    A, Bu, Bv = O.lattice_maps(I, sigma, R)
    Mu, Mv = O.moment_maps(A, Bu, Bv)
    return A, Mu, Mv


def normwise(got, ref):
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


def gpu_maps(itc, img_np, sigma, scale=1.0, radius=0, real=torch.float32, aligned=True):
    """Maps of a host image. 8-bit images are stored with a row pitch rounded up to 16 bytes and the
    padding filled with 255 (the kernels must ignore it), so that they take the matrix-core
    convolution; aligned=False keeps the contiguous layout (rows not 4-byte aligned when the width
    is not a multiple of 4: the vector-ALU convolution)."""
    img = torch.from_numpy(np.ascontiguousarray(img_np)).to(DEV)
    if aligned and img.dtype == torch.uint8 and img.shape[1] % 16:
        H, W = img.shape
        buf = torch.full((H, (W + 15) // 16 * 16), 255, dtype=torch.uint8, device=DEV)
        buf[:, :W].copy_(img)
        img = buf[:, :W]
    m = itc.precompute(img, sigma, scale=scale, radius=radius, real_dtype=real)
    torch.cuda.synchronize()
    return m, [p.cpu().double().numpy() for p in m.planes()], float(m.s_x.cpu()[0])


MAP_CASES = [
    # name, builder, sigma, scale, radius
    ("ellipses64", lambda: S.config1_case(1).img, 2.0, 1.0, 0),
    ("ragged70x133", lambda: (np.random.default_rng(1).uniform(size=(70, 133)) < 0.3).astype(np.uint8), 4.0, 1.0, 0),
    ("gray100x77_r24", lambda: S.gray_gaussians((7, 0), H=100, W=77, n=8, major=(5, 30)), 8.0, 1 / 255, 0),
    ("tiny1x1", lambda: np.ones((1, 1), np.uint8), 1.0, 1.0, 0),
    ("small3x5_r6", lambda: np.array([[0, 1, 1, 0, 1], [1, 1, 0, 0, 1], [0, 0, 1, 1, 1]], np.uint8), 2.0, 1.0, 0),
    ("explicit_r5", lambda: S.config1_case(2).img, 3.0, 1.0, 5),
    ("class_pad_r8", lambda: S.config1_case(3).img, 2.5, 1.0, 0),
    ("class_pad_r17", lambda: (np.random.default_rng(4).uniform(size=(90, 150)) < 0.5).astype(np.uint8), 5.5, 1.0, 0),
    ("tall300x40_r3", lambda: (np.random.default_rng(5).uniform(size=(300, 40)) < 0.2).astype(np.uint8), 1.0, 2.0, 0),
    # largest aligned radius class of the 8-bit path, gray levels up to 255
    ("gray160x210_r30", lambda: S.gray_gaussians((7, 1), H=160, W=210, n=10, major=(8, 40)), 10.0, 1 / 255, 0),
    # radius 32 with every weight 255: the largest row-pass values the FP16 split must hold
    ("const255_70x300_r32", lambda: np.full((70, 300), 255, np.uint8), 10.6, 1.0, 0),
    # tall enough for the single-image launch to split the rows into many segments
    ("segments700x150_r9", lambda: (np.random.default_rng(6).uniform(size=(700, 150)) < 0.4).astype(np.uint8), 3.0, 1.0, 0),
]


@pytest.mark.parametrize("name,build,sigma,scale,radius", MAP_CASES, ids=[c[0] for c in MAP_CASES])
def test_maps_fp32(gpu_lib, name, build, sigma, scale, radius):
    img = build()
    R = radius or S.radius_for(sigma)
    _, got, sx = gpu_maps(gpu_lib, img, sigma, scale, radius)
    I = img.astype(np.float64) * scale
    ref = ref_maps(I, sigma, R)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5
    sx_ref = float(np.sum(I * ref[0]))
    assert sx == pytest.approx(sx_ref, rel=1e-6)


UNALIGNED = [c for c in MAP_CASES if c[0] in ("ragged70x133", "gray100x77_r24", "small3x5_r6", "class_pad_r17")]


@pytest.mark.parametrize("name,build,sigma,scale,radius", UNALIGNED, ids=[c[0] for c in UNALIGNED])
def test_maps_unaligned_rows(gpu_lib, name, build, sigma, scale, radius):
    """8-bit rows that do not start 4-byte aligned (contiguous images of odd width) take the
    vector-ALU convolution; both kernels match the oracle and each other."""
    img = build()
    R = radius or S.radius_for(sigma)
    _, got_v, sx_v = gpu_maps(gpu_lib, img, sigma, scale, radius, aligned=False)
    _, got_m, sx_m = gpu_maps(gpu_lib, img, sigma, scale, radius, aligned=True)
    I = img.astype(np.float64) * scale
    ref = ref_maps(I, sigma, R)
    for gv, gm, r in zip(got_v, got_m, ref):
        assert normwise(gv, r) <= 1e-5 and normwise(gm, r) <= 1e-5
        assert normwise(gm, gv) <= 1e-5
    sx_ref = float(np.sum(I * ref[0]))
    assert sx_v == pytest.approx(sx_ref, rel=1e-6) and sx_m == pytest.approx(sx_ref, rel=1e-6)


@pytest.mark.parametrize("name,build,sigma,scale,radius", [c for c in MAP_CASES if c[2] <= 8.0],
                         ids=[c[0] for c in MAP_CASES if c[2] <= 8.0])
def test_maps_fp64(gpu_lib, name, build, sigma, scale, radius):
    img = build()
    R = radius or S.radius_for(sigma)
    _, got, sx = gpu_maps(gpu_lib, img, sigma, scale, radius, real=torch.float64)
    I = img.astype(np.float64) * scale
    ref = ref_maps(I, sigma, R)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-12
    assert sx == pytest.approx(float(np.sum(I * ref[0])), rel=1e-12)


def test_maps_float_weights_with_pitch(gpu_lib):
    """f32 weights stored with a row pitch larger than the width."""
    rng = np.random.default_rng(9)
    big = rng.uniform(0, 1, (50, 96)).astype(np.float32)
    t = torch.from_numpy(big).to(DEV)[:, 10:81]          # 50 x 71, pitch 96
    m = gpu_lib.precompute(t, 3.0)
    torch.cuda.synchronize()
    got = [p.cpu().double().numpy() for p in m.planes()]
    ref = ref_maps(big[:, 10:81].astype(np.float64), 3.0, 9)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5


def test_maps_full_size_512(gpu_lib):
    case = S.config2_case()
    _, got, sx = gpu_maps(gpu_lib, case.img, case.sigma)
    ref = ref_maps(case.weights, case.sigma, case.R)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5
    assert sx == pytest.approx(float(np.sum(case.weights * ref[0])), rel=1e-6)


# --------------------------------------------------------------------------- fit

def run_fit(itc, case, real=torch.float32, iters=None, theta=-1.0, w0=None):
    img = torch.from_numpy(case.img).to(DEV)
    m = itc.precompute(img, case.sigma, scale=case.scale, real_dtype=real)
    w0 = case.w0 if w0 is None else w0
    w, tr, done = itc.fit(m, torch.from_numpy(w0).to(DEV), case.iters if iters is None else iters, theta=theta)
    torch.cuda.synchronize()
    return m, w.cpu().double().numpy(), tr.cpu().numpy(), int(done.cpu()[0])


def wdist(a, b):
    return float(np.linalg.norm(a - b, axis=1).max())


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_fit_config1_fp64(gpu_lib, seed):
    case = S.config1_case(seed)
    _, w, tr, done = run_fit(gpu_lib, case, torch.float64)
    W_ref, tr_ref, _, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters)
    assert done == case.iters
    assert wdist(w, W_ref) <= 1e-9
    assert np.abs(tr - tr_ref).max() <= 1e-10 * max(1.0, abs(tr_ref).max())


@pytest.mark.parametrize("seed", [1, 2, 3, 4])
def test_fit_config1_fp32(gpu_lib, seed):
    case = S.config1_case(seed)
    _, w, tr, _ = run_fit(gpu_lib, case)
    W_ref, tr_ref, _, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters)
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


def test_one_step_config2(gpu_lib):
    case = S.config2_case()
    maps_ref = O.lattice_maps(case.weights, case.sigma, case.R)
    W5 = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, 5, maps=maps_ref)[0]
    _, w, tr, _ = run_fit(gpu_lib, case, iters=1, w0=W5)
    W6 = O.lattice_step(maps_ref, W5, case.sigma)
    assert wdist(w, W6) <= 1e-4
    d_ref = O.lattice_divergence(case.weights, maps_ref, W5, case.sigma)
    assert abs(tr[0] - d_ref) <= 1e-5 * max(1.0, abs(d_ref))


def test_fit_config2_full(gpu_lib):
    case = S.config2_case()
    _, w, tr, _ = run_fit(gpu_lib, case)
    W_ref, tr_ref, _, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters)
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


@functools.lru_cache(maxsize=1)
def config4_oracle():
    case = S.config4_case()
    return O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters)


def test_fit_config4_full(gpu_lib):
    """2048 x 2048 gray weights g/255, M = 500, sigma = 6, 200 sweeps."""
    case = S.config4_case()
    m, w, tr, _ = run_fit(gpu_lib, case)
    W_ref, tr_ref, _, maps_ref = config4_oracle()
    got = [p.cpu().double().numpy() for p in m.planes()]
    ref = (maps_ref[0],) + O.moment_maps(*maps_ref)
    for g, r in zip(got, ref):
        assert normwise(g, r) <= 1e-5
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


def test_theta_early_exit_fp64(gpu_lib):
    case = S.config1_case(8)
    _, w, tr, done = run_fit(gpu_lib, case, torch.float64, theta=0.05)
    W_ref, tr_ref, done_ref, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters, theta=0.05)
    assert done == done_ref and 0 < done < case.iters
    assert wdist(w, W_ref) <= 1e-9
    assert np.abs(tr[:done + 1] - tr_ref).max() <= 1e-10
    assert np.all(np.isnan(tr[done + 1:]))   # entries past the stop are untouched


def test_zero_iterations_and_divergence(gpu_lib):
    case = S.config1_case(2)
    m, w, tr, done = run_fit(gpu_lib, case, iters=0)
    assert done == 0 and np.array_equal(w, case.w0.astype(np.float32).astype(np.float64))
    d = float(gpu_lib.divergence(m, torch.from_numpy(case.w0).to(DEV)).cpu()[0])
    maps_ref = O.lattice_maps(case.weights, case.sigma, case.R)
    d_ref = O.lattice_divergence(case.weights, maps_ref, case.w0, case.sigma)
    assert tr[0] == d and abs(d - d_ref) <= 1e-5 * max(1, abs(d_ref))


def test_single_codevector_mean_shift(gpu_lib):
    """M = 1 is Gaussian mean shift (Section 2.2): the centre of a centrally symmetric
    shape is a fixed point, and from elsewhere the GPU follows the oracle's ascent."""
    m = np.zeros((41, 41), bool)
    S.fill_ellipse(m, 20.0, 20.0, 9.0, 5.0, 0.3)
    img = m.astype(np.uint8)
    centre = S.LatticeCase(img, 1.0, np.array([[20.0, 20.0]]), 2.0, 6, 50)
    _, w, _, _ = run_fit(gpu_lib, centre)
    assert wdist(w, np.array([[20.0, 20.0]])) <= 1e-5
    case = S.LatticeCase(img, 1.0, np.array([[17.3, 22.6]]), 2.0, 6, 300)
    _, w, tr, _ = run_fit(gpu_lib, case)
    W_ref, tr_ref, _, _ = O.fit_lattice(img.astype(float), case.w0, 2.0, 6, 300)
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())
    assert np.all(np.diff(tr) <= 1e-6)


def test_frozen_codevector_off_data(gpu_lib):
    case = S.config1_case(1)
    w0 = np.vstack([case.w0, [[1.0, 62.0], [-30.0, 5.0]]])
    case2 = S.LatticeCase(case.img, 1.0, w0, case.sigma, case.R, 20)
    _, w, _, _ = run_fit(gpu_lib, case2)
    assert np.array_equal(w[-2:], w0[-2:])
    W_ref = O.fit_lattice(case.weights, w0, case.sigma, case.R, 20)[0]
    assert wdist(w, W_ref) <= 1e-3


def test_output_may_alias_input(gpu_lib):
    case = S.config1_case(4)
    img = torch.from_numpy(case.img).to(DEV)
    m = gpu_lib.precompute(img, case.sigma)
    w = torch.from_numpy(case.w0).to(DEV, torch.float32)
    w2, _, _ = gpu_lib.fit(m, w.clone(), 10)
    wa = w.clone()
    gpu_lib.fit(m, wa, 10, w_out=wa)
    torch.cuda.synchronize()
    assert torch.equal(wa, w2)


def test_bitwise_reproducible(gpu_lib):
    case = S.config2_case()
    a = run_fit(gpu_lib, case, iters=20)
    b = run_fit(gpu_lib, case, iters=20)
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])
    pa = [p.cpu() for p in a[0].planes()]
    pb = [p.cpu() for p in b[0].planes()]
    assert all(torch.equal(x, y) for x, y in zip(pa, pb))


# ----------------------------------------------------------------- wide fit
# The single-image fit over several workgroups, one launch per sweep: the same
# bars against the oracle as the single-workgroup fit.

def run_fit_wide(itc, case, iters=None, theta=-1.0, w0=None, maps=None, work=None):
    m = maps if maps is not None else itc.precompute(torch.from_numpy(case.img).to(DEV), case.sigma,
                                                     scale=case.scale)
    w0 = case.w0 if w0 is None else w0
    w, tr, done = itc.fit_wide(m, torch.from_numpy(w0).to(DEV), case.iters if iters is None else iters,
                               theta=theta, work=work)
    torch.cuda.synchronize()
    return m, w.cpu().double().numpy(), tr.cpu().numpy(), int(done.cpu()[0])


def test_fit_wide_config4_full(gpu_lib):
    """2048 x 2048, M = 500 (16 workgroups), sigma = 6, 200 sweeps."""
    case = S.config4_case()
    _, w, tr, done = run_fit_wide(gpu_lib, case)
    W_ref, tr_ref, _, _ = config4_oracle()
    assert done == case.iters
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


@pytest.mark.parametrize("seed", [1, 4])
def test_fit_wide_config1(gpu_lib, seed):
    case = S.config1_case(seed)
    _, w, tr, done = run_fit_wide(gpu_lib, case)
    W_ref, tr_ref, _, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters)
    assert done == case.iters
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


def test_fit_wide_theta_stop(gpu_lib):
    """theta = 0.15 on the 512 x 512 shapes: the oracle stops after sweep 28 with its largest step
    1.6e-3 px below theta and every earlier one at least 3.9e-3 px above it."""
    case = S.config2_case()
    _, w, tr, done = run_fit_wide(gpu_lib, case, theta=0.15)
    W_ref, tr_ref, done_ref, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters, theta=0.15)
    assert done == done_ref == 28
    assert wdist(w, W_ref) <= 1e-3
    assert np.abs(tr[:done + 1] - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())
    assert np.all(np.isnan(tr[done + 1:]))   # entries past the stop are untouched


@pytest.mark.parametrize("M", [1, 31, 33, 257])
def test_fit_wide_ragged_codebooks(gpu_lib, M):
    """Codebook sizes that leave the last workgroup partly empty (32 codevectors per workgroup),
    two codevectors off the data (frozen) included when M allows."""
    case = S.config2_case()
    rng = np.random.default_rng(M)
    on = np.argwhere(case.img > 0)
    w0 = on[rng.choice(len(on), size=M, replace=False)].astype(np.float64) + 0.25
    if M >= 16:
        w0[-2:] = [[-40.0, 10.0], [600.0, 600.0]]
    c = S.LatticeCase(case.img, case.scale, w0, case.sigma, case.R, 15)
    _, w, tr, done = run_fit_wide(gpu_lib, c)
    W_ref, tr_ref, _, _ = O.fit_lattice(case.weights, w0, case.sigma, case.R, 15)
    assert done == 15
    assert wdist(w, W_ref) <= 1e-3
    if M >= 16:
        assert np.array_equal(w[-2:], w0[-2:])
    assert np.abs(tr - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


def test_fit_wide_zero_iterations_and_alias(gpu_lib):
    case = S.config1_case(2)
    m, w, tr, done = run_fit_wide(gpu_lib, case, iters=0)
    assert done == 0 and np.array_equal(w, case.w0.astype(np.float32).astype(np.float64))
    d = float(gpu_lib.divergence(m, torch.from_numpy(case.w0).to(DEV)).cpu()[0])
    assert abs(tr[0] - d) <= 1e-6 * max(1.0, abs(d))
    wi = torch.from_numpy(case.w0).to(DEV, torch.float32)
    ref, _, _ = gpu_lib.fit_wide(m, wi.clone(), 10)
    wa = wi.clone()
    gpu_lib.fit_wide(m, wa, 10, w_out=wa)
    torch.cuda.synchronize()
    assert torch.equal(wa, ref)


def test_fit_wide_reproducible_and_graph_replays(gpu_lib):
    """Bitwise equal run to run (fixed-order partial sums), and from a captured graph replayed
    three times with other work in between; a dirty work buffer does not matter."""
    case = S.config2_case()
    m = gpu_lib.precompute(torch.from_numpy(case.img).to(DEV), case.sigma)
    w0 = torch.from_numpy(case.w0).to(DEV, torch.float32)
    work = torch.full((gpu_lib.fit_wide_work_bytes(case.M),), 0x7f, dtype=torch.uint8, device=DEV)
    a = gpu_lib.fit_wide(m, w0, 30, work=work)
    b = gpu_lib.fit_wide(m, w0, 30, work=work)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1]) and int(a[2]) == int(b[2]) == 30
    w_out = torch.empty_like(w0)
    side = torch.cuda.Stream(device=DEV)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        gpu_lib.fit_wide(m, w0, 30, w_out=w_out, work=work, trace=False)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        gpu_lib.fit_wide(m, w0, 30, w_out=w_out, work=work, trace=False)
    for _ in range(3):
        w_out.fill_(float("nan"))
        work.fill_(0x55)
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(w_out, a[0])


def test_fit_wide_nonfinite_weights_stop(gpu_lib):
    """A NaN weight makes S_XW non-finite at the first codebook: both fits stop there."""
    case = S.config1_case(3)
    x = torch.from_numpy(case.img.astype(np.float32)).to(DEV)
    i, j = np.floor(case.w0[0]).astype(int)
    x[i, j] = float("nan")   # a corner of codevector 0's cell
    m = gpu_lib.precompute(x, case.sigma)
    w0 = torch.from_numpy(case.w0).to(DEV, torch.float32)
    w, _, done = gpu_lib.fit_wide(m, w0, 20)
    w1, _, done1 = gpu_lib.fit(m, w0, 20)
    torch.cuda.synchronize()
    assert int(done) == int(done1) == 0
    assert torch.equal(w, w0) and torch.equal(w1, w0)
