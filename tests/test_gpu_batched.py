"""Batched persistent form vs the per-image calls and the oracle (config 3)."""
import json
import math
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def make_plan(itc, cases):
    imgs = [torch.from_numpy(c.img) for c in cases]
    plan = itc.BatchPlan(imgs, [c.M for c in cases], [c.sigma for c in cases], [c.iters for c in cases],
                         scales=[c.scale for c in cases])
    w0 = plan.pack_codebooks([c.w0 for c in cases])
    return plan, w0


def run_plan(plan, w0, theta=-1.0):
    n = plan.n
    w = torch.empty_like(w0)
    sx = torch.empty(n, dtype=torch.float64, device="cuda")
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    done = torch.empty(n, dtype=torch.int32, device="cuda")
    plan.run(w0, w, sx, d, done, theta)
    torch.cuda.synchronize()
    return w, sx, d, done


def test_batched_equals_per_image_bitwise(gpu_lib):
    """A 64-image slice of the silhouette batch: batched results are bitwise the per-image ones."""
    cases = S.config3_cases(indices=range(64))
    plan, w0 = make_plan(gpu_lib, cases)
    w, sx, d, done = run_plan(plan, w0)
    for i, c in enumerate(cases):
        img = plan.image(plan.weights, i)  # the packed image: same rows, same convolution kernel
        m = gpu_lib.precompute(img, c.sigma, scale=c.scale)
        wi, tr, di = gpu_lib.fit(m, torch.from_numpy(c.w0).cuda(), c.iters)
        torch.cuda.synchronize()
        assert torch.equal(plan.unpack(w, i), wi), i
        assert float(sx[i]) == float(m.s_x[0]), i
        assert float(d[i]) == float(tr[-1]), i
        assert int(done[i]) == c.iters
        # maps inside the packed buffer equal the per-image maps
        pb = plan.maps_of(i).planes()
        for x, y in zip(pb, m.planes()):
            assert torch.equal(x, y), i


def large_m_cases():
    """Gray images whose codebooks need two and four passes of the fit
    (M = 257..1024) beside small ones, several widths."""
    out = []
    for i, (M, sigma, H, W) in enumerate([(10, 2.0, 96, 120), (257, 3.0, 160, 200), (300, 4.0, 144, 176),
                                          (700, 2.0, 200, 240), (1024, 3.0, 224, 256), (64, 4.0, 128, 128)]):
        img = S.gray_gaussians((9, i), H=H, W=W, n=12, major=(8, 40))
        w0 = S.sample_init(img, M, (9, i, 1))
        out.append(S.LatticeCase(img, 1.0 / 255.0, w0, sigma, S.radius_for(sigma), 20, name=f"gray-M{M}"))
    return out


def test_batched_large_codebooks(gpu_lib):
    """Codebooks of up to 1,024 codevectors in one plan: batched results are
    bitwise the per-image ones. Against the oracle: M = 300 (two passes)
    after the 20 sweeps, M = 1,024 (four passes) after one sweep. With 700 or
    1,024 codevectors on ~5e4 weighted pixels the iteration is unstable
    (codevectors with almost no data in their window take huge steps), so
    rounding differences grow about tenfold per sweep from the second on."""
    cases = large_m_cases()
    plan, w0 = make_plan(gpu_lib, cases)
    w, sx, d, done = run_plan(plan, w0)
    for i, c in enumerate(cases):
        m = gpu_lib.precompute(plan.image(plan.weights, i), c.sigma, scale=c.scale)
        wi, tr, _ = gpu_lib.fit(m, torch.from_numpy(c.w0).cuda(), c.iters)
        torch.cuda.synchronize()
        assert torch.equal(plan.unpack(w, i), wi), c.name
        assert float(d[i]) == float(tr[-1]), c.name
        assert int(done[i]) == c.iters
    c = cases[2]
    W_ref, tr_ref, _, _ = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters)
    got = plan.unpack(w, 2).cpu().double().numpy()
    assert np.linalg.norm(got - W_ref, axis=1).max() <= 1e-3
    assert abs(float(d[2]) - tr_ref[-1]) <= 1e-5 * max(1.0, abs(tr_ref[-1]))
    c = cases[4]
    m = gpu_lib.precompute(torch.from_numpy(c.img).cuda(), c.sigma, scale=c.scale)
    w1, tr1, _ = gpu_lib.fit(m, torch.from_numpy(c.w0).cuda(), 1)
    torch.cuda.synchronize()
    W1, trr1, _, _ = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, 1)
    assert np.linalg.norm(w1.cpu().double().numpy() - W1, axis=1).max() <= 1e-4
    assert np.abs(tr1.cpu().numpy() - trr1).max() <= 1e-5 * max(1.0, np.abs(trr1).max())


def test_full_batch_sampled_against_oracle(gpu_lib):
    """All 1,400 silhouettes in one plan (the benchmark's launch configuration);
    sampled images are checked against the oracle one by one."""
    cases = S.config3_cases()
    plan, w0 = make_plan(gpu_lib, cases)
    w, sx, d, done = run_plan(plan, w0)
    assert torch.all(done == 100)
    assert torch.all(torch.isfinite(d))
    rng = np.random.default_rng(0)
    sample = sorted(set([0, len(cases) - 1] + list(rng.choice(len(cases), 5, replace=False))))
    for i in sample:
        c = cases[i]
        W_ref, tr_ref, _, maps_ref = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters)
        got = plan.unpack(w, i).cpu().double().numpy()
        assert np.linalg.norm(got - W_ref, axis=1).max() <= 1e-3, (i, c.sigma, c.M)
        assert abs(float(d[i]) - tr_ref[-1]) <= 1e-5 * max(1.0, abs(tr_ref[-1])), i
        assert float(sx[i]) == pytest.approx(float(np.sum(c.weights * maps_ref[0])), rel=1e-6)


def test_full_batch_divergence_every_image(gpu_lib):
    """All 1,400 silhouettes: D at the final codebook within 1e-5 (relative to
    max(1, |D|)) of the oracle's for every image; the oracle's values are
    written by tests/golden/make_silhouettes_d.py. D is what is unique here:
    on a few wide-kernel images the objective is flat along some directions,
    and rounding moves codevectors along them without changing D."""
    path = os.path.join(os.path.dirname(__file__), "golden", "silhouettes1400_d.json")
    with open(path) as f:
        ref = np.array(json.load(f)["d"])
    cases = S.config3_cases()
    assert ref.shape == (len(cases),)
    plan, w0 = make_plan(gpu_lib, cases)
    _, _, d, done = run_plan(plan, w0)
    assert torch.all(done == 100)
    err = np.abs(d.cpu().numpy() - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 1e-5, (int(err.argmax()), float(err.max()))


# ---------------------------------------------------------------------------
# every codebook of the silhouette batch against the oracle
# ---------------------------------------------------------------------------
_CASES = None  # the batch, shared with forked oracle workers


def _oracle_final(i):
    c = _CASES[i]
    W, tr, _, _ = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters)
    return W, float(tr[-1])


def _oracle_exception(args):
    """Oracle evidence at a codebook W_gpu that is farther than 1e-3 px from the oracle's:
    D at W_gpu, the length of one oracle sweep from W_gpu, the oracle's own last sweep length,
    and the spread FP64 rounding alone gives the oracle's final codebook (maps times 1 + 1e-15 xi)."""
    i, wg, W100 = args
    c = _CASES[i]
    maps = O.lattice_maps(c.weights, c.sigma, c.R)
    d_at = O.lattice_divergence(c.weights, maps, wg, c.sigma)
    w1 = O.fit_lattice(c.weights, wg, c.sigma, c.R, 1, maps=maps)[0]
    W99 = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters - 1, maps=maps)[0]
    rng = np.random.default_rng(i)
    noisy = tuple(m * (1.0 + 1e-15 * rng.standard_normal(m.shape)) for m in maps)
    Wn = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters, maps=noisy)[0]
    step = lambda a, b: float(np.linalg.norm(a - b, axis=1).max())  # noqa: E731
    return d_at, step(w1, wg), step(W100, W99), step(Wn, W100)


def test_full_batch_codebooks_every_image(gpu_lib):
    """All 1,400 silhouettes in the benchmark's launch: every final codebook is within 1e-3 px of the
    oracle's, except on ill-conditioned images, where it must be a state the oracle's own iteration
    accepts. On those images (about 18, sigma 4 and 8, still moving 0.02-0.2 px per sweep after the
    100 sweeps) rounding the oracle's own maps to FP32 alone moves its codebook by 1e-3 to 54 px, so no
    FP32 computation meets the 1e-3 px bar there. For each exception:
      - the oracle's D at the GPU codebook is within 1e-5 max(1, |D|) of the oracle's final D;
      - one oracle sweep from the GPU codebook moves it no farther than 1.05 times the oracle's own
        last sweep, plus 1e-4 px (the GPU codebook is at the same stage of the iteration);
      - the FP64 instantiation of the kernels (FP64 maps and fit, same image) is within
        max(1e-9, 20 s) px of the oracle, s the spread that FP64 rounding alone gives the oracle
        (its maps times 1 + 1e-15 N(0, 1)), which proves the kernels on those images."""
    import multiprocessing as mp

    global _CASES
    cases = S.config3_cases()
    _CASES = cases
    plan, w0 = make_plan(gpu_lib, cases)
    w, sx, d, done = run_plan(plan, w0)
    assert torch.all(done == 100)
    wg_all = w.cpu().double().numpy()
    nproc = max(1, min(16, len(os.sched_getaffinity(0))))
    with mp.get_context("fork").Pool(nproc) as pool:
        ref = pool.map(_oracle_final, range(len(cases)), chunksize=4)
        exc = []
        for i, c in enumerate(cases):
            wg = wg_all[plan.w_offsets[i]: plan.w_offsets[i] + c.M]
            if np.linalg.norm(wg - ref[i][0], axis=1).max() > 1e-3:
                exc.append((i, wg, ref[i][0]))
        evidence = pool.map(_oracle_exception, exc)
    print(f"{len(exc)} of {len(cases)} codebooks beyond 1e-3 px: {[e[0] for e in exc]}")
    assert len(exc) <= 40
    for (i, wg, W100), (d_at, step_gpu, step_last, spread) in zip(exc, evidence):
        c = cases[i]
        D = ref[i][1]
        assert c.sigma >= 4.0, i
        assert abs(d_at - D) <= 1e-5 * max(1.0, abs(D)), (i, d_at, D)
        assert step_gpu <= 1.05 * step_last + 1e-4, (i, step_gpu, step_last)
        m = gpu_lib.precompute(plan.image(plan.weights, i), c.sigma, scale=c.scale, real_dtype=torch.float64)
        w64, _, _ = gpu_lib.fit(m, torch.from_numpy(c.w0).cuda().double(), c.iters)
        torch.cuda.synchronize()
        err64 = float(np.linalg.norm(w64.cpu().numpy() - W100, axis=1).max())
        assert err64 <= max(1e-9, 20.0 * spread), (i, err64, spread)


def test_full_batch_maps_largest_per_sigma(gpu_lib):
    """The maps of the largest silhouette of each sigma class, as the batched launch wrote them, against
    the oracle element by element (normwise 1e-5 per plane) and S_X (1e-6)."""
    cases = S.config3_cases()
    plan, w0 = make_plan(gpu_lib, cases)
    w, sx, d, done = run_plan(plan, w0)
    for sigma in (2.0, 4.0, 8.0):
        i = max((k for k, c in enumerate(cases) if c.sigma == sigma), key=lambda k: cases[k].img.size)
        c = cases[i]
        got = [p.cpu().double().numpy() for p in plan.maps_of(i).planes()]
        A, Bu, Bv = O.lattice_maps(c.weights, c.sigma, c.R)
        ref = (A,) + tuple(O.moment_maps(A, Bu, Bv))
        for g, r in zip(got, ref):
            assert float(np.abs(g - r).max() / np.abs(r).max()) <= 1e-5, (i, sigma)
        assert float(sx[i]) == pytest.approx(float(np.sum(c.weights * A)), rel=1e-6)


def oracle_accepts(c, wg, W_ref, D_ref, k, maps):
    """On an ill-conditioned image whose GPU codebook wg (after k sweeps) is farther than 1e-3 px from
    the oracle's W_ref: the oracle's D at wg within 1e-5 max(1, |D|) of D_ref, and one oracle sweep
    from wg no longer than 1.05 times the oracle's own last sweep plus 1e-4 px."""
    d_at = O.lattice_divergence(c.weights, maps, wg, c.sigma)
    w1 = O.fit_lattice(c.weights, wg, c.sigma, c.R, 1, maps=maps)[0]
    W_prev = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, k - 1, maps=maps)[0]
    step_gpu = float(np.linalg.norm(w1 - wg, axis=1).max())
    step_last = float(np.linalg.norm(W_ref - W_prev, axis=1).max())
    return abs(d_at - D_ref) <= 1e-5 * max(1.0, abs(D_ref)) and step_gpu <= 1.05 * step_last + 1e-4


def test_batched_theta_stop_against_oracle(gpu_lib):
    """The batched theta stop (stop after the first sweep whose largest codevector step is <= theta)
    against the oracle's rule on 40 silhouettes: the same sweep count, except where the deciding step
    lies within 1e-3 theta of theta (FP32 rounding may then decide either way, by one sweep), and the
    codebooks within 1e-3 px where the counts agree (or, on the ill-conditioned images of the batch, a
    codebook the oracle's iteration accepts, as in test_full_batch_codebooks_every_image)."""
    theta = 0.05
    cases = S.config3_cases(indices=range(200, 240))
    plan, w0 = make_plan(gpu_lib, cases)
    w, sx, d, done = run_plan(plan, w0, theta=theta)
    stopped = 0
    for i, c in enumerate(cases):
        W_ref, tr_ref, done_ref, maps = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters, theta=theta)
        k = int(done[i])
        stopped += k < c.iters
        if k != done_ref:
            assert abs(k - done_ref) == 1, (i, k, done_ref)
            # the oracle's step at the earlier of the two sweeps decides: it must be a near-tie
            Wa = O.fit_lattice(c.weights, c.w0, c.sigma, c.R, min(k, done_ref) - 1, maps=maps)[0]
            Wb = O.fit_lattice(c.weights, Wa, c.sigma, c.R, 1, maps=maps)[0]
            step = float(np.linalg.norm(Wb - Wa, axis=1).max())
            assert abs(step - theta) <= 1e-3 * theta, (i, step)
            continue
        got = plan.unpack(w, i).cpu().double().numpy()
        if np.linalg.norm(got - W_ref, axis=1).max() > 1e-3:  # an ill-conditioned image (see above)
            assert oracle_accepts(c, got, W_ref, tr_ref[-1], k, maps), (i, c.sigma, c.M)
        assert abs(float(d[i]) - tr_ref[-1]) <= 1e-5 * max(1.0, abs(tr_ref[-1])), i
    assert stopped >= 5  # the stop is exercised


def test_batched_status_flags_nonfinite_weights(gpu_lib):
    """FP32 weights with a NaN under a codevector of one image: that image's status has the non-finite-sums bit, its fit
    stops at once (iters_done 0, w_out the initial codebook) with D not finite; the other images are
    untouched (status 0, the same results as without the bad image)."""
    cases = S.config3_cases(indices=range(300, 306))
    imgs = [torch.from_numpy(c.img.astype(np.float32)) for c in cases]
    def plan_of(images):
        p = gpu_lib.BatchPlan(images, [c.M for c in cases], [c.sigma for c in cases], [c.iters for c in cases])
        return p, p.pack_codebooks([c.w0 for c in cases])
    good, w0 = plan_of(imgs)
    bad_imgs = list(imgs)
    bad_imgs[2] = imgs[2].clone()
    u0, v0 = (int(round(x)) for x in cases[2].w0[0])  # under codevector 0: its first map read is NaN
    bad_imgs[2][u0, v0] = float("nan")
    bad, _ = plan_of(bad_imgs)
    outs = []
    for p in (good, bad):
        n = p.n
        w = torch.empty_like(w0)
        d = torch.empty(n, dtype=torch.float64, device="cuda")
        done = torch.empty(n, dtype=torch.int32, device="cuda")
        st = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        p.run(w0, w, d_out=d, iters_done=done, status=st)
        torch.cuda.synchronize()
        outs.append((w, d, done, st))
    (wg, dg, doneg, stg), (wb, db, doneb, stb) = outs
    assert torch.all(stg == 0) and torch.all(doneg == 100)
    assert int(stb[2]) & gpu_lib.ITC_FIT_NONFINITE_SUMS and int(stb[2]) & gpu_lib.ITC_FIT_NONFINITE_D
    assert int(doneb[2]) == 0 and not math.isfinite(float(db[2]))
    assert torch.equal(bad.unpack(wb, 2), bad.unpack(w0, 2))
    for i in (0, 1, 3, 4, 5):
        assert int(stb[i]) == 0 and int(doneb[i]) == 100
        assert torch.equal(bad.unpack(wb, i), good.unpack(wg, i)) and float(db[i]) == float(dg[i])


def test_batched_theta_and_graph_replay(gpu_lib):
    """The plan's launches capture into a HIP graph; every replay matches eager."""
    cases = S.config3_cases(indices=range(100, 116))
    plan, w0 = make_plan(gpu_lib, cases)
    w_e, sx_e, d_e, done_e = run_plan(plan, w0, theta=1e-3)
    assert torch.all(done_e <= 100)
    n = plan.n
    w = torch.empty_like(w0)
    sx = torch.empty(n, dtype=torch.float64, device="cuda")
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    done = torch.empty(n, dtype=torch.int32, device="cuda")
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        plan.run(w0, w, sx, d, done, 1e-3)        # warm-up outside capture
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        plan.run(w0, w, sx, d, done, 1e-3)
    for _ in range(3):
        w.zero_(); d.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(w, w_e) and torch.equal(d, d_e) and torch.equal(done, done_e)
        assert torch.equal(sx, sx_e)
