"""Chamfer distance transform (Section 5 weighting) on the GPU vs the oracle's
Borgefors two-pass propagation: integer costs, compared bit for bit; then the
weighted fit P = T(X) * G_xi against the oracle's lattice fit on T / a."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def rand_img(seed, H, W, p):
    return (np.random.default_rng(seed).uniform(size=(H, W)) < p).astype(np.uint8)


def gpu_chamfer(itc, img, a=3, b=4, pitch=None):
    H, W = img.shape
    if pitch is None:
        x = torch.from_numpy(img).cuda()
    else:
        buf = torch.zeros((H, pitch), dtype=torch.uint8, device="cuda")
        buf[:, :W] = torch.from_numpy(img).cuda()
        x = buf[:, :W]
    t = itc.chamfer(x, a, b)
    torch.cuda.synchronize()
    return t.cpu().numpy()


CASES = [
    ("ellipses64", lambda: S.config1_case(1).img),
    ("shapes512", lambda: S.config2_case(0).img),
    ("ragged37x1000", lambda: rand_img(1, 37, 1000, 0.93)),
    ("tiny1x1_fg", lambda: np.ones((1, 1), np.uint8)),
    ("tiny1x1_bg", lambda: np.zeros((1, 1), np.uint8)),
    ("row1x300", lambda: rand_img(2, 1, 300, 0.97)),
    ("col300x1", lambda: rand_img(3, 300, 1, 0.97)),
    ("all_fg_70x129", lambda: np.ones((70, 129), np.uint8)),
    ("all_bg_40x40", lambda: np.zeros((40, 40), np.uint8)),
    ("gray_levels", lambda: S.gray_gaussians((7, 2), H=90, W=140, n=6, major=(10, 30))),
    # columns of at most 1,024 rows take the bit-mask column pass, taller ones the two-walk pass
    ("rows1024", lambda: rand_img(8, 1024, 70, 0.995)),
    ("rows1025", lambda: rand_img(9, 1025, 70, 0.995)),
    ("tall1500x33", lambda: rand_img(10, 1500, 33, 0.99)),
]


@pytest.mark.parametrize("name,build", CASES, ids=[c[0] for c in CASES])
def test_chamfer_34(gpu_lib, name, build):
    img = build()
    ref = O.chamfer_transform(img, 3, 4)
    got = gpu_chamfer(gpu_lib, img)
    assert np.array_equal(got, ref.astype(np.float32))


@pytest.mark.parametrize("a,b", [(1, 1), (1, 2), (5, 7), (2, 3), (64, 100)])
def test_chamfer_masks(gpu_lib, a, b):
    img = rand_img(5, 61, 77, 0.9)
    assert np.array_equal(gpu_chamfer(gpu_lib, img, a, b), O.chamfer_transform(img, a, b).astype(np.float32))


def test_chamfer_pitch_and_widest(gpu_lib):
    img = rand_img(6, 45, 200, 0.9)
    assert np.array_equal(gpu_chamfer(gpu_lib, img, pitch=256), O.chamfer_transform(img).astype(np.float32))
    wide = rand_img(7, 3, 16384, 0.99)  # the widest accepted row: 64 KB of LDS
    assert np.array_equal(gpu_chamfer(gpu_lib, wide), O.chamfer_transform(wide).astype(np.float32))


def test_chamfer_rejects_bad_masks(gpu_lib):
    img = torch.ones((4, 4), dtype=torch.uint8, device="cuda")
    for a, b in ((0, 0), (3, 2), (3, 7), (65, 65)):
        with pytest.raises(gpu_lib.ItcError):
            gpu_lib.chamfer(img, a, b)


def test_chamfer_batched(gpu_lib):
    """48 silhouettes in one plan: batched equals per-image bit for bit; two checked against the oracle."""
    cases = S.config3_cases(indices=range(48))
    plan = gpu_lib.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                             [c.sigma for c in cases], [c.iters for c in cases])
    t = plan.chamfer()
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        ti = plan.image(t, i)
        assert torch.equal(ti, gpu_lib.chamfer(torch.from_numpy(c.img).cuda())), i
    for i in (0, 17):
        got = plan.image(t, i).cpu().numpy()
        assert np.array_equal(got, O.chamfer_transform(cases[i].img).astype(np.float32)), i


def ragged_batch_images():
    """300 binary images: ragged widths around the 64-column strips, single rows and columns, all foreground,
    all background."""
    rng = np.random.default_rng(11)
    imgs = [np.ones((1, 1), np.uint8), np.zeros((1, 1), np.uint8), rand_img(20, 1, 1024, 0.98),
            rand_img(21, 60, 1024, 0.97), rand_img(22, 60, 1, 0.97), np.ones((40, 129), np.uint8),
            np.zeros((33, 77), np.uint8), np.ones((1, 1024), np.uint8), np.ones((97, 1), np.uint8)]
    imgs += [rand_img(30 + k, 23, w, 0.95) for k, w in enumerate((63, 64, 65, 127, 128, 129, 960, 1023))]
    while len(imgs) < 300:
        H, W = int(rng.integers(1, 48)), int(rng.integers(1, 1025))
        imgs.append(rand_img(1000 + len(imgs), H, W, float(rng.uniform(0.6, 1.0))))
    return imgs


def test_chamfer_batched_ragged_every_image(gpu_lib):
    """The batched transform over 300 ragged images: every image against the oracle for five masks."""
    imgs = ragged_batch_images()
    plan = gpu_lib.BatchPlan([torch.from_numpy(im) for im in imgs], [1] * len(imgs), [2.0] * len(imgs),
                             [1] * len(imgs))
    for a, b in ((3, 4), (1, 1), (1, 2), (5, 7), (64, 100)):
        t = plan.chamfer(a, b)
        torch.cuda.synchronize()
        for i, im in enumerate(imgs):
            got = plan.image(t, i).cpu().numpy()
            assert np.array_equal(got, O.chamfer_transform(im, a, b).astype(np.float32)), (a, b, i, im.shape)


def test_chamfer_batched_silhouettes_full(gpu_lib):
    """All 1,400 silhouettes in one plan (the batch the benchmark times): the tallest, the widest, the smallest
    and every 97th image equal the per-image transform bit for bit; two also against the oracle."""
    cases = S.config3_cases(1400)
    plan = gpu_lib.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                             [c.sigma for c in cases], [c.iters for c in cases])
    t = plan.chamfer()
    torch.cuda.synchronize()
    shapes = [c.img.shape for c in cases]
    pick = {int(np.argmax([h for h, _ in shapes])), int(np.argmax([w for _, w in shapes])),
            int(np.argmin([h * w for h, w in shapes]))} | set(range(0, 1400, 97))
    for i in sorted(pick):
        ref = gpu_lib.chamfer(torch.from_numpy(cases[i].img).cuda())
        assert torch.equal(plan.image(t, i), ref), i
    for i in sorted(pick)[:2]:
        got = plan.image(t, i).cpu().numpy()
        assert np.array_equal(got, O.chamfer_transform(cases[i].img).astype(np.float32)), i


@pytest.mark.parametrize("seed", [1, 2])
def test_weighted_fit_config1(gpu_lib, seed):
    """Section 5: P = T(X) * G_xi with the 3-4 chamfer T; the fit on T / 3 matches the oracle."""
    case = S.config1_case(seed)
    x = torch.from_numpy(case.img).cuda()
    t = gpu_lib.chamfer(x, 3, 4).contiguous()
    m = gpu_lib.precompute(t, case.sigma, scale=1.0 / 3.0)
    w, tr, done = gpu_lib.fit(m, torch.from_numpy(case.w0).cuda(), case.iters)
    torch.cuda.synchronize()
    weights = O.chamfer_transform(case.img, 3, 4) / 3.0
    W_ref, tr_ref, _, _ = O.fit_lattice(weights, case.w0, case.sigma, case.R, case.iters)
    w = w.cpu().double().numpy()
    assert float(np.linalg.norm(w - W_ref, axis=1).max()) <= 1e-3
    assert np.abs(tr.cpu().numpy() - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())
    # interior weighting pulls the codebook inward: it differs from the unweighted fit
    W_plain, _, _, _ = O.fit_lattice(case.weights, case.w0, case.sigma, case.R, case.iters)
    assert float(np.linalg.norm(W_ref - W_plain, axis=1).max()) > 0.1


def test_weighted_batched_equals_per_image(gpu_lib):
    """plan.weighted(): the chamfer-weighted batch equals the per-image weighted calls bit for bit."""
    cases = S.config3_cases(indices=range(16))
    plan = gpu_lib.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                             [c.sigma for c in cases], [c.iters for c in cases])
    t = plan.chamfer()
    wp = plan.weighted(3)
    w0 = wp.pack_codebooks([c.w0 for c in cases])
    w = torch.empty_like(w0)
    d = torch.empty(len(cases), dtype=torch.float64, device="cuda")
    wp.run(w0, w, d_out=d, weights=t)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        ti = gpu_lib.chamfer(torch.from_numpy(c.img).cuda()).contiguous()
        m = gpu_lib.precompute(ti, c.sigma, scale=1.0 / 3.0)
        wi, tr, _ = gpu_lib.fit(m, torch.from_numpy(c.w0).cuda(), c.iters)
        torch.cuda.synchronize()
        assert torch.equal(wp.unpack(w, i), wi), i
        assert float(d[i]) == float(tr[-1]), i
