"""Segments (nearest codevector per foreground pixel) on the GPU vs the oracle: exact labels."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def gpu_label(itc, img, W, scale=1.0, real=torch.float32):
    x = torch.from_numpy(img).cuda()
    lab = itc.label(x, torch.from_numpy(np.asarray(W)).cuda(), scale=scale, real_dtype=real)
    torch.cuda.synchronize()
    return lab.cpu().numpy()


@pytest.mark.parametrize("idx", [0, 5, 11])
def test_silhouettes(gpu_lib, idx):
    c = S.config3_cases(indices=[idx])[0]
    W = (c.w0 + np.random.default_rng(idx).uniform(-0.5, 0.5, c.w0.shape)).astype(np.float32).astype(np.float64)
    assert np.array_equal(gpu_label(gpu_lib, c.img, W), O.label_pixels(c.img, W))


def test_fp64_codebook_and_gray_weights(gpu_lib):
    c = S.config1_case(2)
    W = c.w0 + np.random.default_rng(3).uniform(-0.5, 0.5, c.w0.shape)
    assert np.array_equal(gpu_label(gpu_lib, c.img, W, real=torch.float64), O.label_pixels(c.img, W))
    g = S.gray_gaussians((7, 3), H=120, W=90, n=5, major=(8, 20))
    Wg = np.random.default_rng(4).uniform(0, 90, (40, 2)).astype(np.float32).astype(np.float64)
    assert np.array_equal(gpu_label(gpu_lib, g, Wg, scale=1 / 255), O.label_pixels(g, Wg))


def test_ties_and_max_codebook(gpu_lib):
    I = np.ones((5, 5), np.uint8)
    W = np.array([[2.0, 4.0], [2.0, 0.0], [2.0, 0.0]])
    assert np.array_equal(gpu_label(gpu_lib, I, W), O.label_pixels(I, W))
    img = (np.random.default_rng(5).uniform(size=(40, 50)) < 0.8).astype(np.uint8)
    Wm = np.random.default_rng(6).integers(0, 50, (1024, 2)).astype(np.float64)  # many exact ties
    assert np.array_equal(gpu_label(gpu_lib, img, Wm), O.label_pixels(img, Wm))


def test_batched_segments(gpu_lib):
    """Fitted codebooks of 32 silhouettes: batched labels equal per-image labels; two against the oracle."""
    cases = S.config3_cases(indices=range(32))
    plan = gpu_lib.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                             [c.sigma for c in cases], [c.iters for c in cases])
    w0 = plan.pack_codebooks([c.w0 for c in cases])
    w = torch.empty_like(w0)
    plan.run(w0, w)
    lab = plan.label(w)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        li = plan.image(lab, i)
        assert torch.equal(li, gpu_lib.label(torch.from_numpy(c.img).cuda(), plan.unpack(w, i))), i
    for i in (0, 9):
        got = plan.image(lab, i).cpu().numpy()
        Wi = plan.unpack(w, i).cpu().double().numpy()
        assert np.array_equal(got, O.label_pixels(cases[i].img, Wi)), i


def test_full_batch_segments(gpu_lib):
    """All 1,400 silhouettes with their fitted codebooks (the batch the benchmark labels): every image labels
    exactly its foreground with indices below M; the tallest, the widest, the largest codebook and every 97th
    image equal the per-image labels bit for bit; the three smallest and a median-sized image against the
    oracle."""
    cases = S.config3_cases(1400)
    plan = gpu_lib.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                             [c.sigma for c in cases], [c.iters for c in cases])
    w0 = plan.pack_codebooks([c.w0 for c in cases])
    w = torch.empty_like(w0)
    plan.run(w0, w)
    lab = plan.label(w)
    torch.cuda.synchronize()
    for i, c in enumerate(cases):
        li = plan.image(lab, i)
        fg = torch.from_numpy(c.img).cuda() > 0
        assert torch.equal(li >= 0, fg), i
        assert int(li.max()) < c.M, i
    shapes = [c.img.shape for c in cases]
    sizes = [h * w_ for h, w_ in shapes]
    pick = {int(np.argmax([h for h, _ in shapes])), int(np.argmax([w_ for _, w_ in shapes])),
            int(np.argmax([c.M for c in cases]))} | set(range(0, 1400, 97))
    for i in sorted(pick):
        ref = gpu_lib.label(torch.from_numpy(cases[i].img).cuda(), plan.unpack(w, i))
        assert torch.equal(plan.image(lab, i), ref), i
    order = np.argsort(sizes, kind="stable")
    for i in list(order[:3]) + [int(order[len(order) // 2])]:
        got = plan.image(lab, int(i)).cpu().numpy()
        Wi = plan.unpack(w, int(i)).cpu().double().numpy()
        assert np.array_equal(got, O.label_pixels(cases[int(i)].img, Wi)), int(i)
