"""Adjoint kernels (dD/dw, dD/dh) vs the oracle's analytic gradient and FP64
finite differences; batched == single image; the torch.autograd op.

Tolerance: normwise max|gpu - ref| / max|ref| <= 1e-4 (FP32), 1e-10 (FP64).
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fd_config5.json")


def normwise(got, ref):
    return float(np.abs(np.asarray(got) - ref).max() / max(np.abs(ref).max(), 1e-300))


def small_case(seed, H=150, W=170, M=20, sigma=2.5):
    img = S.gray_gaussians((55, seed), H=H, W=W, n=12, major=(5.0, 30.0))
    w0 = S.sample_init(img, M, (55, seed, 1), jitter=(0.05, 0.95))
    return img.astype(np.float64) / 255.0, w0, sigma, S.radius_for(sigma)


def gpu_backward(itc, I, w0, sigma, real=torch.float32, gd=1.0):
    t = torch.from_numpy(I).to("cuda", real)
    m = itc.precompute(t, sigma, real_dtype=real)
    w = torch.from_numpy(w0).to("cuda", real)
    g = torch.tensor([gd], dtype=torch.float64, device="cuda")
    gw, gI = itc.divergence_backward(m, w, g)
    d = itc.divergence(m, w)
    torch.cuda.synchronize()
    return gw.cpu().double().numpy(), gI.cpu().double().numpy(), float(d.cpu()[0])


@pytest.mark.parametrize("seed", [0, 1])
def test_backward_matches_oracle_fp32(gpu_lib, seed):
    I, w0, sigma, R = small_case(seed)
    gw, gI, d = gpu_backward(gpu_lib, I, w0, sigma, gd=0.7)
    A = O.density_map(I, sigma, R)
    rw, rI = O.lattice_grad(I, (A,), w0, sigma, R)
    assert normwise(gw, 0.7 * rw) <= 1e-4
    assert normwise(gI, 0.7 * rI) <= 1e-4
    assert d == pytest.approx(O.lattice_divergence(I, (A,), w0, sigma), rel=1e-5)


def test_backward_matches_oracle_fp64(gpu_lib):
    I, w0, sigma, R = small_case(2, H=90, W=77, M=12, sigma=2.0)
    gw, gI, _ = gpu_backward(gpu_lib, I, w0, sigma, real=torch.float64)
    rw, rI = O.lattice_grad(I, (O.density_map(I, sigma, R),), w0, sigma, R)
    assert normwise(gw, rw) <= 1e-10
    assert normwise(gI, rI) <= 1e-10


def test_backward_edge_codevectors(gpu_lib):
    """Codevectors on the border, one off the lattice (no data: zero slope), one on a corner."""
    I, w0, sigma, R = small_case(3, H=70, W=90, M=10, sigma=2.0)
    w0 = w0.copy()
    w0[0] = [-0.4, 10.3]      # half off the top edge
    w0[1] = [68.6, 88.7]      # past the last row and column centres
    w0[2] = [-50.0, -50.0]    # far off the lattice
    gw, gI, _ = gpu_backward(gpu_lib, I, w0, sigma)
    rw, rI = O.lattice_grad(I, (O.density_map(I, sigma, R),), w0, sigma, R)
    assert normwise(gw, rw) <= 1e-4
    assert normwise(gI, rI) <= 1e-4


def test_batched_backward_equals_single(gpu_lib):
    itc = gpu_lib
    cases = [small_case(10 + i, H=128, W=160, M=24, sigma=4.0) for i in range(3)]
    B, H, W, M = 3, 128, 160, 24
    plan = itc.BatchPlan.for_stack(B, H, W, M, 4.0, iters=0)
    h = torch.from_numpy(np.stack([c[0] for c in cases])).to("cuda", torch.float32)
    w = torch.from_numpy(np.concatenate([c[1] for c in cases])).to("cuda", torch.float32)
    maps = plan.new_maps()
    sx = torch.empty(B, dtype=torch.float64, device="cuda")
    d = torch.empty(B, dtype=torch.float64, device="cuda")
    plan.precompute(weights=h, maps=maps)
    plan.fit(w, torch.empty_like(w), s_x=sx, d_out=d, maps=maps)
    gd = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda")
    gw = torch.empty_like(w)
    gh = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    plan.backward(w, sx, gd, grad_w=gw, grad_weights=gh, maps=maps)
    torch.cuda.synchronize()
    for i in range(B):
        m = itc.precompute(h[i], 4.0)
        gwi, ghi = itc.divergence_backward(m, w[i * M:(i + 1) * M], gd[i:i + 1])
        torch.cuda.synchronize()
        assert torch.equal(gwi, gw[i * M:(i + 1) * M])
        assert torch.equal(ghi, gh[i])
        assert float(sx[i]) == float(m.s_x[0])


def test_autograd_function(gpu_lib):
    from paper_1310_7114_amd.autograd import divergence
    cases = [small_case(20 + i, H=96, W=80, M=16, sigma=2.0) for i in range(2)]
    h = torch.from_numpy(np.stack([c[0] for c in cases])).to("cuda", torch.float32).requires_grad_(True)
    w = torch.from_numpy(np.stack([c[1] for c in cases])).to("cuda", torch.float32).requires_grad_(True)
    D = divergence(h, w, 2.0)
    coef = torch.tensor([0.3, -1.1], dtype=torch.float64, device="cuda")
    (D * coef).sum().backward()
    torch.cuda.synchronize()
    for i, (I, w0, sigma, R) in enumerate(cases):
        A = O.density_map(I, sigma, R)
        assert float(D.detach()[i]) == pytest.approx(O.lattice_divergence(I, (A,), w0, sigma), rel=1e-5)
        rw, rI = O.lattice_grad(I, (A,), w0, sigma, R)
        assert normwise(w.grad[i].cpu().double().numpy(), float(coef[i]) * rw) <= 1e-4
        assert normwise(h.grad[i].cpu().double().numpy(), float(coef[i]) * rI) <= 1e-4
    # single image form
    h1 = h.detach()[0].clone().requires_grad_(True)
    w1 = w.detach()[0].clone().requires_grad_(True)
    d1 = divergence(h1, w1, 2.0)
    d1.backward()
    assert d1.dim() == 0 and h1.grad.shape == h1.shape and w1.grad.shape == w1.shape


def test_config5_full_batch(gpu_lib):
    """64 x 1024 x 1024 gray weights (g/255), M = 256, sigma = 4: forward D and the adjoint for
    the whole batch in the batched launch; images 0 and 1 checked against the oracle's analytic
    gradient over the whole image and against FP64 finite differences on a 32 x 32 crop."""
    from paper_1310_7114_amd.autograd import divergence
    cases = S.config5_cases()
    h = torch.stack([torch.from_numpy(c.img) for c in cases]).to("cuda", torch.float32).mul_(1.0 / 255.0)
    h.requires_grad_(True)
    w = torch.from_numpy(np.stack([c.w0 for c in cases])).to("cuda", torch.float32).requires_grad_(True)
    D = divergence(h, w, 4.0)
    D.sum().backward()
    torch.cuda.synchronize()
    assert torch.all(torch.isfinite(D)) and torch.all(torch.isfinite(h.grad)) and torch.all(torch.isfinite(w.grad))
    golden = json.load(open(GOLDEN))["cases"]
    for i in (0, 1):
        c = cases[i]
        I = h.detach()[i].cpu().double().numpy()   # the FP32 weights the GPU saw
        A = O.density_map(I, c.sigma, c.R)
        rw, rI = O.lattice_grad(I, (A,), c.w0.astype(np.float32).astype(np.float64), c.sigma, c.R)
        gI = h.grad[i].cpu().double().numpy()
        gw = w.grad[i].cpu().double().numpy()
        assert normwise(gw, rw) <= 1e-4
        assert normwise(gI, rI) <= 1e-4
        g = golden[i]
        u0, u1 = g["crop"]
        assert normwise(gI[u0:u1, u0:u1], np.array(g["grad_weights_crop"])) <= 1e-4
        assert normwise(gw[:len(g["grad_w_first"])], np.array(g["grad_w_first"])) <= 1e-4
        assert float(D.detach()[i]) == pytest.approx(g["D"], rel=1e-5)
