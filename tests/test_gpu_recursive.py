"""Maps for large widths by recursive filtering: the HIP path against the
oracle's Young-van Vliet maps (FP64 recursions on both sides, FP32 maps), and
the fit on those maps against the oracle's lattice fit on the same maps."""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def normwise(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_rec(itc, img, sigma, scale=1.0, pitch=None):
    H, W = img.shape
    if pitch is None:
        x = torch.from_numpy(img).cuda()
    else:
        buf = torch.zeros((H, pitch), dtype=torch.from_numpy(img).dtype, device="cuda")
        buf[:, :W] = torch.from_numpy(img).cuda()
        x = buf[:, :W]
    m = itc.precompute_recursive(x, sigma, scale=scale)
    torch.cuda.synchronize()
    return m, [p.cpu().double().numpy() for p in m.planes()], float(m.s_x.cpu()[0])


CASES = [
    ("ellipses64_s2", lambda: S.config1_case(1).img, 2.0, 1.0),
    ("ellipses64_s6", lambda: S.config1_case(2).img, 6.0, 1.0),
    ("ragged70x133_s4", lambda: (np.random.default_rng(1).uniform(size=(70, 133)) < 0.3).astype(np.uint8), 4.0, 1.0),
    ("gray100x77_s12", lambda: S.gray_gaussians((7, 0), H=100, W=77, n=8, major=(5, 30)), 12.0, 1 / 255),
    ("f32_90x200_s25", lambda: np.random.default_rng(2).uniform(size=(90, 200)).astype(np.float32), 25.0, 1.0),
    ("tiny1x1_s1", lambda: np.ones((1, 1), np.uint8), 1.0, 1.0),
    ("small3x5_s0.5", lambda: np.array([[0, 1, 1, 0, 1], [1, 1, 0, 0, 1], [0, 0, 1, 1, 1]], np.uint8), 0.5, 1.0),
    ("shapes512_s40", lambda: S.config2_case(0).img, 40.0, 1.0),
]


@pytest.mark.parametrize("name,build,sigma,scale", CASES, ids=[c[0] for c in CASES])
def test_recursive_maps(gpu_lib, name, build, sigma, scale):
    img = build()
    m, got, sx = gpu_rec(gpu_lib, img, sigma, scale)
    A, Mu, Mv, sx_ref = O.recursive_maps(img.astype(np.float64) * scale, sigma)
    for g, r in zip(got, (A, Mu, Mv)):
        assert normwise(g, r) <= 1e-6
    assert sx == pytest.approx(sx_ref, rel=1e-6)
    # columns past the width inside the last map panel are written as zero
    H, W = img.shape
    full = (W + 15) // 16 * 16
    if full > W:
        n = gpu_lib.plane_elems(m.desc)
        flat = m.buf[: 3 * n * 4].view(torch.float32)
        for i in range(3):
            assert torch.all(gpu_lib.panel_view(flat[i * n:(i + 1) * n], H, full)[:, W:] == 0)


def test_recursive_pitch(gpu_lib):
    img = (np.random.default_rng(3).uniform(size=(45, 70)) < 0.4).astype(np.uint8)
    _, got, _ = gpu_rec(gpu_lib, img, 5.0, pitch=128)
    A, Mu, Mv, _ = O.recursive_maps(img.astype(np.float64), 5.0)
    for g, r in zip(got, (A, Mu, Mv)):
        assert normwise(g, r) <= 1e-6


def test_fit_on_recursive_maps(gpu_lib):
    """512 x 512 shapes, M = 100, sigma = 16 (beyond the masks' radius limit).

    At this width the sweeps amplify any perturbation by about 1.15 per sweep
    (the oracle's own codebook moves by 2e-6 px after 10 sweeps and 2e-4 px
    after 40 when only its maps are rounded to FP32), so the codebook is
    compared after one sweep and after 10, with the bars of the mask path;
    D is compared over 40 sweeps."""
    case = S.config2_case(0)
    sigma = 16.0
    m, _, _ = gpu_rec(gpu_lib, case.img, sigma)
    A, Mu, Mv, _ = O.recursive_maps(case.weights, sigma)
    U, V = np.meshgrid(np.arange(512.0), np.arange(512.0), indexing="ij")
    maps = (A, U * A - Mu, V * A - Mv)  # the oracle reads B = x A - M
    for sweeps, bar in ((1, 1e-4), (10, 1e-3)):
        w, _, _ = gpu_lib.fit(m, torch.from_numpy(case.w0).cuda(), sweeps)
        torch.cuda.synchronize()
        W_ref, _, _, _ = O.fit_lattice(case.weights, case.w0, sigma, 0, sweeps, maps=maps)
        assert float(np.linalg.norm(w.cpu().double().numpy() - W_ref, axis=1).max()) <= bar
    _, tr, _ = gpu_lib.fit(m, torch.from_numpy(case.w0).cuda(), 40)
    _, tr_ref, _, _ = O.fit_lattice(case.weights, case.w0, sigma, 0, 40, maps=maps)
    assert np.abs(tr.cpu().numpy() - tr_ref).max() <= 1e-5 * max(1.0, abs(tr_ref).max())


def test_recursive_rejects(gpu_lib):
    x = torch.ones((8, 8), dtype=torch.uint8, device="cuda")
    with pytest.raises(gpu_lib.ItcError):
        gpu_lib.precompute_recursive(x, 0.3)
