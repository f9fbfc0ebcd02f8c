"""The allocation-free Algorithm 1 entry point (static work array) against the
entry point with a caller work buffer: the same kernels, so results must be
equal bit for bit. Two calls in a row on one GPU, the second on a smaller
image (the array keeps the first call's contents), and a problem larger than
the array rejected on the host."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
from paper_1310_7114_amd import synth as S

pytestmark = pytest.mark.gpu


def test_noalloc_equals_work_buffer_entry_point(gpu_lib):
    for case, iters in ((S.config2_case(0), 6), (S.config1_case(1), 12)):  # 512 x 512, then 64 x 64
        x = torch.from_numpy(case.img).cuda()
        w0 = torch.from_numpy(np.asarray(case.w0)).cuda().to(torch.int32)
        xi, om = O.paper_widths(float(case.img.sum()), case.M)
        wa, ta, da = gpu_lib.fit_literal(x, w0, xi, om, iters, scale=case.scale)
        wb, tb, db = gpu_lib.fit_literal_noalloc(x, w0, xi, om, iters, scale=case.scale)
        torch.cuda.synchronize()
        assert torch.equal(wa, wb), case.name
        assert torch.equal(ta, tb) and torch.equal(da, db), case.name
        assert int(db[0]) == iters


def test_noalloc_theta_stop_equals(gpu_lib):
    case = S.config1_case(2)
    x = torch.from_numpy(case.img).cuda()
    w0 = torch.from_numpy(np.asarray(case.w0)).cuda().to(torch.int32)
    wa, ta, da = gpu_lib.fit_literal(x, w0, 2.0, 2.0, 100, theta=0.5)
    wb, tb, db = gpu_lib.fit_literal_noalloc(x, w0, 2.0, 2.0, 100, theta=0.5)
    torch.cuda.synchronize()
    assert torch.equal(wa, wb) and int(da[0]) == int(db[0]) < 100
    n = int(da[0]) + 1
    assert torch.equal(ta[:n], tb[:n])


def test_noalloc_rejects_a_problem_beyond_the_array(gpu_lib):
    lib = gpu_lib.load()
    x = torch.zeros((8, 8), dtype=torch.uint8, device="cuda")
    w0 = torch.zeros((4, 2), dtype=torch.int32, device="cuda")
    wo = torch.empty_like(w0)
    d = gpu_lib.make_desc(4096, 4096, 2.0, torch.uint8, torch.float32, 1.0, 0)  # maps alone exceed 64 MiB
    assert lib.itc_lattice_literal_work_bytes(ctypes.byref(d), 4, 4.0, 0) > (64 << 20)
    st = lib.itc_lattice_literal_fit_noalloc(ctypes.byref(d), gpu_lib._ptr(x), 4.0, 0, 4, gpu_lib._ptr(w0), 1, -1.0,
                                             gpu_lib._ptr(wo), None, None, None)
    assert st == 3 and b"work memory" in lib.itc_last_error()
