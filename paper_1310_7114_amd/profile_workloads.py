"""Workloads launched once each (no graphs), for rocprofv3 kernel traces and
counter runs that ``profsummary`` turns into the summaries under ``profiles/``.

    python3 -m paper_1310_7114_amd.profile_workloads differentiation [--copy-calib-mib 1024]
    python3 -m paper_1310_7114_amd.profile_workloads gray2048 [--copy-calib-mib 1024]

* differentiation: 64 weighted 1024 x 1024 gray images (weights g/255 as
  FP32, M 256, sigma 4): the convolution (vector-ALU kernel, FP32 weights),
  D at the initial codebooks, dD/dw and dD/dh.
* gray2048: the 2048 x 2048 gray image (M 500, sigma 6): its maps and 200
  sweeps of the multi-workgroup fit.

With --copy-calib-mib N a plain device copy of N MiB runs first, so that the
HBM byte counters can be scaled by what they read for a copy of known size.
"""
from __future__ import annotations

import argparse
import sys

import torch

from . import itc, synth


def differentiation(dev):
    cases = synth.config5_cases(64)
    B, H, W, M = len(cases), 1024, 1024, 256
    plan = itc.BatchPlan.for_stack(B, H, W, M, 4.0, iters=0, dtype=torch.float32, device=dev)
    h = torch.stack([torch.from_numpy(c.img) for c in cases]).to(dev).float() / 255.0
    w = torch.cat([torch.from_numpy(c.w0) for c in cases]).to(dev, torch.float32)
    maps = plan.new_maps()
    w_out = torch.empty_like(w)
    s_x = torch.empty(B, dtype=torch.float64, device=dev)
    d = torch.empty(B, dtype=torch.float64, device=dev)
    grad_d = torch.ones(B, dtype=torch.float64, device=dev)
    grad_w = torch.empty_like(w)
    grad_h = torch.empty((B, H, W), dtype=torch.float32, device=dev)
    for _ in range(2):
        plan.precompute(weights=h, maps=maps)
        plan.fit(w, w_out, s_x=s_x, d_out=d, maps=maps)
        plan.backward(w, s_x, grad_d, grad_w=grad_w, maps=maps)
        plan.backward(w, s_x, grad_d, grad_weights=grad_h, maps=maps)
    torch.cuda.synchronize()
    print(f"differentiation: 2 passes over {B} images, D[0] = {float(d[0]):.6f}", flush=True)


def gray2048(dev):
    c = synth.config4_case(0)
    img = torch.from_numpy(c.img).to(dev)
    w0 = torch.from_numpy(c.w0).to(dev, torch.float32)
    work = torch.empty(itc.fit_wide_work_bytes(c.M), dtype=torch.uint8, device=dev)
    for _ in range(2):
        maps = itc.precompute(img, c.sigma, scale=c.scale)
        w, _, done = itc.fit_wide(maps, w0, c.iters, work=work)
    torch.cuda.synchronize()
    print(f"gray2048: {int(done[0])} sweeps", flush=True)


WORKLOADS = {"differentiation": differentiation, "gray2048": gray2048}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=sorted(WORKLOADS))
    ap.add_argument("--copy-calib-mib", type=int, default=0)
    a = ap.parse_args(argv)
    itc.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if a.copy_calib_mib > 0:
        src = torch.ones(a.copy_calib_mib * (1 << 20) // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    WORKLOADS[a.workload](dev)
    return 0


if __name__ == "__main__":
    sys.exit(main())
