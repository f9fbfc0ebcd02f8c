"""Benchmark: images/s to the converged codebook, batched vs per-image, with the
fit's and the convolution's rooflines and the FP64 oracle timed beside it.

Default workload: the batch of 1,400 star silhouettes (W 128..1024 x H 128..768,
binary uint8, M in 10..200, sigma in {2, 4, 8}, 100 sweeps, FP32), inputs
resident in HBM. One step = batched convolution maps of every image + fit of
every image + D at its final codebook, replayed from a HIP graph.

Prints one JSON line (rank 0). Runs on one GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "images/sec to converged codebook (batched vs per-image); conv HBM GB/s vs peak"
HBM_PEAK_GBS = 8000.0
# Convolution: algorithmic bytes per pixel, 1 B of 8-bit weight in and 3 x 4 B of FP32 maps out.
CONV_BYTES_PER_PX = 13.0
# Fit: algorithmic work per unordered codebook pair of a sweep (the M(M-1)/2 distinct pairs):
# 2 differences, |d|^2 (mul + fma), one exp2, C_k and C_j (2 adds), E_k and E_j (4 fmas) = 16 flop
# in 10 FP32 VALU instructions and one transcendental. Its ceiling comes from the issue rates a probe
# kernel measures on the chip, in SIMD cycles per wave64 instruction: unpacked FP32 3.1 (the build
# disables packed FP32), v_exp_f32 9.8; 256 CUs x 4 SIMDs at 2.4 GHz.
FIT_FLOPS_PER_PAIR = 16.0
FIT_VALU_PER_PAIR, FIT_VALU_CYCLES, FIT_EXP_CYCLES = 10, 3.1, 9.8
FIT_PEAK_PAIRS_PER_S = 1024 * 2.4e9 * 64.0 / (FIT_VALU_PER_PAIR * FIT_VALU_CYCLES + FIT_EXP_CYCLES)


def profile_figures(group: str):
    """Key/value figures of a committed rocprofv3 summary (profiles/<group>.md), or None when the
    kernel sources no longer hash to the value recorded with the counters."""
    path = os.path.join(ROOT, "profiles", f"{group}.md")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        line = line.strip()
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k] = v
    try:
        h = hashlib.sha256()
        for f in kv["source_files"].split():
            with open(os.path.join(ROOT, f), "rb") as fh:
                h.update(fh.read())
        if h.hexdigest() != kv["source_sha256"]:
            return None
        return {k: float(kv[k]) for k in ("traffic_bytes_per_step", "average_us_per_step")}
    except (KeyError, OSError, ValueError):
        return None


def paper_widths(N: float, M: int):
    """(xi, omega) of the paper's runtime experiments (Section 4): omega = sqrt(N/M)/2, xi = omega/2."""
    omega = (float(N) / M) ** 0.5 / 2.0
    return omega / 2.0, omega


def _pool_init():
    from threadpoolctl import threadpool_limits
    threadpool_limits(limits=1)


def _oracle_fit(args):
    import oracle as O
    weights, w0, sigma, R, iters = args
    O.fit_lattice(weights, w0, sigma, R, iters)
    return 1


def synth_config2():
    from paper_1310_7114_amd import synth
    return synth.config2_case(0)


def cpu_legs(cases, seconds):
    """The FP64 oracle on the host cores, run before the GPU is touched: the
    lattice variant on one core (the reported baseline) and on every core of
    the process's affinity set, and one sweep of the original point-set
    update beside one lattice sweep on a sample stratified by N*M."""
    import multiprocessing as mp
    import numpy as np
    import oracle as O
    from threadpoolctl import threadpool_limits

    n = len(cases)
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        k = 0
        while k < n and time.perf_counter() - t < seconds:
            c = cases[k]
            O.fit_lattice(c.weights, c.w0, c.sigma, c.R, c.iters)
            k += 1
        el = time.perf_counter() - t
    cpu = {"value": k / el, "unit": "images/s", "cores": 1, "kind": "oracle",
           "sample": f"first {k} of the {n} silhouettes (same sizes, M, sigma, 100 sweeps), "
                     f"FP64 NumPy lattice variant, {el:.1f}s"}
    print(f"[bench] oracle on one core: {k} images in {el:.1f}s", file=sys.stderr, flush=True)

    ctx = {"cpu_model": None, "cores_available": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                ctx["cpu_model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    P = ctx["cores_available"]
    with mp.get_context("fork").Pool(P, initializer=_pool_init) as pool:
        t = time.perf_counter()
        k2 = 0
        while k2 < n and time.perf_counter() - t < seconds / 2:
            idx = range(k2, min(n, k2 + P))
            pool.map(_oracle_fit, [(cases[i].weights, cases[i].w0, cases[i].sigma, cases[i].R, cases[i].iters)
                                   for i in idx])
            k2 += len(idx)
        el2 = time.perf_counter() - t
    ctx["lattice_all_cores"] = {"value": k2 / el2, "unit": "images/s", "cores": P,
                                "sample": f"first {k2} silhouettes, one image per process, {el2:.1f}s"}
    print(f"[bench] oracle on {P} cores: {k2} images in {el2:.1f}s", file=sys.stderr, flush=True)

    # original eq. (4) over the point set vs the lattice sweep, one sweep each
    npts = np.array([int(np.count_nonzero(c.img)) * c.M for c in cases], dtype=np.float64)
    order = np.argsort(npts, kind="stable")
    strata = [int(order[int((i + 0.5) * n / 14)]) for i in range(14)] if n >= 14 else list(range(n))
    t_orig = t_lat = 0.0
    done = 0
    with threadpool_limits(limits=1):
        t_all = time.perf_counter()
        for i in strata:
            if time.perf_counter() - t_all > seconds:
                break
            c = cases[i]
            X = np.argwhere(c.img > 0).astype(np.float64)
            h = c.weights[c.img > 0]
            xi, om = O.widths(c.sigma)
            t = time.perf_counter()
            O.original_step(X, h, c.w0, xi, om)
            t_orig += time.perf_counter() - t
            maps = O.lattice_maps(c.weights, c.sigma, c.R)
            t = time.perf_counter()
            O.lattice_step(maps, c.w0, c.sigma)
            t_lat += time.perf_counter() - t
            done += 1
    ctx["original_vs_lattice_sweep"] = {
        "images": done, "stratified_by": "on-pixels x M",
        "original_s_per_sweep": t_orig / max(done, 1), "lattice_s_per_sweep": t_lat / max(done, 1),
        "ratio": t_orig / t_lat if t_lat > 0 else None,
        "original_images_per_s_extrapolated_100_sweeps": done / (100.0 * t_orig) if t_orig > 0 else None}
    # Algorithm 1 (eq. (6) on the lattice): one oracle sweep on the 512 x 512
    # shapes with the paper's widths
    c2 = synth_config2()
    xi2, om2 = O.paper_widths(float(c2.img.sum()), c2.M)
    P2 = O.density_map(c2.weights, xi2, int(np.ceil(3 * xi2 - 1e-12)))
    t = time.perf_counter()
    O.literal_step(P2, c2.w0, om2, int(np.ceil(3 * om2 - 1e-12)))
    ctx["literal_shapes512_sweep_s"] = time.perf_counter() - t
    # recursive maps (large widths): the oracle on the 512 x 512 shapes at sigma = 16
    t = time.perf_counter()
    O.recursive_maps(c2.weights, 16.0)
    ctx["recursive_maps_shapes512_s16_s"] = time.perf_counter() - t

    # 3-D lattice: the oracle's maps and fit on a 48 x 56 x 64 volume (M = 24, 30 sweeps)
    from paper_1310_7114_amd import synth as _s
    vc = _s.volume_case(0)
    t = time.perf_counter()
    O.fit_volume(vc.weights, vc.w0, vc.sigma, vc.R, vc.iters)
    ctx["volume_48x56x64_fit_s"] = time.perf_counter() - t

    # Section 5: the oracle's two-pass chamfer transform on the first silhouettes
    t = time.perf_counter()
    k3, px3 = 0, 0
    while k3 < n and time.perf_counter() - t < seconds / 5:
        O.chamfer_transform(cases[k3].img, 3, 4)
        px3 += cases[k3].img.size
        k3 += 1
    el3 = time.perf_counter() - t
    ctx["chamfer_oracle"] = {"images": k3, "pixels_per_s": px3 / el3, "cores": 1}
    return cpu, ctx


def capture(fn, dev="cuda"):
    """fn captured in a HIP graph, after one warm-up call on a side stream."""
    import torch

    side = torch.cuda.Stream(device=dev)
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        fn()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fn()
    return g


def gpu_extras(dev, cases, itc, synth):
    """Secondary measurements: device copy and fill rates, the convolution per
    sigma class of the silhouette batch, the single-image workloads (512^2 and
    2048^2) end to end, differentiation of the 64-image 1024^2 batch, the
    theta stop, and the convolution of the 64-image 1024^2 batch."""
    import numpy as np
    import torch

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps / 1e3

    out = {}
    nb = 1 << 30
    a = torch.ones(nb // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    t = timed(lambda: b.copy_(a))
    out["copy_gbs"] = 2.0 * nb / t / 1e9
    t = timed(lambda: a.fill_(0.5))
    out["fill_gbs"] = nb / t / 1e9
    del a, b

    def mx_flops_per_px(R):
        ra = (R + 7) // 8 * 8
        k = (16 + 2 * ra + 31) // 32 * 32
        return 16.0 * (k // 32) * 16384.0 / 256.0

    classes = []
    for sigma in sorted({c.sigma for c in cases}):
        sub = [c for c in cases if c.sigma == sigma]
        p = itc.BatchPlan([torch.from_numpy(c.img) for c in sub], [c.M for c in sub], [c.sigma for c in sub],
                          [c.iters for c in sub], device=dev)
        t = timed(p.precompute)
        px = float(sum(c.img.size for c in sub))
        gbs = 13.0 * px / t / 1e9
        classes.append({"sigma": sigma, "R": sub[0].R, "images": len(sub), "pixels": int(px), "ms": t * 1e3,
                        "gbs": gbs, "frac_hbm_peak": gbs / HBM_PEAK_GBS, "frac_copy": gbs / out["copy_gbs"],
                        "mfma_tflops": mx_flops_per_px(sub[0].R) * px / t / 1e12})
        del p
    out["conv_per_sigma"] = classes

    singles = []
    lib = itc.load()
    for c in (synth.config2_case(0), synth.config4_case(0)):
        img = torch.from_numpy(c.img).to(dev)
        maps = itc.precompute(img, c.sigma, scale=c.scale)
        w0 = torch.from_numpy(c.w0).to(dev, torch.float32)
        wout = torch.empty_like(w0)
        dtr = torch.empty(c.iters + 1, dtype=torch.float64, device=dev)
        dn = torch.empty(1, dtype=torch.int32, device=dev)
        work = torch.empty(itc.fit_wide_work_bytes(c.M), dtype=torch.uint8, device=dev)

        def conv():
            itc.precompute(img, c.sigma, scale=c.scale, out=maps)

        def run_one():   # Algorithm 1's loop in one workgroup
            conv()
            itc._check(lib.itc_lattice_fit(itc.ctypes.byref(maps.desc), itc._ptr(maps.buf), itc._ptr(maps.s_x),
                                           c.M, itc._ptr(w0), c.iters, -1.0, itc._ptr(wout), itc._ptr(dtr),
                                           itc._ptr(dn), itc._stream()))

        def run_wide():  # one launch per sweep over M / 32 workgroups
            conv()
            itc._check(lib.itc_lattice_fit_wide(itc.ctypes.byref(maps.desc), itc._ptr(maps.buf),
                                                itc._ptr(maps.s_x), c.M, itc._ptr(w0), c.iters, -1.0,
                                                itc._ptr(wout), itc._ptr(dtr), itc._ptr(dn), itc._ptr(work),
                                                work.numel(), itc._stream()))

        t_conv, t_one, t_wide = (timed(capture(fn).replay) for fn in (conv, run_one, run_wide))
        singles.append({"workload": c.name, "H": int(c.img.shape[0]), "W": int(c.img.shape[1]), "M": c.M,
                        "sigma": c.sigma, "sweeps": c.iters, "conv_ms": t_conv * 1e3,
                        "conv_gbs": 13.0 * c.img.size / t_conv / 1e9,
                        "one_workgroup": {"ms": t_one * 1e3, "images_per_s": 1.0 / t_one},
                        "wide": {"ms": t_wide * 1e3, "images_per_s": 1.0 / t_wide,
                                 "us_per_sweep": (t_wide - t_conv) / (c.iters + 2) * 1e6}})
        del maps
    out["single_image"] = singles

    # Section 5 weighting: chamfer transform of every silhouette, then the
    # fit of the chamfer-weighted batch (weights T/3, FP32 convolution)
    pu8 = itc.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                        [c.sigma for c in cases], [c.iters for c in cases], device=dev)
    tch = pu8.chamfer()
    t_ch = timed(lambda: pu8.chamfer(out=tch))
    pw = pu8.weighted(3)
    w0w = pw.pack_codebooks([c.w0 for c in cases], device=dev)
    ww = torch.empty_like(w0w)
    t_wrun = timed(lambda: pw.run(w0w, ww, weights=tch), reps=3)
    npx_all = float(sum(c.img.size for c in cases))
    out["chamfer_silhouettes"] = {"images": len(cases), "pixels": int(npx_all), "ms": t_ch * 1e3,
                                  "gpx_per_s": npx_all / t_ch / 1e9,
                                  "gbs_algorithmic": 5.0 * npx_all / t_ch / 1e9, "bytes_per_px": 5,
                                  "weighted_fit_ms": t_wrun * 1e3,
                                  "weighted_images_per_s": len(cases) / (t_ch + t_wrun)}
    # segments of every silhouette for its fitted codebook (nearest codevector per pixel)
    w0s = pu8.pack_codebooks([c.w0 for c in cases], device=dev)
    wfit = torch.empty_like(w0s)
    pu8.run(w0s, wfit)
    lab = pu8.label(wfit)
    t_lab = timed(lambda: pu8.label(wfit, out=lab))
    out["segments_silhouettes"] = {"images": len(cases), "pixels": int(npx_all), "ms": t_lab * 1e3,
                                   "gpx_per_s": npx_all / t_lab / 1e9}
    del pu8, pw, tch, lab

    # Algorithm 1 as printed (eq. (6), lattice codevectors) on the 512 x 512
    # shapes with the paper's widths: time per sweep (the paper's Fig. 4 metric)
    c2 = synth.config2_case(0)
    xi2, om2 = paper_widths(float(c2.img.sum()), c2.M)
    x2 = torch.from_numpy(c2.img).to(dev)
    w02 = torch.from_numpy(c2.w0).to(dev).to(torch.int32)
    work = torch.empty(1 << 26, dtype=torch.uint8, device=dev)
    t20 = timed(lambda: itc.fit_literal(x2, w02, xi2, om2, 20, work=work), reps=3)
    t0 = timed(lambda: itc.fit_literal(x2, w02, xi2, om2, 0, work=work), reps=3)
    # the same calls replayed from HIP graphs (no host enqueue cost per launch)
    graphs = {}
    for k in (20, 0):
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side):
            itc.fit_literal(x2, w02, xi2, om2, k, work=work)
        torch.cuda.current_stream().wait_stream(side)
        torch.cuda.synchronize()
        graphs[k] = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graphs[k]):
            itc.fit_literal(x2, w02, xi2, om2, k, work=work)
    g20 = timed(graphs[20].replay, reps=5)
    g0 = timed(graphs[0].replay, reps=5)
    out["literal_shapes512"] = {"xi": xi2, "omega": om2, "M": c2.M, "sweeps": 20, "ms_total": t20 * 1e3,
                                "ms_per_sweep": (t20 - t0) / 20 * 1e3, "ms_setup": t0 * 1e3,
                                "graph_ms_total": g20 * 1e3, "graph_ms_per_sweep": (g20 - g0) / 20 * 1e3}
    del work, graphs

    # Algorithm 1 with the paper's widths where xi exceeds the masks: P by
    # recursive filtering once, then the sweeps (silhouette 49 of the batch)
    c49 = synth.config3_cases(indices=[49])[0]
    xi49, om49 = paper_widths(float(c49.img.sum()), c49.M)
    x49 = torch.from_numpy(c49.img).to(dev)
    w049 = torch.from_numpy(c49.w0).to(dev).to(torch.int32)
    m49 = itc.precompute_recursive(x49, xi49)
    t_p = timed(lambda: itc.precompute_recursive(x49, xi49))
    g_lit = {k: capture(lambda k=k: itc.fit_literal_density(m49, w049, om49, k, trace=False)) for k in (20, 0)}
    t20, t0 = timed(g_lit[20].replay, reps=5), timed(g_lit[0].replay, reps=5)
    out["literal_recursive_silhouette"] = {"index": 49, "H": int(c49.img.shape[0]), "W": int(c49.img.shape[1]),
                                           "M": c49.M, "xi": xi49, "omega": om49, "p_ms": t_p * 1e3,
                                           "ms_per_sweep": (t20 - t0) / 20 * 1e3}
    del m49, g_lit

    # maps by recursive filtering: cost per pixel independent of sigma
    c4 = synth.config4_case(0)
    x4 = torch.from_numpy(c4.img).to(dev)
    recs = []
    for sig in (4.0, 16.0, 40.0):
        t_r = timed(lambda: itc.precompute_recursive(x4, sig, scale=c4.scale))
        recs.append({"sigma": sig, "ms": t_r * 1e3, "gpx_per_s": c4.img.size / t_r / 1e9})
    out["recursive_gray2048"] = recs

    # 3-D lattice: a 96 x 192 x 256 ellipsoid volume, sigma = 2, M = 64, 50 sweeps
    vc = synth.volume_case(0, D=96, H=192, W=256, M=64, iters=50)
    xv = torch.from_numpy(vc.vol).to(dev)
    wv0 = torch.from_numpy(vc.w0).to(dev)
    vm = itc.volume_precompute(xv, vc.sigma)
    t_vm = timed(lambda: itc.volume_precompute(xv, vc.sigma))
    t_vf = timed(lambda: itc.volume_fit(vm, wv0, vc.iters), reps=3)
    out["volume_96x192x256"] = {"voxels": int(vc.vol.size), "M": vc.M, "sweeps": vc.iters, "maps_ms": t_vm * 1e3,
                                "maps_gvox_per_s": vc.vol.size / t_vm / 1e9, "fit_ms": t_vf * 1e3,
                                "volumes_per_s": 1.0 / (t_vm + t_vf)}
    del vm

    # differentiation: forward D and the adjoint (dD/dw, dD/dh) of 64 weighted
    # 1024 x 1024 images, M = 256, sigma = 4, FP32 per-pixel weights h = g/255
    # (the autograd path: FP32 weights take the vector-ALU convolution)
    c5 = synth.config5_cases(64)
    B5, H5, W5, M5 = len(c5), 1024, 1024, 256
    p5 = itc.BatchPlan.for_stack(B5, H5, W5, M5, 4.0, iters=0, dtype=torch.float32, device=dev)
    h5 = torch.stack([torch.from_numpy(c.img) for c in c5]).to(dev).float() / 255.0
    w5 = torch.cat([torch.from_numpy(c.w0) for c in c5]).to(dev, torch.float32)
    maps5 = p5.new_maps()
    wout5 = torch.empty_like(w5)
    sx5 = torch.empty(B5, dtype=torch.float64, device=dev)
    d5 = torch.empty(B5, dtype=torch.float64, device=dev)
    gd5 = torch.ones(B5, dtype=torch.float64, device=dev)
    gw5 = torch.empty_like(w5)
    gh5 = torch.empty((B5, H5, W5), dtype=torch.float32, device=dev)
    f_conv = lambda: p5.precompute(weights=h5, maps=maps5)  # noqa: E731
    f_d = lambda: p5.fit(w5, wout5, s_x=sx5, d_out=d5, maps=maps5)  # noqa: E731
    f_gw = lambda: p5.backward(w5, sx5, gd5, grad_w=gw5, maps=maps5)  # noqa: E731
    f_gh = lambda: p5.backward(w5, sx5, gd5, grad_weights=gh5, maps=maps5)  # noqa: E731
    parts = {k: timed(f) for k, f in (("conv", f_conv), ("divergence", f_d), ("grad_w", f_gw), ("grad_h", f_gh))}
    tot = sum(parts.values())
    px5 = float(B5 * H5 * W5)
    out["differentiation_gray1024x64"] = {
        "images": B5, "M": M5, "sigma": 4.0, "weights": "FP32", "images_per_s": B5 / tot, "ms_total": tot * 1e3,
        "ms": {k: v * 1e3 for k, v in parts.items()},
        "conv_gbs_algorithmic": 16.0 * px5 / parts["conv"] / 1e9, "conv_bytes_per_px": 16,
        "grad_h_gbs_algorithmic": 8.0 * px5 / parts["grad_h"] / 1e9, "grad_h_bytes_per_px": 8}
    del p5, maps5, gh5, h5

    # convergence: the theta stop on the silhouettes (largest codevector step <= theta px)
    pc = itc.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases], [c.sigma for c in cases],
                       [c.iters for c in cases], device=dev)
    w0c = pc.pack_codebooks([c.w0 for c in cases], device=dev)
    wc = torch.empty_like(w0c)
    sxc = torch.empty(len(cases), dtype=torch.float64, device=dev)
    dc = torch.empty_like(sxc)
    donec = torch.empty(len(cases), dtype=torch.int32, device=dev)
    conv_t = []
    for theta in (1e-2, 1e-3):
        t_run = timed(lambda: pc.run(w0c, wc, sxc, dc, donec, theta=theta), reps=3)
        k = donec.cpu().numpy()
        conv_t.append({"theta_px": theta, "images_per_s": len(cases) / t_run, "ms": t_run * 1e3,
                       "sweeps_median": float(np.median(k)), "sweeps_p90": float(np.percentile(k, 90)),
                       "sweeps_max": int(k.max()), "fraction_under_20": float(np.mean(k < 20)),
                       "fraction_stopped": float(np.mean(k < 100))})
    out["theta_stop_silhouettes"] = conv_t
    del pc

    p = itc.BatchPlan([torch.from_numpy(c.img) for c in c5], [c.M for c in c5], [c.sigma for c in c5],
                      [c.iters for c in c5], device=dev)
    t = timed(p.precompute)
    px = float(sum(c.img.size for c in c5))
    out["conv_gray1024x64"] = {"images": len(c5), "pixels": int(px), "ms": t * 1e3, "gbs": 13.0 * px / t / 1e9,
                               "frac_hbm_peak": 13.0 * px / t / 1e9 / HBM_PEAK_GBS}
    del p
    return out


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--images", type=int, default=1400, help="silhouettes in the batch")
    p.add_argument("--cpu-seconds", type=float, default=15.0, help="budget of the oracle leg")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--no-per-image", action="store_true")
    p.add_argument("--no-extras", action="store_true",
                   help="skip the secondary measurements (copy peak, per-sigma conv, single-image workloads)")
    p.add_argument("--eager", action="store_true",
                   help="launch on the stream instead of replaying a HIP graph (for counter profiling)")
    p.add_argument("--no-tune", action="store_true",
                   help="keep the default convolution tile shapes instead of autotuning them")
    p.add_argument("--tune-cache", default=None,
                   help="JSON cache of tuned shapes (default: $ITC_TUNE_CACHE or ~/.cache/itc_lattice/tune.json)")
    p.add_argument("--copy-calib-mib", type=int, default=0,
                   help="also run one device copy of this many MiB (calibrates HBM byte counters)")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: there is no multi-GPU path "
              "(images would shard across GPUs with no communication); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1310_7114_amd import itc, synth

    t0 = time.time()
    cases = synth.config3_cases(args.images)
    print(f"[bench] generated {len(cases)} silhouettes in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    n = len(cases)
    npx = int(sum(c.img.size for c in cases))
    # ---------------- oracle on the host cores (before the GPU is touched) ----------------
    cpu, cpu_context = None, None
    if not args.no_cpu:
        cpu, cpu_context = cpu_legs(cases, args.cpu_seconds)

    itc.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.copy_calib_mib > 0:  # a plain copy kernel of known size, for counter calibration
        nel = args.copy_calib_mib * (1 << 20) // 4
        src = torch.ones(nel, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    plan = itc.BatchPlan([torch.from_numpy(c.img) for c in cases], [c.M for c in cases],
                         [c.sigma for c in cases], [c.iters for c in cases], device=dev)
    w0 = plan.pack_codebooks([c.w0 for c in cases], device=dev)
    # tile shapes of the convolution per radius class, chosen on this batch
    # before anything is captured or timed (not part of the timed step)
    tuned = None
    if not args.no_tune:
        from paper_1310_7114_amd import autotune
        tuned = {str(k): v for k, v in autotune.tune_conv(plan, path=args.tune_cache).items()}
        print(f"[bench] autotuned convolution shapes {tuned}", file=sys.stderr, flush=True)
    w = torch.empty_like(w0)
    sx = torch.empty(n, dtype=torch.float64, device=dev)
    dd = torch.empty(n, dtype=torch.float64, device=dev)
    done = torch.empty(n, dtype=torch.int32, device=dev)

    # ---------------- batched step: two HIP graphs (convolution, fit + D) ----------------
    # The convolution of an 8-bit batch is one persistent kernel launch and the
    # fit another; each is captured in a graph of its own, and HIP events
    # recorded between the replays (on the replay stream) time every launch of
    # the timed steps.
    conv_fn = plan.precompute
    fit_fn = lambda: plan.fit(w0, w, sx, dd, done)  # noqa: E731
    if args.eager:
        conv_step, fit_step = conv_fn, fit_fn
    else:
        g_conv, g_fit = capture(conv_fn), capture(fit_fn)
        conv_step, fit_step = g_conv.replay, g_fit.replay
    for _ in range(max(1, args.warmup)):
        conv_step()
        fit_step()
    torch.cuda.synchronize()
    print("[bench] warm-up done; timing batched steps", file=sys.stderr, flush=True)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t = time.perf_counter()
    for k in range(args.steps):
        evs[k][0].record()
        conv_step()
        evs[k][1].record()
        fit_step()
        evs[k][2].record()
    torch.cuda.synchronize()
    step_s = (time.perf_counter() - t) / args.steps
    assert bool(torch.all(done == 100)) and bool(torch.all(torch.isfinite(dd)))
    conv_ms = [e[0].elapsed_time(e[1]) for e in evs]
    fit_ms = [e[1].elapsed_time(e[2]) for e in evs]
    conv_s = float(np.median(conv_ms)) / 1e3
    fit_s = float(np.median(fit_ms)) / 1e3
    conv_launches = plan.conv_launches()

    # ---------------- secondary: the step with its weights uploaded from pinned host memory ----------------
    # (the library takes device buffers; this is the rate with the PCIe upload included, never `value`)
    pcie = None
    if not args.eager:
        host_w = torch.empty(plan.weights.numel(), dtype=plan.weights.dtype, pin_memory=True)
        host_w.copy_(plan.weights)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for _ in range(args.steps):
            plan.weights.copy_(host_w, non_blocking=True)
        torch.cuda.synchronize()
        h2d_s = (time.perf_counter() - t) / args.steps
        t = time.perf_counter()
        for _ in range(args.steps):
            plan.weights.copy_(host_w, non_blocking=True)
            conv_step()
            fit_step()
        torch.cuda.synchronize()
        both_s = (time.perf_counter() - t) / args.steps
        nbytes = host_w.numel() * host_w.element_size()
        pcie = {"bytes": int(nbytes), "h2d_gbs": nbytes / h2d_s / 1e9, "images_per_s": n / both_s,
                "note": "pinned host-to-device upload of the packed 8-bit weights before every step"}
        del host_w

    # algorithmic work of the convolution (13 B per pixel) over the median
    # duration of its launch; 5 filters x (2R+1) taps FMA per pixel (2 flop
    # each) is what the direct form would compute
    conv_bytes = CONV_BYTES_PER_PX * npx
    conv_flops = float(sum(2.0 * 5 * (2 * c.R + 1) * c.img.size for c in cases))
    conv_gbs = conv_bytes / conv_s / 1e9
    conv_tfs = conv_flops / conv_s / 1e12
    # algorithmic work of the fit: every sweep, and the final divergence,
    # evaluates the M(M-1)/2 distinct codebook pairs of every image
    fit_pairs = float(sum((c.iters + 1) * c.M * (c.M - 1) / 2 for c in cases))
    fit_tfs = FIT_FLOPS_PER_PAIR * fit_pairs / fit_s / 1e12
    fit_peak_tfs = FIT_FLOPS_PER_PAIR * FIT_PEAK_PAIRS_PER_S / 1e12
    fit_prof = profile_figures("fit_silhouettes1400")
    conv_prof = profile_figures("conv_silhouettes1400")

    # ---------------- per-image loop (same kernels, one image at a time) ----------------
    per_image = None
    if not args.no_per_image:
        maps = [plan.maps_of(i) for i in range(n)]
        ws = [plan.unpack(w0, i) for i in range(n)]
        outs = [plan.unpack(w, i) for i in range(n)]
        imgs = [plan.image(plan.weights, i) for i in range(n)]
        dtr = [torch.empty(c.iters + 1, dtype=torch.float64, device=dev) for c in cases]
        dn = torch.empty(n, dtype=torch.int32, device=dev)

        def loop():
            for i, c in enumerate(cases):
                itc.precompute(imgs[i], c.sigma, scale=c.scale, out=maps[i])
                lib = itc.load()
                st = lib.itc_lattice_fit(itc.ctypes.byref(maps[i].desc), itc._ptr(maps[i].buf),
                                         itc._ptr(maps[i].s_x), c.M, itc._ptr(ws[i]), c.iters, -1.0,
                                         itc._ptr(outs[i]), itc._ptr(dtr[i]), itc._ptr(dn[i:i + 1]),
                                         itc._stream())
                itc._check(st)

        pg = capture(loop)
        pg.replay()
        torch.cuda.synchronize()
        reps = max(1, min(3, args.steps))
        t = time.perf_counter()
        for _ in range(reps):
            pg.replay()
        torch.cuda.synchronize()
        pi_s = (time.perf_counter() - t) / reps
        per_image = {"value": n / pi_s, "unit": "images/s", "ms_per_pass": pi_s * 1e3,
                     "launches": "precompute (2 kernels) + fit (1 kernel) per image, one stream, HIP graph"}
        print(f"[bench] per-image loop {pi_s * 1e3:.1f} ms per pass", file=sys.stderr, flush=True)

    extras = None
    if not args.no_extras:
        extras = gpu_extras(dev, cases, itc, synth)
        print("[bench] secondary measurements done", file=sys.stderr, flush=True)

    value = n / step_s
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "images/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": step_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"silhouettes-{n}: binary star polygons, W 128..1024 x H 128..768, "
                               f"M 10..200, sigma 2/4/8, 100 sweeps, batched persistent + "
                               + ("stream launches" if args.eager else "HIP graph"),
                   "images": n, "pixels": npx, "iters": 100},
        "phases_ms": {"conv": conv_s * 1e3, "fit_and_divergence": fit_s * 1e3,
                      "timing": f"median over the {args.steps} timed steps, HIP events between graph replays"},
        "per_image": per_image,
        "pcie_inclusive": pcie,
        "autotune": tuned,
        "batched_over_per_image": (value / per_image["value"]) if per_image else None,
        "roofline": {"bound": "hbm", "achieved": conv_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": conv_gbs / HBM_PEAK_GBS,
                     "traffic": conv_prof["traffic_bytes_per_step"] if conv_prof else None,
                     "kernel": "conv_mx_tiles_kernel (one persistent launch per step)",
                     "launches_per_step": conv_launches, "bytes_per_px": CONV_BYTES_PER_PX,
                     "algorithmic_bytes": conv_bytes, "ms": conv_s * 1e3,
                     "direct_form_tflops": conv_tfs},
        "fit_roofline": {"bound": "alu", "achieved": fit_tfs, "peak": fit_peak_tfs, "unit": "TFLOP/s",
                         "frac": fit_tfs / fit_peak_tfs, "pairs": fit_pairs, "flops_per_pair": FIT_FLOPS_PER_PAIR,
                         "pairs_per_s": fit_pairs / fit_s,
                         "traffic": fit_prof["traffic_bytes_per_step"] if fit_prof else None,
                         "kernel": "fit_batched_kernel (all sweeps + D, one launch)", "ms": fit_s * 1e3},
        "cpu_baseline": cpu,
        "cpu_context": cpu_context,
        "extras": extras,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
