"""Summaries of rocprofv3 runs of ``bench.py`` for ``profiles/``.

Reads one kernel-trace run (``--kernel-trace --stats --output-format csv``)
and two counter runs (``--pmc FETCH_SIZE`` and ``--pmc WRITE_SIZE``, with
``bench.py --copy-calib-mib N`` so that a plain device copy of N MiB is
counted beside the kernels) and writes one markdown summary per kernel
group: average launch durations, HBM bytes per launch from the counters
(scaled by what the same counters read for the copy of known size), and the
SHA-256 of the kernel's source files, which ``bench.py`` checks before it
reports the traffic figure.

    python3 -m paper_1310_7114_amd.profsummary --trace T --fetch F --write W \
        --calib-mib 1024 --commands commands.txt --out profiles
    python3 -m paper_1310_7114_amd.profsummary --secondary --trace T2 \
        --commands commands2.txt --out profiles
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import os
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join("paper_1310_7114_amd", "csrc")

SILHOUETTES = ("1400 binary star silhouettes (W 128..1024 x H 128..768, M 10..200, sigma 2/4/8, 100 sweeps), "
               "FP32, inputs resident in HBM")
GRAY1024 = ("64 weighted 1024 x 1024 gray images (weights g/255 in FP32, M 256, sigma 4): convolution, D, "
            "dD/dw and dD/dh, each launched twice (profile_workloads differentiation)")
GRAY2048 = ("the 2048 x 2048 gray image (M 500, sigma 6): maps and 200 sweeps of the multi-workgroup fit, "
            "twice (profile_workloads gray2048)")
SILHOUETTE_PX = 355434824.0
GRAY1024_PX = 64.0 * 1024 * 1024

# kernel group -> kernel-name prefix (after the namespace), source files whose
# hash guards the figures, workload, algorithmic HBM bytes per launch (or None)
GROUPS = {
    "fit_silhouettes1400": ("itc::fit_batched_kernel", [f"{CSRC}/fit.hip", f"{CSRC}/itc_device.h"],
                            SILHOUETTES, None),
    "conv_silhouettes1400": ("itc::conv_mx_tiles_kernel", [f"{CSRC}/conv_mfma.hip", f"{CSRC}/itc_device.h"],
                             SILHOUETTES, 13.0 * SILHOUETTE_PX),
    "conv_valu_gray1024x64": ("itc::conv_tiles_kernel", [f"{CSRC}/conv.hip", f"{CSRC}/itc_device.h"],
                              GRAY1024, 16.0 * GRAY1024_PX),
    "adjoint_gray1024x64": ("itc::grad_weights_tiles_kernel", [f"{CSRC}/adjoint.hip", f"{CSRC}/itc_device.h"],
                            GRAY1024, 8.0 * GRAY1024_PX),
    "fit_wide_gray2048": ("itc::fit_wide_kernel", [f"{CSRC}/fit_wide.hip", f"{CSRC}/itc_device.h"],
                          GRAY2048, None),
}
HBM_PEAK = 8.0e12


def source_sha256(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def short(name: str) -> str:
    return name.replace("(anonymous namespace)::", "").split("(")[0].replace("void ", "")


def kernel_stats(trace_dir: str):
    out = {}
    for f in glob.glob(os.path.join(trace_dir, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            out[short(r["Name"])] = (int(r["Calls"]), float(r["AverageNs"]) / 1e3, float(r["TotalDurationNs"]) / 1e3)
    return out


def counters(pmc_dir: str, counter: str):
    """Per kernel name: list of per-dispatch values (KiB) of one counter."""
    per = defaultdict(list)
    for f in glob.glob(os.path.join(pmc_dir, "**", "*counter_collection.csv"), recursive=True):
        acc = defaultdict(float)
        names = {}
        for r in csv.DictReader(open(f)):
            if r["Counter_Name"] != counter:
                continue
            key = r.get("Dispatch_Id") or r.get("Correlation_Id")
            acc[key] += float(r["Counter_Value"])
            names[key] = short(r["Kernel_Name"])
        for key, v in acc.items():
            per[names[key]].append(v)
    return per


def copy_kernel_value(per, expected_kib: float):
    """The copy of known size: the copy-named dispatch closest to the expected size."""
    best = None
    for name, vals in per.items():
        if "copy" not in name.lower():
            continue
        for v in vals:
            if best is None or abs(v - expected_kib) < abs(best - expected_kib):
                best = v
    return best


# secondary workloads of the benchmark's extras: summary name -> (title, kernel name fragments)
SECONDARY = {
    "volume_96x192x256": ("3-D lattice maps and fit: 96 x 192 x 256 ellipsoid volume, sigma 2, M 64, 50 sweeps",
                          ["vol_"]),
    "recursive_gray2048": ("recursive Gaussian maps of the 2048 x 2048 gray image, sigma 4, 16 and 40",
                           ["rec_"]),
    "chamfer_silhouettes1400": ("chamfer transform of the 1400 silhouettes (batched)", ["chamfer_"]),
    "literal_shapes512_silhouette49": ("Algorithm 1 with the paper's widths: the 512 x 512 shapes (M 100, masks) "
                                       "and silhouette 49 of the batch (M 17, xi 15.6, recursive P), 20 and 0 "
                                       "sweeps each", ["literal_"]),
    "segments_silhouettes1400": ("nearest-codevector labels of the 1400 silhouettes (batched)", ["label_"]),
}


def secondary(trace: str, commands: str, out: str) -> None:
    """Kernel-duration tables of the secondary workloads from one kernel-trace run of bench.py with extras."""
    stats = kernel_stats(trace)
    cmds = open(commands).read().strip()
    os.makedirs(out, exist_ok=True)
    for name, (title, frags) in SECONDARY.items():
        names = sorted(k for k in stats if any(f in k for f in frags))
        if not names:
            continue
        lines = [f"# {name}", "", f"{title}; kernel durations (rocprofv3 --kernel-trace --stats) from the",
                 "benchmark's secondary measurements, every launch of the run. Produced by these commands, from",
                 "the repository root:", "", "```", cmds, "```", "",
                 "| kernel | calls | average us | total us |", "|---|---|---|---|"]
        for k in names:
            c, avg, tot = stats[k]
            lines.append(f"| {k} | {c} | {avg:.1f} | {tot:.1f} |")
        path = os.path.join(out, f"{name}.md")
        with open(path, "w") as fh:
            fh.write("\n".join(lines) + "\n")
        print("wrote", path)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--trace", required=True)
    ap.add_argument("--secondary", action="store_true",
                    help="write the secondary workloads' kernel tables from --trace (no counter runs)")
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--calib-mib", type=float)
    ap.add_argument("--commands", required=True, help="text file with the commands that produced the runs")
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles"))
    ap.add_argument("--groups", nargs="*", default=None, help="write only these kernel groups")
    a = ap.parse_args()
    if a.secondary:
        secondary(a.trace, a.commands, a.out)
        return
    if not (a.fetch and a.write and a.calib_mib):
        ap.error("--fetch, --write and --calib-mib are required without --secondary")

    stats = kernel_stats(a.trace)
    fetch = counters(a.fetch, "FETCH_SIZE")
    write = counters(a.write, "WRITE_SIZE")
    exp_kib = a.calib_mib * 1024.0
    cf, cw = copy_kernel_value(fetch, exp_kib), copy_kernel_value(write, exp_kib)
    sf = exp_kib / cf if cf else None
    sw = exp_kib / cw if cw else None
    commands = open(a.commands).read().strip()
    os.makedirs(a.out, exist_ok=True)
    for group, (prefix, files, title, algo) in GROUPS.items():
        if a.groups and group not in a.groups:
            continue
        names = sorted(k for k in stats if k.startswith(prefix + "<") or k == prefix)
        if not names:
            continue
        lines = [f"# {prefix.split('::')[-1]}: {group}", "", title + ".",
                 "Produced by these commands, from the repository root:", "",
                 "```", commands, "```", "",
                 "| kernel | calls | average us | total us |", "|---|---|---|---|"]
        for k in names:
            c, avg, tot = stats[k]
            lines.append(f"| {k} | {c} | {avg:.1f} | {tot:.1f} |")
        lines += ["", f"Copy calibration: a {a.calib_mib:.0f} MiB device copy read FETCH_SIZE {cf} KiB and "
                      f"WRITE_SIZE {cw} KiB (expected {exp_kib:.0f} KiB each): scale factors "
                      f"{sf if sf is None else round(sf, 4)} (fetch), {sw if sw is None else round(sw, 4)} (write).", "",
                  "| kernel | FETCH_SIZE KiB/dispatch | WRITE_SIZE KiB/dispatch | HBM bytes per launch (scaled) |",
                  "|---|---|---|---|"]
        total_f = total_w = 0.0
        for k in names:
            fv = sum(fetch.get(k, [0.0])) / max(1, len(fetch.get(k, [])))
            wv = sum(write.get(k, [0.0])) / max(1, len(write.get(k, [])))
            fb = fv * 1024.0 * (sf or 1.0)
            wb = wv * 1024.0 * (sw or 1.0)
            total_f += fb
            total_w += wb
            lines.append(f"| {k} | {fv:.0f} | {wv:.0f} | {fb + wb:.4g} |")
        avg_launch = sum(stats[k][1] for k in names)
        if algo:
            gbs = algo / (avg_launch * 1e-6) / 1e9
            lines += ["", f"Roofline: {algo:.6g} algorithmic HBM bytes per launch / {avg_launch:.1f} us = "
                          f"{gbs:.0f} GB/s, {gbs * 1e9 / HBM_PEAK:.3f} of 8 TB/s; counted traffic "
                          f"{(total_f + total_w) / algo:.3f} x the algorithmic bytes."]
        lines += ["", "Figures read by bench.py (valid while the kernel sources hash to source_sha256):", "",
                  f"- source_files: {' '.join(files)}",
                  f"- source_sha256: {source_sha256(files)}",
                  f"- launches_per_step: {len(names)}",
                  f"- average_us_per_step: {avg_launch:.1f}",
                  f"- fetch_bytes_per_step: {total_f:.6g}",
                  f"- write_bytes_per_step: {total_w:.6g}",
                  f"- traffic_bytes_per_step: {total_f + total_w:.6g}", ""]
        path = os.path.join(a.out, f"{group}.md")
        with open(path, "w") as fh:
            fh.write("\n".join(lines))
        print("wrote", path)


if __name__ == "__main__":
    main()
