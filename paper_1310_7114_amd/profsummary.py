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

# kernel group -> (name fragment, source files whose hash guards the figures)
GROUPS = {
    "fit_silhouettes1400": ("fit_batched_kernel", [f"{CSRC}/fit.hip", f"{CSRC}/itc_device.h"]),
    "conv_silhouettes1400": ("conv_mx_tiles_kernel", [f"{CSRC}/conv_mfma.hip", f"{CSRC}/itc_device.h"]),
}


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
    "literal_shapes512": ("Algorithm 1 on the 512 x 512 shapes with the paper's widths (M 100, 20 and 0 sweeps)",
                          ["literal_"]),
    "recursive_gray2048": ("recursive Gaussian maps of the 2048 x 2048 gray image, sigma 4, 16 and 40",
                           ["rec_"]),
    "chamfer_silhouettes1400": ("chamfer transform of the 1400 silhouettes (batched)", ["chamfer_"]),
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
    for group, (frag, files) in GROUPS.items():
        names = sorted(k for k in stats if frag in k)
        if not names:
            continue
        lines = [f"# {frag}: silhouettes-1400 workload", "",
                 "1400 binary star silhouettes (W 128..1024 x H 128..768, M 10..200, sigma 2/4/8, 100 sweeps),",
                 "FP32, inputs resident in HBM. Produced by these commands, from the repository root:", "",
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
