"""Autotuner of the batched convolution's tile shapes.

A plan's convolution (Section 3.1's convolutions over a batch) runs one
persistent launch per radius class over 64-column strips cut into segments.
The segment height trades the recomputed halo rows of every segment (2R per
segment) against the number of tiles that balance the compute units, and
the workgroups per compute unit trade latency hiding against the tail of the
tile queue. `tune_conv` times `plan.precompute()` on the plan's own images for
every candidate shape of one class at a time (the other classes held),
keeps the fastest and records it in a JSON cache keyed by device, batch and
class. The maps are bitwise the same for every shape, so tuning changes only
the time.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional, Sequence

import torch

SEG_CANDIDATES = (128, 192, 256, 384, 512)


def cache_path(path: Optional[str] = None) -> str:
    """The JSON cache: `path`, else $ITC_TUNE_CACHE, else ~/.cache/itc_lattice/tune.json."""
    return path or os.environ.get("ITC_TUNE_CACHE") or os.path.join(
        os.path.expanduser("~"), ".cache", "itc_lattice", "tune.json")


def batch_signature(plan) -> str:
    """Identifies a batch layout for the cache: image count and stored weight elements."""
    return f"images={plan.n}|weights={int(plan.weights.numel())}"


def _time_ms(fn, reps: int) -> float:
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def _store(path: str, data: dict) -> None:
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs the next run a search


def tune_conv(plan, seg_candidates: Sequence[int] = SEG_CANDIDATES, reps: int = 5, use_cache: bool = True,
              path: Optional[str] = None) -> Dict[int, dict]:
    """Chooses and applies the tile shape of every convolution class of `plan`.

    Candidates: `seg_candidates` segment heights x (the most workgroups per
    compute unit, one fewer). Returns {class key: {seg_rows, blocks_per_cu,
    ms, cached}}, `ms` being the whole convolution phase with that choice.
    Call before capturing graphs of the plan."""
    path = cache_path(path)
    store = _load(path) if use_cache else {}
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    dev = f"{getattr(props, 'gcnArchName', props.name)}|cus={props.multi_processor_count}"
    sig = batch_signature(plan)
    chosen: Dict[int, dict] = {}
    changed = False
    for cl in plan.conv_classes():
        key, top = cl["key"], cl["max_blocks_per_cu"]
        ck = f"{dev}|{sig}|class={key}"
        hit = store.get(ck)
        if hit is not None:
            plan.set_conv_shape(key, int(hit[0]), int(hit[1]))
            chosen[key] = {"seg_rows": int(hit[0]), "blocks_per_cu": int(hit[1]), "ms": None, "cached": True}
            continue
        best = None
        for per in sorted({top, max(1, top - 1)}, reverse=True):
            for seg in seg_candidates:
                plan.set_conv_shape(key, seg, per)
                t = _time_ms(plan.precompute, reps)
                if best is None or t < best[0]:
                    best = (t, seg, per)
        plan.set_conv_shape(key, best[1], best[2])
        chosen[key] = {"seg_rows": best[1], "blocks_per_cu": best[2], "ms": best[0], "cached": False}
        store[ck] = [best[1], best[2]]
        changed = True
    if use_cache and changed:
        _store(path, store)
    return chosen
