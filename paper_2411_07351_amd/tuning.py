"""Schedules and a small autotuner for batched transforms.

A schedule (``fht_schedule`` in ``include/fht.h``) only changes how the
transform is tiled into fused passes, never its result.  The autotuner times
candidate schedules on a given batch (device events on the working stream),
keeps the fastest, and caches the choice in a JSON file keyed by GPU
architecture, dtype, split rule and the batch's size classes, so that later
batches of the same kind reuse it.  The cache is safe to delete.
"""
from __future__ import annotations

import json
import math
import os
from collections import Counter
from typing import Sequence

from . import _binding as B

DEFAULT = dict(s_tile=192, s_tile_first=128, first_levels=5, max_levels=3, t_tile=16,
               threads=512, threads_first=512, lds_budget=65536)

# A modest candidate set around the default: fused depth of the first pass,
# window targets, slope tile and workgroup size of the later passes.
CANDIDATES = [
    DEFAULT,
    dict(DEFAULT, t_tile=8, threads=256),
    dict(DEFAULT, s_tile=128, threads=256),
    dict(DEFAULT, s_tile=256, lds_budget=131072),
    dict(DEFAULT, s_tile_first=192),
    dict(DEFAULT, first_levels=4, s_tile_first=192),
    dict(DEFAULT, threads_first=256),
    dict(DEFAULT, max_levels=4),
    dict(DEFAULT, max_levels=2),
]


def cache_path() -> str:
    return os.environ.get("FHT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fht_autotune.json"))


def size_class(rows: int, cols: int) -> str:
    return f"{math.ceil(math.log2(max(rows, 2)))}x{math.ceil(math.log2(max(cols, 2)))}"


def workload_key(shapes: Sequence[tuple], dtype: str, split: str) -> str:
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0] \
        if torch.cuda.is_available() else "cpu"
    hist = Counter(size_class(r, c) for r, c in shapes)
    classes = ",".join(f"{k}:{hist[k]}" for k in sorted(hist))
    return f"{arch}|{dtype}|{split}|{classes}"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(shapes, dtype="u8", split="S") -> dict | None:
    entry = _load_cache().get(workload_key(shapes, dtype, split))
    return dict(entry["schedule"]) if entry else None


def _store(key: str, schedule: dict, timings: list) -> None:
    cache = _load_cache()
    cache[key] = {"schedule": schedule, "timings_ms": timings}
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch(imgs, schedule: dict, split="S", reps: int = 3, warmup: int = 1) -> float:
    """Milliseconds of one batched transform of `imgs` under `schedule`."""
    import torch
    plans, outs, cache = [], [], {}
    for img in imgs:
        key = (tuple(img.shape), img.dtype)
        if key not in cache:
            cache[key] = B.Plan(img.shape[0], img.shape[1], img.dtype, split, schedule=schedule)
        plans.append(cache[key])
        outs.append(cache[key].new_out(img.device))
    batch = B.Batch(plans, imgs, outs)
    ws = batch.new_ws(imgs[0].device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        batch.run(ws)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        batch.run(ws)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def autotune(imgs, split="S", candidates=None, reps: int = 3, use_cache: bool = True) -> dict:
    """Fastest schedule for this batch (cached by workload kind)."""
    shapes = [tuple(i.shape) for i in imgs]
    dtype = {1: "u8", 4: "f32", 8: "f64"}[imgs[0].element_size()]
    key = workload_key(shapes, dtype, split)
    if use_cache:
        hit = lookup(shapes, dtype, split)
        if hit is not None:
            return hit
    timings = []
    best, best_ms = None, float("inf")
    for cand in candidates or CANDIDATES:
        try:
            ms = time_batch(imgs, cand, split, reps=reps)
        except B.FhtError:
            continue
        timings.append({"schedule": cand, "ms": round(ms, 4)})
        if ms < best_ms:
            best, best_ms = dict(cand), ms
    if best is None:
        raise RuntimeError("no candidate schedule could be planned")
    _store(key, best, timings)
    return best
