"""Autotuner of the fused-pass schedule, one schedule per size class.

A schedule (``fht_schedule`` in ``include/fht.h``) only changes how the
transform is tiled into fused passes, never its result.  Images are grouped
into size classes, ``(ceil log2 rows, ceil log2 cols)``: the heights of the
two order trees (proof of Theorem 1), which fix how many levels the passes
have to cover, and so where the passes can be cut.  For every class present
in a batch the tuner runs a coordinate descent over the knobs that change the
pass structure or the tiles:

* ``first_levels``: levels of the first pass (where it cuts the tree);
* ``max_levels``: levels per later pass (how many passes, and where they cut);
* ``s_tile_first``, ``s_tile``: position windows of the first and later passes;
* ``t_tile``: slope rows per later work item;
* ``threads``, ``threads_first``: workgroup sizes.

Each candidate is timed on that class's images of the batch, run as a batch
of their own (device events on the working stream, best of three groups).
A class's winner then has to pay off in the whole batch, where the classes
share launches: starting from the library default for every class, the
classes are visited largest first, and a class keeps its winner only if the
whole batch gets faster with it (other workgroup sizes, for instance, add
launches of their own).  The result is cached in a JSON file keyed by GPU
architecture, dtype, split rule and class, so a later batch reuses it for
every image of the class.  ``plans_for`` builds a batch's plans with
the cached schedule of each image's class (the library default for classes
never tuned).  The cache is safe to delete.
"""
from __future__ import annotations

import json
import math
import os
import time
from collections import defaultdict
from typing import Sequence

from . import _binding as B

DEFAULT = dict(s_tile=192, s_tile_first=128, first_levels=5, max_levels=3, t_tile=16,
               threads=512, threads_first=512, lds_budget=65536)

# Knobs in the order the descent visits them, with the values it tries.
KNOBS = (
    ("first_levels", (4, 5, 6)),
    ("max_levels", (2, 3, 4, 5)),
    ("s_tile_first", (64, 128, 192)),
    ("s_tile", (128, 192, 256)),
    ("t_tile", (8, 16, 32)),
    ("threads", (256, 512)),
    ("threads_first", (256, 512)),
)

# Report of the last autotune() call (per class: source, schedule, timings).
last_report: dict = {}


def cache_path() -> str:
    return os.environ.get("FHT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "fht_autotune.json"))


def size_class(rows: int, cols: int) -> str:
    """Heights of the two order trees: ceil(log2 rows) x ceil(log2 cols)."""
    def h(n):
        return max(0, math.ceil(math.log2(n))) if n > 1 else 0
    return f"{h(rows)}x{h(cols)}"


def _arch() -> str:
    import torch
    if not torch.cuda.is_available():
        return "cpu"
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def class_key(cls: str, dtype: str, split: str, arch: str | None = None) -> str:
    return f"{arch or _arch()}|{dtype}|{split}|{cls}"


def _dtype_name(img) -> str:
    return {1: "u8", 4: "f32", 8: "f64"}[img.element_size()]


def _split_name(split) -> str:
    return "S" if split in ("S", 0, B.FHT_SPLIT_S) else "T"


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(entries: dict) -> None:
    cache = _load_cache()
    cache.update(entries)
    path = cache_path()
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.{os.getpid()}.tmp"
    with open(tmp, "w") as fh:
        json.dump(cache, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(rows: int, cols: int, dtype="u8", split="S") -> dict | None:
    """The cached schedule of this shape's class, or None."""
    entry = _load_cache().get(class_key(size_class(rows, cols), dtype, _split_name(split)))
    return dict(entry["schedule"]) if entry else None


def time_batch(imgs, schedule: dict, split="S", reps: int = 3, groups: int = 3,
               warmup: int = 1) -> float:
    """Milliseconds of one batched transform of `imgs` under `schedule`
    (best of `groups` groups of `reps` runs)."""
    plans, cache = [], {}
    for img in imgs:
        key = (tuple(img.shape), img.dtype)
        if key not in cache:
            cache[key] = B.Plan(img.shape[0], img.shape[1], img.dtype, split, schedule=schedule)
        plans.append(cache[key])
    return time_plans(imgs, plans, reps, groups, warmup)


def time_plans(imgs, plans, reps: int = 3, groups: int = 3, warmup: int = 1, outs=None) -> float:
    """Milliseconds of one batched transform of `imgs` with one plan each."""
    import torch
    if outs is None:
        outs = [p.new_out(i.device) for p, i in zip(plans, imgs)]
    batch = B.Batch(plans, imgs, outs)
    ws = batch.new_ws(imgs[0].device)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        batch.run(ws)
    best = float("inf")
    for _ in range(groups):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(reps):
            batch.run(ws)
        e1.record(stream)
        torch.cuda.synchronize()
        best = min(best, e0.elapsed_time(e1) / reps)
    return best


def tune_class(imgs, split="S", knobs=KNOBS, reps: int = 3, start: dict | None = None):
    """Coordinate descent over `knobs` for one class's images: returns the
    best schedule and every (schedule, ms) tried."""
    best = dict(start or DEFAULT)
    tried = {}

    def measure(sched):
        key = json.dumps(sched, sort_keys=True)
        if key not in tried:
            try:
                tried[key] = (dict(sched), time_batch(imgs, sched, split, reps=reps))
            except (B.FhtError, ValueError):
                tried[key] = (dict(sched), float("inf"))  # no plan fits: skipped
        return tried[key][1]

    best_ms = measure(best)
    for name, values in knobs:
        for v in values:
            if v == best.get(name):
                continue
            cand = dict(best, **{name: v})
            ms = measure(cand)
            if ms < best_ms:
                best, best_ms = cand, ms
    timings = [{"schedule": s, "ms": round(ms, 4)} for s, ms in tried.values()
               if ms != float("inf")]
    return best, best_ms, timings


def _in_batch(imgs, split, start: dict, proposals: dict, classes_of: list, reps: int):
    """From the schedules `start` (one per class), keeps, largest class
    first, each class's proposal that makes the whole batch faster (by more
    than 0.3 %).  Returns the schedules and the batch milliseconds with
    `start` and with the kept proposals."""
    plan_cache = {}

    def plans_with(scheds):
        plans = []
        for img, cls in zip(imgs, classes_of):
            sc = scheds[cls]
            key = (tuple(img.shape), json.dumps(sc, sort_keys=True))
            if key not in plan_cache:
                plan_cache[key] = B.Plan(img.shape[0], img.shape[1], img.dtype, split, schedule=sc)
            plans.append(plan_cache[key])
        return plans

    cur = dict(start)
    plans = plans_with(cur)
    outs = [p.new_out(i.device) for p, i in zip(plans, imgs)]
    base = default_ms = time_plans(imgs, plans, reps, outs=outs)
    px = defaultdict(int)
    for img, cls in zip(imgs, classes_of):
        px[cls] += img.shape[0] * img.shape[1]
    kept = []
    for cls in sorted(proposals, key=lambda c: -px[c]):
        if proposals[cls] == cur[cls]:
            continue
        trial = dict(cur)
        trial[cls] = proposals[cls]
        ms = time_plans(imgs, plans_with(trial), reps, outs=outs)
        if ms < base * 0.997:
            cur, base = trial, ms
            kept.append(cls)
    return cur, default_ms, base, kept


def autotune(imgs, split="S", knobs=KNOBS, reps: int = 3, use_cache: bool = True,
             max_images_per_class: int = 16, in_batch: bool = True) -> dict:
    """Schedule per size class for the images of this batch, tuned for every
    class not yet in the cache (each class alone, then, with ``in_batch``,
    kept only where it speeds up the whole batch).  Returns {class:
    schedule}; ``last_report`` tells which classes were tuned and which came
    from the cache."""
    global last_report
    split = _split_name(split)
    dtype = _dtype_name(imgs[0])
    if any(_dtype_name(i) != dtype for i in imgs):
        raise ValueError("one dtype per batch")
    arch = _arch()
    by_class = defaultdict(list)
    for img in imgs:
        by_class[size_class(img.shape[0], img.shape[1])].append(img)
    cache = _load_cache() if use_cache else {}
    out, report, new = {}, {}, {}
    t0 = time.perf_counter()
    for cls in sorted(by_class):
        key = class_key(cls, dtype, split, arch)
        if key in cache:
            out[cls] = dict(cache[key]["schedule"])
            report[cls] = {"source": "cache", "schedule": out[cls]}
            continue
        sub = by_class[cls][:max_images_per_class]
        best, best_ms, timings = tune_class(sub, split, knobs, reps)
        default_ms = next((t["ms"] for t in timings if t["schedule"] == DEFAULT), None)
        out[cls] = best
        new[key] = {"schedule": best, "alone": best, "timings_ms": timings, "images": len(sub)}
        report[cls] = {"source": "tuned", "schedule": best, "ms": round(best_ms, 4),
                       "default_ms": default_ms, "candidates": len(timings), "images": len(sub)}
    batch_rep = None
    fresh = [c for c in report if report[c]["source"] == "tuned"]
    if in_batch and fresh:
        classes_of = [size_class(i.shape[0], i.shape[1]) for i in imgs]
        start = {c: (dict(DEFAULT) if c in fresh else out[c]) for c in out}
        _, d_ms, t_ms, kept = _in_batch(imgs, split, start, {c: out[c] for c in fresh},
                                        classes_of, reps)
        for c in fresh:
            if c not in kept:
                out[c] = dict(DEFAULT)
            key = class_key(c, dtype, split, arch)
            new[key]["schedule"] = out[c]
            new[key]["kept_in_batch"] = c in kept
            report[c]["schedule"] = out[c]
            report[c]["kept_in_batch"] = c in kept
        batch_rep = {"default_ms": round(d_ms, 4), "tuned_ms": round(t_ms, 4), "kept": kept}
    if new:
        _store(new)
    last_report = {"classes": report, "batch": batch_rep,
                   "seconds": round(time.perf_counter() - t0, 2)}
    return out


# Schedules for images transformed one at a time (one launch per fused pass
# per image).  Such launches hold at most a few rounds of work items, so each
# costs about one item's latency plus the launch; fewer passes can then win
# even where they lose in a batch.  "two-pass": a 6-level first pass and
# 4-level later passes in up to 160 KB of LDS per item (10 levels, up to 1024
# lanes per view, in two passes instead of three).
PLAIN_SCHEDULES = {
    "default": None,
    "two-pass": dict(first_levels=6, max_levels=4, lds_budget=163840),
}


def tune_plain(imgs, split="S", candidates=("default", "two-pass"), reps: int = 3):
    """Picks the schedule for per-image launches of same-shape `imgs` (device
    tensors): each candidate of PLAIN_SCHEDULES transforms every image with
    its own launches (device events, best of `reps` runs); the fastest wins.
    Candidates must agree on every output (a schedule never changes the
    result), else this raises.  Returns (name, {name: microseconds per image})."""
    import torch
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    R, C = imgs[0].shape
    times, ref = {}, None
    for name in candidates:
        plan = B.Plan(R, C, imgs[0].dtype, _split_name(split), schedule=PLAIN_SCHEDULES[name])
        outs = [plan.new_out(imgs[0].device) for _ in imgs]
        ws = plan.new_ws(imgs[0].device)

        def run():
            for im, o in zip(imgs, outs):
                B.fht_forward(plan.handle, im.data_ptr(), o.data_ptr(), ws.data_ptr(), sh)

        run()
        torch.cuda.synchronize()
        if ref is None:
            ref = outs
        elif not all(torch.equal(a, b) for a, b in zip(ref, outs)):
            raise RuntimeError(f"schedule {name!r} changed the transform's result")
        best = float("inf")
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            run()
            e1.record(stream)
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e3 / len(imgs))
        times[name] = round(best, 2)
    return min(times, key=times.get), times


def plans_for(shapes: Sequence[tuple], dtype, split="S", schedules: dict | None = None):
    """One plan per shape (shared between equal shapes), each with its size
    class's schedule from `schedules` (as autotune returns) or the cache, the
    library default otherwise."""
    split_n = _split_name(split)
    dname = {B.FHT_U8: "u8", B.FHT_F32: "f32", B.FHT_F64: "f64"}[B._dtype_code(dtype)]
    plans, made = [], {}
    for r, c in shapes:
        if (r, c) not in made:
            cls = size_class(r, c)
            sched = (schedules or {}).get(cls)
            if sched is None:
                sched = lookup(r, c, dname, split_n)
            made[(r, c)] = B.Plan(r, c, dtype, split_n, schedule=sched)
        plans.append(made[(r, c)])
    return plans
