#!/usr/bin/env python3
"""Throughput of the dyadic-pattern fast Hough transform on one MI355X.

Headline workload (one "step"): 64 uint8 edge maps of 1021 x 1021
(Bernoulli(0.05) background plus 20 Bresenham segments, seed 2411_07351 + 2),
all four quadrant Hough images with int32 outputs, FHT2DS split, launched per
image (``fht_forward_launch`` for every fused pass of every image), with the
schedule for per-image launches that the tuner picks on this workload (the
library default or a two-pass schedule; both timings are reported).  The same
batch also runs batched (library default schedule) (one launch per fused pass for all 64 images,
replayed from a captured HIP graph), and a ragged batch of 512 edge maps with
sides log-uniform in [32, 2048] runs both ways.  Inputs are resident in HBM
before timing starts.

Prints one JSON line.  ``--gpus`` above 1 is rejected: the benchmark measures
one GPU (several GPUs would each transform their own share of the images, with
no exchange between them).
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

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "input Mpixel/s + achieved HBM GB/s (batched vs plain); p50/p99 latency at fixed QPS"
COMPULSORY_BPP = 17  # read a uint8 pixel once, write four int32 outputs once
COMPULSORY_BPP_F32_FWD_ADJ = 40  # forward 4 + 16, adjoint 16 + 4 bytes per float32 pixel
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_pass_kernels_1021x1021_u8.txt")


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--images", type=int, default=64)
    ap.add_argument("--rows", type=int, default=1021)
    ap.add_argument("--cols", type=int, default=1021)
    ap.add_argument("--split", default="S", choices=["S", "T"])
    ap.add_argument("--ragged", type=int, default=512, help="images in the ragged batch (0: skip)")
    ap.add_argument("--tune", type=int, default=1,
                    help="also run the ragged batch with autotuned per-size-class schedules")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU oracle sample budget (0 disables the cpu_baseline leg)")
    ap.add_argument("--diff-images", type=int, default=32,
                    help="float32 384x257 images of the forward+adjoint leg (0: skip)")
    ap.add_argument("--serve-requests", type=int, default=300,
                    help="requests per serving run (0: skip the serving leg)")
    ap.add_argument("--serve-qps", type=float, default=200.0,
                    help="the fixed absolute request rate of the serving leg")
    ap.add_argument("--ceilings", type=int, default=1,
                    help="also measure torch's fill/copy/sum rates (1) or not (0)")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a device copy of this many MiB (counter calibration)")
    ap.add_argument("--plain-schedule", default="auto", choices=["auto", "default", "two-pass"],
                    help="schedule of the per-image launches: picked by timing both (auto) or fixed")
    return ap.parse_args()


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("kernels.hip", "kernels.hpp", "plan.cpp", "plan.hpp"):
        with open(os.path.join(ROOT, "paper_2411_07351_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _traffic(kernel: str, batched: bool = False, plain_schedule: str = "default"):
    """HBM bytes per launch of `kernel` from the committed counter summary, if it
    was taken on the current kernel sources (else None); `batched`: per launch
    of the 64-image batch, else per launch of the per-image path, which must
    have run the schedule the summary was taken with."""
    try:
        vals = {}
        with open(TRAFFIC_FILE) as fh:
            for line in fh:
                line = line.split("#", 1)[0].strip()
                if "=" in line:
                    k, v = (p.strip() for p in line.split("=", 1))
                    vals[k] = v
    except OSError:
        return None
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    if not batched and vals.get("plain_schedule") != plain_schedule:
        return None
    key = "batched_bytes_per_launch" if batched else "bytes_per_launch"
    v = vals.get(f"{key}[{kernel}]")
    return float(v) if v is not None else None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_baseline(imgs_np, split: int, budget_s: float):
    from oracle import native
    done, t0 = 0, time.perf_counter()
    for img in imgs_np:
        native.hough4_u8(img, split)
        done += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    R, C = imgs_np.shape[1:]
    return {"value": round(done * R * C / dt / 1e6, 3), "unit": "Mpixel/s",
            "cores": native.num_threads(), "kind": "oracle",
            "sample": f"{done} of {len(imgs_np)} images {R}x{C}, 4 quadrants, direct sums along "
                      f"the generating patterns (C, OpenMP), {dt:.1f} s",
            "cpu_model": cpu_model()}


def _cpu_alg1(imgs_np, split: int, budget_s: float):
    """Alg. 1's own recursion in C (O(W H log W) per quadrant, OpenMP over
    images and quadrants): the like-for-like CPU counterpart of the GPU path,
    over all the images, repeated while the budget lasts."""
    from oracle import native
    native.alg1_u8_batch(imgs_np[:2], split)  # warm: pages, threads
    reps, t0 = 0, time.perf_counter()
    while True:
        native.alg1_u8_batch(imgs_np, split)
        reps += 1
        if time.perf_counter() - t0 >= budget_s:
            break
    dt = time.perf_counter() - t0
    n, R, C = imgs_np.shape
    return {"value": round(reps * n * R * C / dt / 1e6, 1), "unit": "Mpixel/s",
            "cores": native.num_threads(), "kind": "alg1_recursion",
            "sample": f"{reps} x {n} images {R}x{C}, 4 quadrants, int32, {dt:.1f} s",
            "cpu_model": cpu_model()}


def _peaks(torch, F, WL):
    """Peak finding after the transform (device time of the fht_peaks call,
    events around it): the planted segments of a 1021 x 1021 edge map, and
    k = 4096 peaks of a uniform 1021 x 1021 image (about 137 000 candidates)."""
    import numpy as np
    res = {}
    for name, kind, k, radius, floor in (("edge_map_1021_k80_r8", "edge", 80, 8, 120.0),
                                         ("uniform_1021_k4096_r2", "u8", 4096, 2, 0.0)):
        rng = WL.rng_for(2, salt=50)
        img = WL.edge_map(rng, 1021, 1021) if kind == "edge" else WL.uniform_u8(rng, 1021, 1021)
        plan = F.Plan(1021, 1021, "u8", "S")
        out = plan.new_out("cuda")
        plan.forward(torch.from_numpy(np.ascontiguousarray(img)).cuda(), out)
        cap = 1 << 20
        ws = torch.empty(F.fht_peaks_workspace_bytes(cap), dtype=torch.uint8, device="cuda")
        rec = torch.empty(k * F.PEAK_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        found = torch.zeros(2, dtype=torch.int32, device="cuda")
        sh = torch.cuda.current_stream().cuda_stream

        def call():
            F.fht_peaks(plan.handle, out.data_ptr(), k, radius, floor, cap, ws.data_ptr(),
                        rec.data_ptr(), found.data_ptr(), sh)

        call()
        torch.cuda.synchronize()
        a, b = _events(torch)
        a.record()
        for _ in range(5):
            call()
        b.record()
        torch.cuda.synchronize()
        n, cands = (int(v) for v in found.cpu())
        res[name] = {"ms": round(a.elapsed_time(b) / 5, 4), "k": k, "radius": radius,
                     "peaks": n, "candidates": cands}
    return res


def _latency_config1(torch, F, WL, reps: int = 400):
    """One 61 x 47 uint8 image (the smallest workload): latency of single
    transforms, each launched alone and waited for, under each schedule for
    per-image launches (their outputs must agree); the faster is reported."""
    import numpy as np
    from paper_2411_07351_amd import tuning as T
    img = torch.from_numpy(WL.uniform_u8(WL.rng_for(1), 61, 47)).cuda()
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    pct = lambda v, p: round(float(np.percentile(v, p)), 4)
    runs, ref = {}, None
    for name, sched in T.PLAIN_SCHEDULES.items():
        plan = F.Plan(61, 47, "u8", "S", schedule=sched)
        out = plan.new_out("cuda")
        ws = plan.new_ws("cuda")
        for _ in range(20):
            F.fht_forward(plan.handle, img.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
        torch.cuda.synchronize()
        if ref is None:
            ref = out.clone()
        elif not torch.equal(ref, out):
            raise RuntimeError(f"schedule {name!r} changed the 61x47 transform")
        gpu, host = [], []
        for _ in range(reps):
            a, b = _events(torch)
            t0 = time.perf_counter()
            a.record(stream)
            F.fht_forward(plan.handle, img.data_ptr(), out.data_ptr(), ws.data_ptr(), sh)
            b.record(stream)
            b.synchronize()
            host.append((time.perf_counter() - t0) * 1e3)
            gpu.append(a.elapsed_time(b))
        runs[name] = {"launches": F.fht_plan_num_launches(plan.handle),
                      "gpu_ms": {"p50": pct(gpu, 50), "p99": pct(gpu, 99)},
                      "host_ms": {"p50": pct(host, 50), "p99": pct(host, 99)}}
    best = min(runs, key=lambda k: runs[k]["gpu_ms"]["p50"])
    return {"workload": "one 61x47 uint8 image, 4 quadrants, FHT2DS, int32 outputs, "
                        f"{runs[best]['launches']} launch(es), each transform launched alone "
                        "and waited for",
            "seed": WL.SEED_BASE + 1,
            "reps": reps,
            "schedule": best,
            "gpu_ms": runs[best]["gpu_ms"],
            "host_ms": runs[best]["host_ms"],
            "by_schedule": runs}


def _ceilings(torch, mib: int = 2048):
    """Practical HBM rates on this part: torch's fill (write only), copy and
    sum (read only) over buffers much larger than the 256 MB memory-side
    cache, timed with events."""
    n = mib << 20
    a = torch.empty(n, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    x = a.view(torch.float32)
    stream = torch.cuda.current_stream()

    def rate(fn, nbytes):
        for _ in range(2):
            fn()
        e0, e1 = _events(torch)
        e0.record(stream)
        for _ in range(5):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return round(nbytes * 5 / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)

    res = {"write_gbps": rate(lambda: a.fill_(1), n),
           "copy_gbps": rate(lambda: b.copy_(a), 2 * n),
           "read_gbps": rate(lambda: x.sum(), n),
           "buffer_mib": mib, "how": "torch fill_, copy_, sum over uint8/float32 buffers"}
    del a, b, x
    torch.cuda.empty_cache()
    return res


def _serving(args, torch, F, WL):
    """Poisson request stream through the continuous-batching server: a
    closed burst measures capacity, then Poisson arrivals at 50 % and 80 % of
    it and at a fixed rate give p50/p99 latency (arrival to completion)."""
    import numpy as np

    from paper_2411_07351_amd import serving as S

    n = args.serve_requests
    # every run serves requests of its own (fresh shapes, so the plan cache is
    # warm only for lane counts seen before, as in a running server)
    sets = []
    for k in range(4):
        items = WL.serving_requests(WL.rng_for(5, salt=k), n, 64, 4096)
        sets.append((items, [torch.from_numpy(img).pin_memory() for _, img in items]))
    # one burst of its own first: the runtime, allocators and planner threads
    # are warm, as in a running server (its shapes mostly differ from the
    # measured runs', so their plans are still made cold)
    warm = WL.serving_requests(WL.rng_for(5, salt=9), n, 64, 4096)
    warm_imgs = [torch.from_numpy(img).pin_memory() for _, img in warm]
    cfg = dict(max_batch_images=64, max_batch_px=32 << 20, depth=2,
               plan_threads=min(16, os.cpu_count() or 1), keep_outputs=False)
    budget = 32 << 30

    def run(images, arrivals):
        reqs = [S.Request(i, im, float(t)) for i, (im, t) in enumerate(zip(images, arrivals))]
        srv = S.Server(S.GpuExecutor(streams=2), budget, **cfg)
        try:
            srv.run(reqs)
        finally:
            srv.close()
        torch.cuda.synchronize()
        out = S.summarize(reqs)
        out["peak_admitted_gb"] = round(srv.peak_in_use / 1e9, 2)
        out["batches"] = srv.batches
        out["max_batch"] = max(srv.batch_sizes) if srv.batch_sizes else 0
        return out

    run(warm_imgs, np.zeros(len(warm_imgs)))
    cap = run(sets[0][1], np.zeros(n))
    rng = np.random.default_rng(WL.SEED_BASE + 5 + 7)
    runs = []
    for k, (label, qps) in enumerate((("50% of capacity", 0.5 * cap["req_per_s"]),
                                      ("80% of capacity", 0.8 * cap["req_per_s"]),
                                      ("fixed", args.serve_qps)), start=1):
        res = run(sets[k][1], WL.poisson_arrivals(rng, n, qps))
        runs.append({"qps": round(qps, 1), "load": label, **res})
    shapes = [tuple(im.shape) for im in sets[0][1]]
    return {
        "workload": f"{n} requests per run (a fresh set each run), sides log-uniform in "
                    "[64, 4096], 70% uint8 edge maps / 30% float32 N(0,1), Poisson arrivals, "
                    "4 quadrants, FHT2DS",
        "seed": f"{WL.SEED_BASE} + 5 + 1000 k for run k (0: capacity, 1-3: the rates; 9: warm-up)",
        "mpixels": round(sum(r * c for r, c in shapes) / 1e6, 1),
        "shape_histogram": _side_histogram(shapes),
        "u8_requests": sum(k == "u8" for k, _ in sets[0][0]),
        "hbm_budget_gb": budget / 1e9,
        "streams": 2, **{k: v for k, v in cfg.items() if k != "keep_outputs"},
        "capacity": cap,
        "runs": runs,
    }


def _differentiable(args, torch, F, WL):
    """Forward transform plus hand-written adjoint (the backward pass of
    ``HoughFunction``) of float32 384 x 257 N(0,1) images, per image."""
    import numpy as np

    n, R, C = args.diff_images, 384, 257
    rng = WL.rng_for(4)
    imgs = torch.from_numpy(np.stack([WL.normal_f32(rng, R, C) for _ in range(n)])).cuda()
    plan = F.Plan(R, C, "f32", "S")
    outs = torch.empty((n, plan.out_elems), dtype=torch.float32, device="cuda")
    gouts = torch.from_numpy(rng.standard_normal((n, plan.out_elems)).astype(np.float32)).cuda()
    gimgs = torch.empty_like(imgs)
    fws = plan.new_ws("cuda")
    aws = torch.empty(max(F.fht_plan_adjoint_workspace_bytes(plan.handle), 1), dtype=torch.uint8,
                      device="cuda")
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    def fwd():
        for i in range(n):
            F.fht_forward(plan.handle, imgs[i].data_ptr(), outs[i].data_ptr(), fws.data_ptr(), sh)

    def bwd():
        for i in range(n):
            F.fht_adjoint(plan.handle, gouts[i].data_ptr(), gimgs[i].data_ptr(), aws.data_ptr(), sh)

    def timed(fn):
        for _ in range(args.warmup):
            fn()
        a, b = _events(torch)
        a.record(stream)
        for _ in range(args.steps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / args.steps

    # the same batch as one tensor: one launch per pass / level for all images
    mws = torch.empty(max(F.fht_plan_workspace_bytes_many(plan.handle, n), 1), dtype=torch.uint8,
                      device="cuda")
    maws = torch.empty(max(F.fht_plan_adjoint_workspace_bytes_many(plan.handle, n), 1),
                       dtype=torch.uint8, device="cuda")

    def fwd_many():
        plan.forward_many(imgs, outs, mws)

    def bwd_many():
        plan.adjoint_many(gouts, gimgs, maws)

    f_ms, b_ms = timed(fwd), timed(bwd)
    fb_ms = timed(lambda: (fwd(), bwd()))
    mf_ms, mb_ms = timed(fwd_many), timed(bwd_many)
    mfb_ms = timed(lambda: (fwd_many(), bwd_many()))
    px = n * R * C
    fbytes = n * sum(sum(F.fht_plan_launch_info(plan.handle, l)[k] for k in ("bytes_in", "bytes_out"))
                     for l in range(F.fht_plan_num_launches(plan.handle)))
    comp = COMPULSORY_BPP_F32_FWD_ADJ * px
    return {"workload": f"{n} float32 {R}x{C} N(0,1) images, forward + adjoint, 4 quadrants, "
                        "one launch per pass or level for the whole batch",
            "seed": WL.SEED_BASE + 4,
            "value": round(px / (mfb_ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
            "roofline": {"bound": "hbm", "unit": "GB/s", "peak": HBM_PEAK_GBPS,
                         "compulsory_bytes": comp,
                         "achieved_compulsory": round(comp / (mfb_ms * 1e-3) / 1e9, 1),
                         "frac_compulsory": round(comp / (mfb_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
                         "forward_bytes_scheduled": fbytes,
                         "forward_gbps_scheduled": round(fbytes / (mf_ms * 1e-3) / 1e9, 1),
                         "working_set_mb": round((px * 4 + 2 * n * plan.out_elems * 4 +
                                                  mws.numel() + maws.numel()) / 1e6, 1),
                         "note": "the working set fits the 256 MB memory-side cache, so these "
                                 "rates are not HBM-only"},
            "forward_ms": round(mf_ms, 4), "adjoint_ms": round(mb_ms, 4),
            "forward_adjoint_ms": round(mfb_ms, 4),
            "per_image": {"value": round(px / (fb_ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
                          "forward_ms": round(f_ms, 4), "adjoint_ms": round(b_ms, 4),
                          "forward_adjoint_ms": round(fb_ms, 4)},
            # every gather pass but the last, plus the final launch (the last
            # gathers fused with the sum into the image gradient)
            "adjoint_launches": max(1, max(F.fht_plan_adjoint_num_passes(plan.handle, v)
                                           for v in (0, 1)))}


def _side_histogram(shapes) -> dict:
    """Images per octave of their larger side, e.g. {"<=64": 12, "<=128": 40, ...}."""
    hist = {}
    for r, c in shapes:
        k = 1 << max(0, (max(r, c) - 1).bit_length())
        hist[k] = hist.get(k, 0) + 1
    return {f"<={k}": hist[k] for k in sorted(hist)}


def _ragged_tuned(args, torch, F, shapes, rimgs, routs, rpx, stream):
    """The ragged batch with a schedule per size class from the autotuner
    (tuned here, outside the timed region, unless the cache already holds the
    classes), replayed from a HIP graph like the default-schedule batch."""
    import tempfile

    from paper_2411_07351_amd import tuning as T
    cache_dir = None
    if "FHT_AUTOTUNE_CACHE" not in os.environ:
        cache_dir = tempfile.mkdtemp(prefix="fht_tune_")
        os.environ["FHT_AUTOTUNE_CACHE"] = os.path.join(cache_dir, "tune.json")
    try:
        scheds = T.autotune(rimgs, "S" if args.split == "S" else "T")
        report = T.last_report
        plans = T.plans_for(shapes, "u8", args.split, scheds)
        batch = F.Batch(plans, rimgs, routs)
        ws = batch.new_ws(rimgs[0].device)
        graph = batch.capture(ws)
        for _ in range(args.warmup):
            graph.replay()
        torch.cuda.synchronize()
        a, b = _events(torch)
        a.record(stream)
        for _ in range(args.steps):
            graph.replay()
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.steps
        changed = {}
        for cls, sc in sorted(scheds.items()):
            diff = {k: v for k, v in sc.items() if T.DEFAULT.get(k) != v}
            if diff:
                changed[cls] = diff
        cls_rep = report["classes"].values()
        return {"value": round(rpx / (ms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
                "ms_per_step": round(ms, 3), "graph": True, "launches": batch.num_launches,
                "classes": len(scheds),
                "classes_tuned": sum(1 for r in cls_rep if r["source"] == "tuned"),
                "tune_seconds": report["seconds"],
                "class_ms_default_vs_tuned_alone": [
                    round(sum(r.get("default_ms") or 0 for r in cls_rep), 3),
                    round(sum(r.get("ms") or 0 for r in cls_rep), 3)],
                "in_batch": report["batch"],
                "schedules_changed": changed}
    finally:
        if cache_dir:
            del os.environ["FHT_AUTOTUNE_CACHE"]


def _events(torch):
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): several GPUs would each "
              "transform their own share of the images, with no exchange, and that is not "
              "implemented.", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    import paper_2411_07351_amd as F
    import workloads as WL

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    split = 0 if args.split == "S" else 1
    n, R, C = args.images, args.rows, args.cols
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream

    imgs_np = WL.edge_maps(WL.rng_for(2), n, R, C)
    imgs = torch.from_numpy(imgs_np).to(dev)
    plan = F.Plan(R, C, "u8", split)  # the batched legs: library default schedule
    outs = torch.empty((n, plan.out_elems), dtype=torch.int32, device=dev)
    px_per_step = n * R * C

    # The per-image launches' schedule (untimed): each candidate transforms
    # 16 of the images, and they must agree on every output.
    from paper_2411_07351_amd import tuning as T
    if args.plain_schedule == "auto":
        pname, ptimes = T.tune_plain([imgs[i] for i in range(min(n, 16))], args.split)
    else:
        pname, ptimes = args.plain_schedule, None
    psched = T.PLAIN_SCHEDULES[pname]
    pplan = F.Plan(R, C, "u8", split, schedule=psched) if psched else plan
    ws = pplan.new_ws(dev)
    nl = F.fht_plan_num_launches(pplan.handle)
    info = [F.fht_plan_launch_info(pplan.handle, l) for l in range(nl)]

    def plain_step():
        for i in range(n):
            ip, op = imgs[i].data_ptr(), outs[i].data_ptr()
            for l in range(nl):
                F.fht_forward_launch(pplan.handle, l, ip, op, ws.data_ptr(), sh)

    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()

    # Timed region: K plain steps, bracketed by HIP events on the stream the
    # kernels run on (and by the host clock around synchronisations).
    a, b = _events(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    a.record(stream)
    for _ in range(args.steps):
        plain_step()
    b.record(stream)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    plain_event_ms = a.elapsed_time(b) / args.steps

    # Kernel durations: for each launch of the plan, the n images' launches
    # back to back between one pair of events on the same stream, K times.
    # Back-to-back launches of one kernel leave only the hardware's dispatch
    # gap between them, so the mean is the kernel's average duration.
    events = [[] for _ in range(nl)]
    for _ in range(args.steps):
        for l in range(nl):
            e = _events(torch)
            e[0].record(stream)
            for i in range(n):
                F.fht_forward_launch(pplan.handle, l, imgs[i].data_ptr(), outs[i].data_ptr(),
                                     ws.data_ptr(), sh)
            e[1].record(stream)
            events[l].append(e)
    torch.cuda.synchronize()
    launch_ms = [float(np.mean([x.elapsed_time(y) for x, y in ev])) / n for ev in events]
    dom = int(np.argmax(launch_ms))
    dom_bytes = info[dom]["bytes_in"] + info[dom]["bytes_out"]
    achieved = dom_bytes / (launch_ms[dom] * 1e-3) / 1e9
    dom_kernel = F.fht_plan_launch_kernel(pplan.handle, dom)
    traffic = _traffic(dom_kernel, plain_schedule=pname)

    value = px_per_step * args.steps / plain_s / 1e6
    result = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(plain_s / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": f"{n} x {R}x{C} uint8 edge maps (Bernoulli 0.05 + 20 segments), "
                        f"4 quadrants, FHT2D{args.split}, int32 outputs, plain per-image launches",
            "images": n, "rows": R, "cols": C, "split": args.split, "path": "plain",
            "launches_per_image": nl, "seed": WL.SEED_BASE + 2,
            "plain_schedule": pname, "plain_schedule_knobs": psched or "library default",
        },
        "plain_schedule_us_per_image": ptimes,
        "effective_gbps": round(COMPULSORY_BPP * px_per_step * args.steps / plain_s / 1e9, 1),
        "frac_compulsory": round(COMPULSORY_BPP * px_per_step * args.steps / plain_s / 1e9 /
                                 HBM_PEAK_GBPS, 4),
        "bytes_per_px_scheduled": round(sum(i["bytes_in"] + i["bytes_out"] for i in info) /
                                        (R * C), 2),
        "event_ms_per_step": round(plain_event_ms, 3),
        "roofline": {
            "bound": "hbm",
            "kernel": dom_kernel,
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": round(traffic, 0) if traffic is not None else None,
            "traffic_note": "FETCH_SIZE + WRITE_SIZE per launch (profiles/), scaled by a 1 GiB "
                            "device copy; these count L2<->fabric requests, hits in the 256 MB "
                            "memory-side cache included, and the plain path's working set (one "
                            "image, its output, a reused workspace) fits that cache",
            "bytes_per_launch": dom_bytes,
            "avg_launch_us": round(launch_ms[dom] * 1e3, 2),
            "launch_avg_us": [round(m * 1e3, 2) for m in launch_ms],
            "launch_bytes": [i["bytes_in"] + i["bytes_out"] for i in info],
            "launch_kernels": [F.fht_plan_launch_kernel(pplan.handle, l) for l in range(nl)],
            "kernel_source_hash": kernel_source_hash(),
            "schedule_note": ("the dominant kernel of the per-image schedule in use; the two-pass "
                              "schedule's 6-level first pass moves the same bytes as the default's "
                              "5-level one in more time, but saves the third launch per image"
                              if pname == "two-pass" else "library default schedule"),
        },
    }

    # Batched: one launch per fused pass for all images, replayed from a graph.
    batch = F.Batch([plan] * n, [imgs[i] for i in range(n)], [outs[i] for i in range(n)])
    bws = batch.new_ws(dev)
    graph = batch.capture(bws)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    a, b = _events(torch)
    a.record(stream)
    for _ in range(args.steps):
        graph.replay()
    b.record(stream)
    torch.cuda.synchronize()
    bms = a.elapsed_time(b) / args.steps
    per = [[] for _ in range(batch.num_launches)]
    for _ in range(3):
        for l in range(batch.num_launches):
            e = _events(torch)
            e[0].record(stream)
            F.fht_batch_run_launch(batch.handle, l, bws.data_ptr(), sh)
            e[1].record(stream)
            per[l].append(e)
    torch.cuda.synchronize()
    per_ms = [float(np.median([x.elapsed_time(y) for x, y in ev])) for ev in per]
    binfo = [F.fht_plan_launch_info(plan.handle, l)
             for l in range(F.fht_plan_num_launches(plan.handle))]
    lbytes = [n * (i["bytes_in"] + i["bytes_out"]) for i in binfo]
    result["batched"] = {
        "value": round(px_per_step / (bms * 1e-3) / 1e6, 1),
        "unit": "Mpixel/s",
        "ms_per_step": round(bms, 4),
        "graph": True,
        "effective_gbps": round(COMPULSORY_BPP * px_per_step / (bms * 1e-3) / 1e9, 1),
        "frac_compulsory": round(COMPULSORY_BPP * px_per_step / (bms * 1e-3) / 1e9 /
                                 HBM_PEAK_GBPS, 4),
        "launch_ms": [round(m, 4) for m in per_ms],
        "launch_gbps": ([round(by / (m * 1e-3) / 1e9, 1) for by, m in zip(lbytes, per_ms)]
                        if len(per_ms) == len(lbytes) else None),
        "path_gbps": round(sum(lbytes) / (bms * 1e-3) / 1e9, 1),
        "path_frac": round(sum(lbytes) / (bms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
    }
    traf = [_traffic(F.fht_plan_launch_kernel(plan.handle, l), batched=True)
            for l in range(len(binfo))]
    if all(t is not None for t in traf):
        result["batched"]["launch_traffic_bytes"] = [round(t, 0) for t in traf]
        result["batched"]["traffic_gbps"] = round(sum(traf) / (bms * 1e-3) / 1e9, 1)
        result["batched"]["traffic_frac"] = round(sum(traf) / (bms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4)
    result["batched"]["working_set_mb"] = round((imgs.numel() + outs.numel() * 4 +
                                                 bws.numel()) / 1e6, 1)
    del graph, batch, bws

    if args.ragged > 0:
        rng = WL.rng_for(3)
        shapes = WL.ragged_shapes(rng, args.ragged, 32, 2048)
        rimgs = [torch.from_numpy(WL.edge_map(rng, r, c)).to(dev) for r, c in shapes]
        cache = {}
        rplans = []
        for r, c in shapes:
            if (r, c) not in cache:
                cache[(r, c)] = F.Plan(r, c, "u8", split)
            rplans.append(cache[(r, c)])
        routs = [p.new_out(dev) for p in rplans]
        rpx = sum(r * c for r, c in shapes)
        rb = F.Batch(rplans, rimgs, routs)
        rws = rb.new_ws(dev)
        rgraph = rb.capture(rws)
        for _ in range(args.warmup):
            rgraph.replay()
        torch.cuda.synchronize()
        a, b = _events(torch)
        a.record(stream)
        for _ in range(args.steps):
            rgraph.replay()
        b.record(stream)
        torch.cuda.synchronize()
        rbms = a.elapsed_time(b) / args.steps
        pws = torch.empty(max(p.ws_bytes for p in rplans) + 1, dtype=torch.uint8, device=dev)

        def ragged_plain():
            for p, im, o in zip(rplans, rimgs, routs):
                F.fht_forward(p.handle, im.data_ptr(), o.data_ptr(), pws.data_ptr(), sh)

        ragged_plain()
        torch.cuda.synchronize()
        psteps = max(1, args.steps // 3)
        t0 = time.perf_counter()
        for _ in range(psteps):
            ragged_plain()
        torch.cuda.synchronize()
        rpms = (time.perf_counter() - t0) / psteps * 1e3
        result["ragged"] = {
            "workload": f"{args.ragged} uint8 edge maps, sides log-uniform in [32, 2048], "
                        "4 quadrants, int32 outputs",
            "seed": WL.SEED_BASE + 3,
            "mpixels": round(rpx / 1e6, 2),
            "shape_histogram": _side_histogram(shapes),
            "batched": {"value": round(rpx / (rbms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
                        "ms_per_step": round(rbms, 3), "graph": True,
                        "launches": rb.num_launches, "schedule": "library default"},
            "plain": {"value": round(rpx / (rpms * 1e-3) / 1e6, 1), "unit": "Mpixel/s",
                      "ms_per_step": round(rpms, 3)},
        }
        del rgraph, rb, rws, pws
        if args.tune:
            # tuned last, after the other legs: tuning plans hundreds of
            # schedules, which fills the process-wide program cache
            tune_leg = (shapes, rimgs, routs, rpx)
        else:
            del routs, rimgs

    if args.diff_images > 0:
        result["differentiable"] = _differentiable(args, torch, F, WL)

    if args.serve_requests > 0:
        result["serving"] = _serving(args, torch, F, WL)

    if args.copy_mib > 0:
        # A plain device copy of known size, for calibrating byte counters.
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        result["copy_calibration_bytes"] = 2 * (args.copy_mib << 20)

    result["latency_61x47"] = _latency_config1(torch, F, WL)
    result["peaks"] = _peaks(torch, F, WL)
    if args.ragged > 0 and args.tune:
        result["ragged"]["batched_tuned"] = _ragged_tuned(args, torch, F, *tune_leg, stream)
        del tune_leg
    if args.ceilings:
        result["hbm_ceilings"] = _ceilings(torch)

    if args.cpu_seconds > 0:
        result["cpu_baseline"] = _cpu_baseline(imgs_np, split, args.cpu_seconds)
        result["cpu_alg1"] = _cpu_alg1(imgs_np, split, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
