#!/usr/bin/env python3
"""Throughput of the dyadic-pattern fast Hough transform on one MI355X.

Workload (one "step"): a batch of 64 uint8 edge maps of 1021 x 1021
(Bernoulli(0.05) background plus 20 Bresenham segments, seed 2411_07351 + 2),
all four quadrant Hough images with int32 accumulators, FHT2DS split.  The
headline path launches each image separately (``fht_forward_launch`` for every
fused pass); the same batch also runs batched (``fht_batch_run``: one launch
per fused pass for all 64 images).  Inputs are resident in HBM before timing.

Prints one JSON line.  ``--gpus`` above 1 is rejected: this build runs on one
GPU (images would be sharded across GPUs with no exchange).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "input Mpixel/s + achieved HBM GB/s (batched vs plain); p50/p99 latency at fixed QPS"


def _parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--images", type=int, default=64)
    ap.add_argument("--rows", type=int, default=1021)
    ap.add_argument("--cols", type=int, default=1021)
    ap.add_argument("--split", default="S", choices=["S", "T"])
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU oracle sample budget (0 disables the cpu_baseline leg)")
    ap.add_argument("--no-batched", action="store_true")
    return ap.parse_args()


def _launch_bytes(plan, launch: int, in_bytes: int) -> int:
    """Algorithmic HBM bytes of one launch of one image: compulsory reads + writes.

    The first launch reads the image once and writes one accumulator per
    output element of every quadrant; a later launch reads the previous pass's
    accumulators and writes the next ones (4 bytes each).
    """
    elems = plan.out_elems
    acc = 4
    if launch == 0:
        return plan.rows * plan.cols * in_bytes + elems * acc
    return 2 * elems * acc


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
    return {"value": done * R * C / dt / 1e6, "unit": "Mpixel/s", "cores": native.num_threads(),
            "kind": "oracle",
            "sample": f"{done} of {len(imgs_np)} images {R}x{C}, 4 quadrants, direct pattern sums "
                      f"(C, OpenMP), {dt:.1f} s"}


def main():
    args = _parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); images would be sharded "
              "across GPUs with no exchange, which this build does not do.", file=sys.stderr)
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

    imgs_np = WL.edge_maps(WL.rng_for(2), n, R, C)
    imgs = torch.from_numpy(imgs_np).to(dev)
    plan = F.Plan(R, C, "u8", split)
    outs = torch.empty((n, plan.out_elems), dtype=torch.int32, device=dev)
    ws = plan.new_ws(dev)
    nl = F.fht_plan_num_launches(plan.handle)
    stream = torch.cuda.current_stream()
    sh = stream.cuda_stream
    px_per_step = n * R * C

    def plain_step(events=None):
        for i in range(n):
            ip, op = imgs[i].data_ptr(), outs[i].data_ptr()
            for l in range(nl):
                if events is not None:
                    events[l].append((torch.cuda.Event(enable_timing=True),
                                      torch.cuda.Event(enable_timing=True)))
                    events[l][-1][0].record(stream)
                F.fht_forward_launch(plan.handle, l, ip, op, ws.data_ptr(), sh)
                if events is not None:
                    events[l][-1][1].record(stream)

    for _ in range(args.warmup):
        plain_step()
    torch.cuda.synchronize()

    # Timed region: K plain steps, every launch bracketed by HIP events on the
    # stream it runs on.
    events = [[] for _ in range(nl)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step(events)
    torch.cuda.synchronize()
    plain_s = time.perf_counter() - t0
    launch_ms = [float(np.mean([a.elapsed_time(b) for a, b in ev])) for ev in events]
    launch_total = [m * len(ev) for m, ev in zip(launch_ms, events)]
    dom = int(np.argmax(launch_total))
    dom_bytes = _launch_bytes(plan, dom, 1)
    achieved = dom_bytes / (launch_ms[dom] * 1e-3) / 1e9

    # Same steps without per-launch events (launch overhead of the events themselves).
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plain_step()
    torch.cuda.synchronize()
    plain_noev_s = time.perf_counter() - t0

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
                        f"4 quadrants, FHT2D{args.split}, int32, plain per-image launches",
            "images": n, "rows": R, "cols": C, "split": args.split, "path": "plain",
            "launches_per_image": nl,
        },
        "effective_gbps": round(17 * px_per_step * args.steps / plain_s / 1e9, 1),
        "plain_without_events_mpx_s": round(px_per_step * args.steps / plain_noev_s / 1e6, 1),
        "roofline": {
            "bound": "hbm",
            "kernel": f"launch {dom} of {nl} (fht_pass_kernel, "
                      f"{'image' if dom == 0 else 'accumulator'} input)",
            "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4),
            "traffic": None,
            "bytes_per_launch": dom_bytes,
            "avg_launch_us": round(launch_ms[dom] * 1e3, 2),
            "launch_avg_us": [round(m * 1e3, 2) for m in launch_ms],
        },
    }

    if not args.no_batched:
        batch = F.Batch([plan] * n, [imgs[i] for i in range(n)], [outs[i] for i in range(n)])
        bws = batch.new_ws(dev)
        bl = batch.num_launches
        for _ in range(args.warmup):
            batch.run(bws)
        torch.cuda.synchronize()
        bev = [[] for _ in range(bl)]
        t0 = time.perf_counter()
        for _ in range(args.steps):
            for l in range(bl):
                a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                a.record(stream)
                F.fht_batch_run_launch(batch.handle, l, bws.data_ptr(), sh)
                b.record(stream)
                bev[l].append((a, b))
        torch.cuda.synchronize()
        bs = time.perf_counter() - t0
        bms = [float(np.mean([a.elapsed_time(b) for a, b in ev])) for ev in bev]
        bbytes = [n * _launch_bytes(plan, l, 1) for l in range(bl)]
        bgbps = [by / (m * 1e-3) / 1e9 for by, m in zip(bbytes, bms)]
        result["batched"] = {
            "value": round(px_per_step * args.steps / bs / 1e6, 1),
            "unit": "Mpixel/s",
            "ms_per_step": round(bs / args.steps * 1e3, 3),
            "launch_avg_us": [round(m * 1e3, 2) for m in bms],
            "launch_achieved_gbps": [round(g, 1) for g in bgbps],
            "launch_frac": [round(g / HBM_PEAK_GBPS, 4) for g in bgbps],
            "effective_gbps": round(17 * px_per_step * args.steps / bs / 1e9, 1),
        }
        del batch

    if args.cpu_seconds > 0:
        result["cpu_baseline"] = _cpu_baseline(imgs_np, split, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
