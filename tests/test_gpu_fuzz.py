"""Seeded fuzz of the GPU paths against the oracle: random shapes, dtypes,
split rules, quadrant subsets and schedules (forward), mixed-size batches,
and the adjoint of single images and same-shape batches.

Integer outputs must match bit for bit; float outputs must stay within the
per-line bound (1e-5 of the line's absolute sum for float32, 1e-12 for
float64).  Small cases are compared in full with the C oracle; larger ones on
sampled outputs the oracle computes one by one.
"""
import numpy as np
import pytest
import torch

import paper_2411_07351_amd as F
import workloads as WL
from oracle import fht_oracle as O
from oracle import native

pytestmark = pytest.mark.gpu

SCHEDULES = [None, None, None,
             dict(first_levels=4, max_levels=3, t_tile=8),
             dict(first_levels=6, max_levels=2, s_tile=256, lds_budget=98304),
             dict(first_levels=5, max_levels=4, t_tile=32, threads=256, threads_first=256),
             dict(s_tile_first=64, s_tile=128, max_levels=5),
             dict(first_levels=6, max_levels=4, lds_budget=163840)]  # the per-image two-pass
SUBSETS = [(0, 1, 2, 3), (0, 1, 2, 3), (0, 1, 2, 3), (0,), (1, 3), (2, 3), (0, 2)]
FULL_WORK = 3e9  # oracle work (R * C * (R + C)) up to which every output is compared


def _image(rng, kind, R, C):
    if kind == "u8":
        return WL.uniform_u8(rng, R, C)
    img = WL.normal_f32(rng, R, C)
    return img if kind == "f32" else img.astype(np.float64)


def _check(img, split, quadrants, got, rng):
    """Compare the quadrant outputs `got` (in `quadrants` order) with the oracle."""
    R, C = img.shape
    shapes = {q: ((R, C) if q < 2 else (C, R)) for q in range(4)}
    if R * C * (R + C) <= FULL_WORK:
        if img.dtype == np.uint8:
            ref = native.hough4_u8(img, split)
            for g, q in zip(got, quadrants):
                assert (g == ref[q]).all(), (R, C, split, q)
        else:
            ref, ab = native.hough4_f64(img.astype(np.float64), split)
            tol = 1e-5 if img.dtype == np.float32 else 1e-12
            for g, q in zip(got, quadrants):
                assert (np.abs(g.astype(np.float64) - ref[q]) <= tol * ab[q] + 1e-30).all(), \
                    (R, C, split, q)
        return
    for g, q in zip(got, quadrants):
        W, H = shapes[q]
        n = 300
        t = rng.integers(0, W, n).astype(np.int32)
        s = rng.integers(0, H, n).astype(np.int32)
        qq = np.full(n, q, dtype=np.int32)
        vals = g[t, s]
        if img.dtype == np.uint8:
            assert (vals == native.sample_u8(img, split, qq, t, s)).all(), (R, C, split, q)
        else:
            ref, ab = native.sample_f64(img.astype(np.float64), split, qq, t, s)
            tol = 1e-5 if img.dtype == np.float32 else 1e-12
            assert (np.abs(vals.astype(np.float64) - ref) <= tol * ab + 1e-30).all(), \
                (R, C, split, q)


def test_fuzz_forward():
    rng = np.random.default_rng(WL.SEED_BASE + 71)
    for i in range(36):
        kind = ["u8", "u8", "u8", "f32", "f32", "f64"][i % 6]
        hi = 300 if kind == "f64" else 2600
        R, C = (int(v) for v in np.exp(rng.uniform(0.0, np.log(hi), size=2)))
        split = int(rng.integers(0, 2))
        quadrants = SUBSETS[int(rng.integers(0, len(SUBSETS)))]
        sched = SCHEDULES[int(rng.integers(0, len(SCHEDULES)))]
        img = _image(rng, kind, R, C)
        try:
            plan = F.Plan(R, C, kind, "S" if split == 0 else "T", quadrants, sched)
        except F.FhtError:
            assert sched is not None  # only a custom schedule may fail to fit
            continue
        out = plan.new_out()
        plan.forward(torch.from_numpy(img).cuda(), out)
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in plan.split_out(out)]
        _check(img, split, quadrants, got, rng)


def test_fuzz_forward_two_pass_schedule():
    # the schedule bench.py's per-image launches may pick, on random shapes
    rng = np.random.default_rng(WL.SEED_BASE + 76)
    for i in range(12):
        kind = ["u8", "u8", "f32"][i % 3]
        R, C = (int(v) for v in np.exp(rng.uniform(0.0, np.log(2600), size=2)))
        split = int(rng.integers(0, 2))
        img = _image(rng, kind, R, C)
        plan = F.Plan(R, C, kind, split, schedule=SCHEDULES[-1])
        out = plan.new_out()
        plan.forward(torch.from_numpy(img).cuda(), out)
        torch.cuda.synchronize()
        _check(img, split, (0, 1, 2, 3), [o.cpu().numpy() for o in plan.split_out(out)], rng)


@pytest.mark.parametrize("kind", ["u8", "f32"])
def test_fuzz_batches(kind):
    rng = np.random.default_rng(WL.SEED_BASE + 72 + (kind == "f32"))
    for _ in range(3):
        n = int(rng.integers(8, 25))
        split = int(rng.integers(0, 2))
        imgs_np = [_image(rng, kind, *(int(v) for v in np.exp(rng.uniform(0.0, np.log(1200), 2))))
                   for _ in range(n)]
        imgs = [torch.from_numpy(i).cuda() for i in imgs_np]
        plans = [F.Plan(i.shape[0], i.shape[1], kind, split) for i in imgs_np]
        outs = [p.new_out() for p in plans]
        batch = F.Batch(plans, imgs, outs)
        ws = batch.new_ws()
        batch.run(ws)
        torch.cuda.synchronize()
        for img, p, o in zip(imgs_np, plans, outs):
            _check(img, split, (0, 1, 2, 3), [x.cpu().numpy() for x in p.split_out(o)], rng)


def test_fuzz_adjoint():
    rng = np.random.default_rng(WL.SEED_BASE + 74)
    for i in range(10):
        kind = "f32" if i % 2 == 0 else "f64"
        R, C = (int(v) for v in np.exp(rng.uniform(0.0, np.log(160), size=2)))
        split = int(rng.integers(0, 2))
        quadrants = SUBSETS[int(rng.integers(0, len(SUBSETS)))]
        plan = F.Plan(R, C, kind, "S" if split == 0 else "T", quadrants)
        dt = torch.float32 if kind == "f32" else torch.float64
        Gs = {q: rng.standard_normal(plan.shapes[q]) for q in quadrants}
        if kind == "f32":
            Gs = {q: G.astype(np.float32) for q, G in Gs.items()}
        g = torch.zeros(plan.out_elems, dtype=dt)
        for q, G in Gs.items():
            g[plan.offsets[q]:plan.offsets[q] + G.size] = torch.from_numpy(G.ravel())
        got = plan.adjoint(g.cuda())
        torch.cuda.synchronize()
        got = got.double().cpu().numpy()
        ref = O.adjoint4({q: G.astype(np.float64) for q, G in Gs.items()}, split, (R, C))
        scale = O.adjoint4({q: np.abs(G.astype(np.float64)) for q, G in Gs.items()}, split, (R, C))
        tol = 1e-5 if kind == "f32" else 1e-12
        assert (np.abs(got - ref) <= tol * np.maximum(scale, 1.0)).all(), (R, C, split, quadrants)


def test_fuzz_adjoint_many():
    # same-shape batches large enough for the fused final launch (at least
    # 256 tiles of 64 x 64) and one too small for it
    rng = np.random.default_rng(WL.SEED_BASE + 75)
    for (n, R, C, split) in ((12, 300, 260, 0), (3, 150, 70, 1), (9, 257, 384, 1)):
        plan = F.Plan(R, C, "f32", "S" if split == 0 else "T")
        gouts = rng.standard_normal((n, plan.out_elems)).astype(np.float32)
        got = plan.adjoint_many(torch.from_numpy(gouts).cuda())
        torch.cuda.synchronize()
        got = got.double().cpu().numpy()
        for b in (0, n - 1):  # the first and last image of the batch
            Gs = {q: gouts[b, plan.offsets[q]:plan.offsets[q] + W * H].reshape(W, H).astype(np.float64)
                  for q, (W, H) in plan.shapes.items()}
            ref = O.adjoint4(Gs, split, (R, C))
            scale = O.adjoint4({q: np.abs(G) for q, G in Gs.items()}, split, (R, C))
            assert (np.abs(got[b] - ref) <= 1e-5 * np.maximum(scale, 1.0)).all(), (n, R, C, b)
