"""Host logic: the planner's tile programs, executed on the CPU, equal the oracle.

No GPU: the tables are read through the C ABI (fht_plan_pass_tables) and run
by a small interpreter with the kernel's semantics (tests/plan_interp.py).
"""
import numpy as np
import pytest

import paper_2411_07351_amd as F
from oracle import fht_oracle as O
from plan_interp import run_plan_tables

SCHEDULES = [
    None,
    dict(s_tile=64, s_tile_first=64, first_levels=2, max_levels=2, lds_budget=8192, t_tile=0),
    dict(s_tile=128, s_tile_first=128, first_levels=3, max_levels=3, lds_budget=16384, t_tile=4),
    dict(s_tile=64, s_tile_first=256, first_levels=1, max_levels=1, lds_budget=65536, t_tile=0),
    dict(s_tile=256, s_tile_first=64, first_levels=6, max_levels=7, lds_budget=65536, t_tile=8),
]


def _plan(R, C, split, sched):
    return F.fht_plan_create(R, C, F.FHT_U8, split, 15, F.fht_schedule(**sched) if sched else None)


@pytest.mark.parametrize("split", [0, 1])
@pytest.mark.parametrize("sched", SCHEDULES)
def test_tables_equal_oracle(split, sched):
    rng = np.random.default_rng(21)
    shapes = [(1, 1), (1, 7), (7, 1), (2, 3), (5, 3), (13, 11), (17, 33), (61, 47), (64, 20),
              (33, 70)]
    for R, C in shapes:
        img = rng.integers(0, 256, size=(R, C), dtype=np.uint8)
        h = _plan(R, C, split, sched)
        try:
            ref = O.hough4(img, split)
            for q in range(4):
                got = run_plan_tables(h, img, q)
                assert (got == ref[q]).all(), (R, C, q, sched)
        finally:
            F.fht_plan_destroy(h)


@pytest.mark.parametrize("split", [0, 1])
def test_tables_large_widths_sampled(split):
    # Wide trees (several fused passes with the default schedule): compare full
    # outputs of the interpreter with the C oracle.
    from oracle import native
    rng = np.random.default_rng(22)
    # 300 and 4096 lanes: the last later pass takes one level more than the
    # schedule's three where that saves a pass (5 + 4 and 5 + 3 + 4 levels)
    for R, C in ((300, 9), (9, 257), (1021, 5), (4096, 3), (8191, 3)):
        img = rng.integers(0, 256, size=(R, C), dtype=np.uint8)
        h = F.fht_plan_create(R, C, F.FHT_U8, split, 15, None)
        if R in (300, 4096):
            assert F.fht_plan_num_passes(h, 0) == (2 if R == 300 else 3)
        try:
            ref = native.hough4_u8(img, split)
            for q in range(4):
                assert (run_plan_tables(h, img, q) == ref[q]).all(), (R, C, q)
        finally:
            F.fht_plan_destroy(h)


def test_pass_structure_1021():
    # Default schedule at 1021 lanes: a first pass of 5 levels (roots of at
    # most 32 lanes), then passes that reach the root; ping-pong workspace.
    h = F.fht_plan_create(1021, 1021, F.FHT_U8, 0, 15, None)
    try:
        n = F.fht_plan_num_passes(h, 0)
        assert n >= 2
        t0 = F.fht_plan_pass_tables(h, 0, 0)
        assert (t0["hdrs"][:, 6] == 0).all() and (t0["hdrs"][:, 7] <= 5).all()
        last = F.fht_plan_pass_tables(h, 0, n - 1)
        assert (last["hdrs"][:, 7] == 10).all()
        one = (1021 * 1021 * 4 + 255) // 256 * 256
        assert F.fht_plan_workspace_bytes(h) == 4 * min(n - 1, 2) * one
    finally:
        F.fht_plan_destroy(h)


def test_invalid_arguments():
    for args in ((0, 5), (5, 0), (-1, 5), (70000, 3)):
        with pytest.raises(F.FhtError) as e:
            F.fht_plan_create(args[0], args[1], F.FHT_U8, 0, 15, None)
        assert e.value.status == -1
    with pytest.raises(F.FhtError) as e:
        F.fht_plan_create(4, 4, 7, 0, 15, None)
    assert e.value.status == -2
    for mask in (0, 16):
        with pytest.raises(F.FhtError):
            F.fht_plan_create(4, 4, F.FHT_U8, 0, mask, None)
    with pytest.raises(F.FhtError):
        F.fht_plan_create(4, 4, F.FHT_U8, 2, 15, None)
    with pytest.raises(F.FhtError):
        F.fht_plan_create(4, 4, F.FHT_U8, 0, 15, F.fht_schedule(s_tile=96))


@pytest.mark.parametrize("split", ["S", "T"])
def test_plan_addition_count_equals_theorem1_count(split):
    # the library's order tree adds exactly what the oracle counts for Alg. 1
    # (Sec. 4); the fused kernels add at least that many
    sp = 0 if split == "S" else 1
    for R, C in [(1, 1), (1, 9), (9, 1), (61, 47), (384, 257), (1021, 1021), (1024, 1024),
                 (3, 3), (17, 17), (1451, 13), (4096, 5)]:
        plan = F.Plan(R, C, "u8", split)  # keep it alive while its handle is used
        w = F.fht_plan_work(plan.handle)
        expect = 2 * O.additions(R, sp, C) + 2 * O.additions(C, sp, R)
        assert w["adds_tree"] == expect, (R, C)
        assert w["adds_executed"] >= expect


def test_random_schedules_and_shapes():
    # Seeded fuzz over the schedule's knobs (within their documented ranges)
    # and shapes, both splits, uint8 and float element rules: every plan that
    # is accepted runs in the interpreter (which checks the kernel's
    # invariants: bounds, no read-after-write inside a step, single writes)
    # and equals the oracle.
    rng = np.random.default_rng(23)
    accepted = 0
    for _ in range(48):
        sched = dict(s_tile=int(rng.choice([64, 128, 192, 256])),
                     s_tile_first=int(rng.choice([64, 128, 192, 256])),
                     first_levels=int(rng.integers(1, 7)), max_levels=int(rng.integers(1, 9)),
                     lds_budget=int(rng.choice([4096, 16384, 65536, 98304])),
                     t_tile=int(rng.choice([0, 4, 8, 16, 32])),
                     threads=int(rng.choice([256, 512])), threads_first=int(rng.choice([256, 512])))
        R, C = (int(v) for v in np.exp(rng.uniform(0, np.log(600), size=2)))
        C = min(C, 40)  # positions: keep the interpreter quick
        split = int(rng.integers(0, 2))
        kind = [F.FHT_U8, F.FHT_F32][int(rng.integers(0, 2))]
        try:
            h = F.fht_plan_create(R, C, kind, split, 15, F.fht_schedule(**sched))
        except F.FhtError:
            continue  # no pass fits this budget: rejected, not mis-planned
        accepted += 1
        try:
            if kind == F.FHT_U8:
                img = rng.integers(0, 256, size=(R, C), dtype=np.uint8)
                ref = O.hough4(img, split)
            else:
                img = rng.integers(-8, 9, size=(R, C)).astype(np.float32)
                ref = O.hough4(img.astype(np.int64), split)
            for q in range(4):
                got = run_plan_tables(h, img, q)
                assert (got == ref[q]).all(), (R, C, split, kind, sched, q)
        finally:
            F.fht_plan_destroy(h)
    assert accepted >= 32
