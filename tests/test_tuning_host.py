"""Host logic of the autotuner (no GPU): size classes, the per-class cache
round trip, and batches whose plans carry different schedules."""
import json

import pytest

import paper_2411_07351_amd as F
from paper_2411_07351_amd import tuning as T


def test_size_class_is_the_tree_heights():
    assert T.size_class(1, 1) == "0x0"
    assert T.size_class(2, 3) == "1x2"
    assert T.size_class(1021, 1024) == "10x10"
    assert T.size_class(1025, 33) == "11x6"


def test_cache_round_trip_per_class(tmp_path, monkeypatch):
    monkeypatch.setenv("FHT_AUTOTUNE_CACHE", str(tmp_path / "c.json"))
    s = dict(T.DEFAULT, first_levels=6, max_levels=4)
    T._store({T.class_key("9x10", "u8", "S", "gfx950"): {"schedule": s, "timings_ms": []}})
    with open(tmp_path / "c.json") as fh:
        assert json.load(fh)["gfx950|u8|S|9x10"]["schedule"] == s
    monkeypatch.setattr(T, "_arch", lambda: "gfx950")
    assert T.lookup(300, 1000, "u8", "S") == s       # same class
    assert T.lookup(300, 1000, "u8", "T") is None    # other split
    assert T.lookup(600, 1000, "u8", "S") is None    # other class


def test_batch_of_plans_with_different_schedules():
    """Plans of other workgroup sizes get launches of their own; equal
    shapes of one schedule share launches."""
    a = F.Plan(300, 200, "u8", "S")
    b = F.Plan(300, 200, "u8", "S", schedule=dict(T.DEFAULT, threads=256, threads_first=256))
    one = F.fht_batch_prepare([a.handle, a.handle], [16, 32], [64, 128])
    two = F.fht_batch_prepare([a.handle, b.handle], [16, 32], [64, 128])
    try:
        assert F.fht_batch_num_launches(two) == 2 * F.fht_batch_num_launches(one)
    finally:
        F.fht_batch_destroy(one)
        F.fht_batch_destroy(two)
