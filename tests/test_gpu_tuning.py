"""The autotuner on the GPU: per-size-class schedules picked on a small
ragged batch, the tuned batch bit-exact against the oracle on every output,
and the cache re-read by a second call and by ``plans_for``."""
import numpy as np
import pytest

import workloads as WL
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

# a reduced search (the pass cuts and the workgroup size) keeps the test short
KNOBS = (("first_levels", (4, 5, 6)), ("max_levels", (2, 3, 4)), ("threads", (256, 512)))


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_07351_amd as F
    return F


def test_tuned_ragged_batch_is_exact_and_cached(F, tmp_path, monkeypatch):
    from paper_2411_07351_amd import tuning as T
    monkeypatch.setenv("FHT_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    rng = WL.rng_for(3, salt=41)
    shapes = WL.ragged_shapes(rng, 24, 20, 300)
    imgs_np = [WL.edge_map(rng, r, c) for r, c in shapes]
    imgs = [torch.from_numpy(i).cuda() for i in imgs_np]

    scheds = T.autotune(imgs, "S", knobs=KNOBS, reps=2)
    classes = {T.size_class(r, c) for r, c in shapes}
    assert set(scheds) == classes
    rep = T.last_report["classes"]
    assert all(rep[c]["source"] == "tuned" for c in classes)
    for c in classes:
        assert rep[c]["ms"] <= rep[c]["default_ms"] + 1e-9

    plans = T.plans_for(shapes, "u8", "S", scheds)
    outs = [p.new_out() for p in plans]
    batch = F.Batch(plans, imgs, outs)
    ws = batch.new_ws()
    batch.run(ws)
    torch.cuda.synchronize()
    for p, img, o in zip(plans, imgs_np, outs):
        ref = native.hough4_u8(img, 0)
        got = p.split_out(o)
        for q in range(4):
            assert (got[q].cpu().numpy() == ref[q]).all(), (img.shape, q)

    # a second call reads every class from the cache; plans_for does too
    again = T.autotune(imgs, "S", knobs=KNOBS, reps=2)
    assert again == scheds
    assert all(v["source"] == "cache" for v in T.last_report["classes"].values())
    for r, c in shapes:
        assert T.lookup(r, c, "u8", "S") == scheds[T.size_class(r, c)]
    plans2 = T.plans_for(shapes, "u8", "S")
    outs2 = [p.new_out() for p in plans2]
    F.Batch(plans2, imgs, outs2).run(ws)
    torch.cuda.synchronize()
    for a, b in zip(outs, outs2):
        assert torch.equal(a, b)


def test_plain_schedule_pick_is_exact(F):
    # both per-image schedules run every image of a small same-shape set; the
    # pick is one of them, and the two-pass schedule really has two passes
    from paper_2411_07351_amd import tuning as T
    rng = WL.rng_for(3, salt=42)
    imgs_np = WL.edge_maps(rng, 4, 300, 517)
    imgs = [torch.from_numpy(i).cuda() for i in imgs_np]
    name, times = T.tune_plain(imgs, "S", reps=2)
    assert name in T.PLAIN_SCHEDULES and set(times) == set(T.PLAIN_SCHEDULES)
    assert times[name] == min(times.values())
    two = F.Plan(300, 517, "u8", "S", schedule=T.PLAIN_SCHEDULES["two-pass"])
    assert [F.fht_plan_num_passes(two.handle, v) for v in (0, 1)] == [2, 2]
    out = two.new_out()
    two.forward(imgs[1], out)
    torch.cuda.synchronize()
    ref = native.hough4_u8(imgs_np[1], 0)
    for q, g in enumerate(two.split_out(out)):
        assert (g.cpu().numpy() == ref[q]).all(), q


@pytest.mark.parametrize("split", [0, 1])
def test_small_image_in_one_launch(F, split):
    # 61 x 47 (the smallest workload): the two-pass schedule's 6-level first
    # pass covers both order trees, so one launch does the whole transform
    from paper_2411_07351_amd import tuning as T
    img_np = WL.uniform_u8(WL.rng_for(1), 61, 47)
    plan = F.Plan(61, 47, "u8", split, schedule=T.PLAIN_SCHEDULES["two-pass"])
    assert F.fht_plan_num_launches(plan.handle) == 1
    out = plan.new_out()
    for _ in range(2):  # twice on one workspace: must repeat bit for bit
        plan.forward(torch.from_numpy(img_np).cuda(), out)
        torch.cuda.synchronize()
        ref = native.hough4_u8(img_np, split)
        for q, g in enumerate(plan.split_out(out)):
            assert (g.cpu().numpy() == ref[q]).all(), q
