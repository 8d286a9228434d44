"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Integer images must match bit for bit (int32 outputs, int64 oracle).  Float
images must satisfy |gpu - oracle_fp64| <= 1e-5 * (sum of |A| along the same
line), the per-line bound the float path is held to.
"""
import numpy as np
import pytest

import workloads as WL
from oracle import fht_oracle as O
from oracle import native

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2411_07351_amd as F
    return F


def _gpu_hough(F, img_np, split, schedule=None, quadrants=(0, 1, 2, 3)):
    """Outputs of the plan's forward; integer images run twice, on one
    workspace, and must repeat bit for bit (a race would show as a change)."""
    img = torch.from_numpy(np.ascontiguousarray(img_np)).cuda()
    plan = F.Plan(img.shape[0], img.shape[1], img.dtype, split, quadrants, schedule)
    ws = plan.new_ws() if plan.ws_bytes else None
    out = plan.new_out()
    plan.forward(img, out, ws)
    if img.dtype == torch.uint8:
        again = torch.full_like(out, -7)
        plan.forward(img, again, ws)
        torch.cuda.synchronize()
        assert torch.equal(out, again), "a second run differs"
    torch.cuda.synchronize()
    return [o.cpu().numpy() for o in plan.split_out(out)]


def _assert_float_close(got, ref, absref, tol=1e-5):
    err = np.abs(got.astype(np.float64) - ref)
    bound = tol * absref + 1e-30
    bad = err > bound
    assert not bad.any(), f"{bad.sum()} elements over tolerance, worst {np.max(err / bound):.3g}"


@pytest.mark.parametrize("split", [0, 1])
def test_config1_61x47_u8_bit_exact(F, split):
    img = WL.uniform_u8(WL.rng_for(1), 61, 47)
    got = _gpu_hough(F, img, split)
    ref = O.hough4(img, split)
    for q in range(4):
        assert got[q].dtype == np.int32
        assert (got[q] == ref[q]).all(), q


@pytest.mark.parametrize("split", [0, 1])
def test_shape_sweep_u8(F, split):
    rng = WL.rng_for(0, salt=7)
    shapes = [(1, 1), (1, 2), (2, 1), (1, 300), (300, 1), (2, 3), (3, 2), (5, 3), (13, 11),
              (31, 33), (32, 32), (33, 31), (64, 65), (100, 37), (129, 257), (257, 129),
              (200, 700)]
    for R, C in shapes:
        img = WL.uniform_u8(rng, R, C)
        got = _gpu_hough(F, img, split)
        ref = native.hough4_u8(img, split)
        for q in range(4):
            assert (got[q] == ref[q]).all(), (R, C, q)


@pytest.mark.parametrize("sched", [
    dict(s_tile=64, s_tile_first=64, first_levels=2, max_levels=2, lds_budget=8192, t_tile=0),
    dict(s_tile=128, s_tile_first=128, first_levels=3, max_levels=3, lds_budget=16384, t_tile=4),
    dict(s_tile=192, s_tile_first=256, first_levels=4, max_levels=5, lds_budget=65536, t_tile=16),
    dict(s_tile=64, s_tile_first=192, first_levels=1, max_levels=1, lds_budget=65536, t_tile=0),
    dict(s_tile=256, s_tile_first=64, first_levels=6, max_levels=7, lds_budget=65536, t_tile=8),
])
def test_schedules_u8(F, sched):
    rng = WL.rng_for(0, salt=8)
    for split in (0, 1):
        for R, C in ((77, 45), (130, 17), (9, 300)):
            img = WL.uniform_u8(rng, R, C)
            got = _gpu_hough(F, img, split, sched)
            ref = native.hough4_u8(img, split)
            for q in range(4):
                assert (got[q] == ref[q]).all(), (R, C, q, sched)


def test_quadrant_subsets(F):
    img = WL.uniform_u8(WL.rng_for(0, salt=9), 40, 23)
    ref = native.hough4_u8(img, 1)
    for qs in ((0,), (3,), (1, 2), (0, 2, 3)):
        got = _gpu_hough(F, img, 1, quadrants=qs)
        for g, q in zip(got, qs):
            assert (g == ref[q]).all(), qs


@pytest.mark.parametrize("split", [0, 1])
def test_1024_equals_brady_yong(F, split):
    # Sec. 3: at n = 2^q both variants coincide with Brady-Yong.
    img = WL.edge_map(WL.rng_for(2, salt=1), 1024, 1024)
    got = _gpu_hough(F, img, split)
    for q, (A, sigma) in enumerate(O.quadrant_views(img)):
        assert (got[q] == O.brady_yong(A, sigma)).all(), q


@pytest.mark.parametrize("split", [0, 1])
def test_config2_1021_full_vs_oracle(F, split):
    # Two full 1021 x 1021 edge maps against the C oracle (about 4.3e9 adds each).
    rng = WL.rng_for(2)
    for _ in range(2 if split == 0 else 1):
        img = WL.edge_map(rng, 1021, 1021)
        got = _gpu_hough(F, img, split)
        ref = native.hough4_u8(img, split)
        for q in range(4):
            assert (got[q] == ref[q]).all(), q


def test_config4_f32_within_tolerance(F):
    rng = WL.rng_for(4)
    for split in (0, 1):
        img = WL.normal_f32(rng, 384, 257)
        got = _gpu_hough(F, img, split)
        ref, absref = native.hough4_f64(img.astype(np.float64), split)
        for q in range(4):
            assert got[q].dtype == np.float32
            _assert_float_close(got[q], ref[q], absref[q])


def test_f64_small(F):
    rng = WL.rng_for(4, salt=2)
    img = rng.standard_normal((13, 11))
    for split in (0, 1):
        got = _gpu_hough(F, img, split)
        ref, absref = native.hough4_f64(img, split)
        for q in range(4):
            _assert_float_close(got[q], ref[q], absref[q], tol=1e-12)


def test_deterministic_and_invariants(F):
    img = WL.edge_map(WL.rng_for(2, salt=3), 517, 300)
    a = _gpu_hough(F, img, 0)
    b = _gpu_hough(F, img, 0)
    total = int(img.sum())
    for q in range(4):
        assert (a[q] == b[q]).all()
        assert (a[q].sum(axis=1) == total).all()


def test_batch_matches_plain(F):
    rng = WL.rng_for(3, salt=1)
    imgs_np = WL.ragged_edge_maps(rng, 12, 1, 300)
    imgs_np[0] = WL.uniform_u8(rng, 1, 1)
    imgs_np[1] = WL.uniform_u8(rng, 61, 47)
    for split in (0, 1):
        imgs = [torch.from_numpy(i).cuda() for i in imgs_np]
        plans = [F.Plan(i.shape[0], i.shape[1], "u8", split) for i in imgs]
        outs = [p.new_out() for p in plans]
        batch = F.Batch(plans, imgs, outs)
        ws = batch.new_ws()
        batch.run(ws)
        torch.cuda.synchronize()
        for img_np, p, out in zip(imgs_np, plans, outs):
            ref = native.hough4_u8(img_np, split)
            for q, g in enumerate(p.split_out(out)):
                assert (g.cpu().numpy() == ref[q]).all(), (img_np.shape, q)


@pytest.mark.parametrize("sched", [None,
                                   dict(first_levels=5, max_levels=4, t_tile=16),
                                   dict(first_levels=4, max_levels=5, t_tile=8),
                                   dict(first_levels=5, max_levels=3, t_tile=32, threads=256)])
def test_u16_intermediates_at_full_range(F, sched):
    # uint8 images keep 16-bit sums while nodes are at most 257 lanes wide;
    # 255 * 257 = 65535 is the largest such sum.  Saturated images hit it.
    for R, C in ((514, 33), (33, 514), (257, 70), (1021, 64)):
        img = np.full((R, C), 255, dtype=np.uint8)
        got = _gpu_hough(F, img, 0, sched)
        for q, (W, H) in enumerate(((R, C), (R, C), (C, R), (C, R))):
            assert (got[q] == 255 * W).all(), (R, C, q)
        rng = WL.rng_for(0, salt=10)
        img = rng.integers(200, 256, size=(R, C), dtype=np.uint8)
        got = _gpu_hough(F, img, 1, sched)
        ref = native.hough4_u8(img, 1)
        for q in range(4):
            assert (got[q] == ref[q]).all(), (R, C, q)


def test_graph_replays_match_eager(F):
    # A captured batch must give the eager result on every replay, with eager
    # work and synchronisations between replays.
    rng = WL.rng_for(3, salt=2)
    imgs_np = WL.ragged_edge_maps(rng, 10, 8, 300)
    imgs = [torch.from_numpy(i).cuda() for i in imgs_np]
    plans = [F.Plan(i.shape[0], i.shape[1], "u8", "S") for i in imgs]
    outs = [p.new_out() for p in plans]
    batch = F.Batch(plans, imgs, outs)
    ws = batch.new_ws()
    batch.run(ws)
    torch.cuda.synchronize()
    eager = [o.clone() for o in outs]
    graph = batch.capture(ws)
    for rep in range(4):
        for o in outs:
            o.fill_(-1)
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # unrelated eager work
        graph.replay()
        torch.cuda.synchronize()
        del junk
        for o, e in zip(outs, eager):
            assert torch.equal(o, e), rep
    ref = native.hough4_u8(imgs_np[3], 0)
    for q, g in enumerate(plans[3].split_out(outs[3])):
        assert (g.cpu().numpy() == ref[q]).all()


@pytest.mark.parametrize("kind,shape,n", [("u8", (61, 47), 5), ("u8", (300, 200), 3),
                                          ("f32", (129, 70), 4), ("u8", (1, 9), 2)])
def test_forward_many_equals_single_images(F, kind, shape, n):
    R, C = shape
    rng = WL.rng_for(2, salt=40 + n)
    if kind == "u8":
        imgs = torch.from_numpy(np.stack([WL.uniform_u8(rng, R, C) for _ in range(n)])).cuda()
    else:
        imgs = torch.from_numpy(np.stack([WL.normal_f32(rng, R, C) for _ in range(n)])).cuda()
    plan = F.Plan(R, C, kind, "S")
    outs = plan.forward_many(imgs)
    torch.cuda.synchronize()
    for b in range(n):
        solo = plan.new_out("cuda")
        plan.forward(imgs[b], solo)
        torch.cuda.synchronize()
        assert torch.equal(outs[b], solo), b


def test_forward_many_config4_f32_vs_oracle(F):
    # the batch the differentiable leg times: 32 float32 384 x 257 images in
    # one launch per pass, every image against the oracle
    n, R, C = 32, 384, 257
    rng = WL.rng_for(4)
    imgs_np = np.stack([WL.normal_f32(rng, R, C) for _ in range(n)])
    plan = F.Plan(R, C, "f32", "S")
    outs = plan.forward_many(torch.from_numpy(imgs_np).cuda())
    torch.cuda.synchronize()
    outs = outs.cpu().numpy()
    for b in range(n):
        ref, ab = native.hough4_f64(imgs_np[b].astype(np.float64), 0)
        for q, (W, H) in plan.shapes.items():
            off = plan.offsets[q]
            _assert_float_close(outs[b, off:off + W * H].reshape(W, H), ref[q], ab[q])


def test_forward_on_a_side_stream_vs_oracle(F):
    # Kernels enqueued on a caller's stream while the current stream allocates
    # and frees memory: the call's own workspace and output must not be
    # handed to that other work (they are allocated on the side stream).
    rng = WL.rng_for(2, salt=50)
    imgs_np = [WL.uniform_u8(rng, 700, 513), WL.normal_f32(rng, 300, 611)]
    side = torch.cuda.Stream()
    results = []
    for img_np in imgs_np:
        plan = F.Plan(img_np.shape[0], img_np.shape[1], "u8" if img_np.dtype == np.uint8 else "f32",
                      "S")
        img = torch.from_numpy(img_np).cuda()
        side.wait_stream(torch.cuda.current_stream())
        quads = plan.forward(img, stream=side)
        for _ in range(20):  # allocation-heavy work on the current stream
            junk = torch.full((1 << 22,), 3, dtype=torch.int32, device="cuda")
            junk.add_(1)
            del junk
        torch.cuda.current_stream().wait_stream(side)
        results.append([g.cpu().numpy() for g in quads])
    ref = native.hough4_u8(imgs_np[0], 0)
    for q in range(4):
        assert (results[0][q] == ref[q]).all(), q
    ref, ab = native.hough4_f64(imgs_np[1].astype(np.float64), 0)
    for q in range(4):
        _assert_float_close(results[1][q], ref[q], ab[q])


@pytest.mark.parametrize("kind", ["u8", "f32", "f64"])
def test_random_shapes_every_path(F, kind):
    # Seeded shapes, log-uniform per side up to 1100 lanes, plus shapes whose
    # widening pass fuses two levels (513..1024 lanes), and quadrant subsets
    # (views without a quadrant pair): every pass kind of the planner (loads,
    # load-merges, merge steps, stores that add) against the C oracle.
    rng = WL.rng_for(6, salt={"u8": 1, "f32": 2, "f64": 3}[kind])
    sides = np.exp(rng.uniform(0.0, np.log(1100.0), size=(6, 2))).astype(int)
    shapes = [tuple(int(v) for v in rc) for rc in sides] + [(700, 90), (90, 700), (1021, 3)]
    subsets = [(0, 1, 2, 3), (0,), (3,), (1, 2)]
    for i, (R, C) in enumerate(shapes):
        split = i % 2
        qs = subsets[i % len(subsets)]
        if kind == "u8":
            img = WL.uniform_u8(rng, R, C)
            got = _gpu_hough(F, img, split, quadrants=qs)
            ref = native.hough4_u8(img, split)
            for g, q in zip(got, qs):
                assert g.dtype == np.int32 and (g == ref[q]).all(), (R, C, split, q)
        else:
            img = WL.normal_f32(rng, R, C)
            if kind == "f64":
                img = img.astype(np.float64)
            got = _gpu_hough(F, img, split, quadrants=qs)
            ref, ab = native.hough4_f64(img.astype(np.float64), split)
            tol = 1e-5 if kind == "f32" else 1e-12
            for g, q in zip(got, qs):
                _assert_float_close(g, ref[q], ab[q], tol)


def test_planner_pool_plans_on_the_device(F):
    """Plans from the native planner pool, their programs copied by its
    uploader in batched copies (fht_plan_upload_programs_many), run a ragged
    batch bit-exactly (a schedule of their own, so no earlier test has put
    these lane views on the device)."""
    import time
    rng = WL.rng_for(3, salt=9)
    imgs_np = WL.ragged_edge_maps(rng, 10, 2, 400)
    sched = F.fht_schedule(s_tile=128, s_tile_first=64, first_levels=4, max_levels=3,
                           lds_budget=64 * 1024, t_tile=8, threads=512, threads_first=512)
    pool = F.fht_planner_create(4, torch.cuda.current_device())
    try:
        tickets = [F.fht_planner_submit(pool, i.shape[0], i.shape[1], F.FHT_U8, 0, 15, sched)
                   for i in imgs_np]
        plans = []
        for t in tickets:
            t0 = time.monotonic()
            while True:
                state, h, st = F.fht_planner_poll(pool, t)
                if state:
                    break
                assert time.monotonic() - t0 < 60
                time.sleep(1e-3)
            assert state == 1 and st == 0
            plans.append(h)
    finally:
        F.fht_planner_destroy(pool)
    wrapped = [F.Plan.adopt(h, i.shape[0], i.shape[1], "u8", "S") for h, i in zip(plans, imgs_np)]
    F.fht_plan_upload_programs_many([p.handle for p in wrapped])  # all there: nothing to copy
    imgs = [torch.from_numpy(i).cuda() for i in imgs_np]
    outs = [p.new_out() for p in wrapped]
    batch = F.Batch(wrapped, imgs, outs, defer_upload=True)
    tables = torch.empty(batch.tables_bytes, dtype=torch.uint8, device="cuda")
    batch.upload(tables)
    batch.run(batch.new_ws())
    torch.cuda.synchronize()
    for img_np, p, out in zip(imgs_np, wrapped, outs):
        ref = native.hough4_u8(img_np, 0)
        for q, g in enumerate(p.split_out(out)):
            assert (g.cpu().numpy() == ref[q]).all(), (img_np.shape, q)


def test_batch_over_pointers_with_image_copies(F):
    """Batch.from_pointers over one image and one output buffer, images
    copied by fht_batch_copy_images from pinned host memory, from device
    memory and in place (NULL), bit-exact against the oracle."""
    rng = WL.rng_for(3, salt=11)
    imgs_np = WL.ragged_edge_maps(rng, 6, 3, 300)
    plans = [F.Plan(i.shape[0], i.shape[1], "u8", "S") for i in imgs_np]
    align = lambda n: (n + 255) // 256 * 256
    img_off, out_off, ib, ob = [], [], 0, 0
    for i, p in zip(imgs_np, plans):
        img_off.append(ib)
        ib += align(i.size)
        out_off.append(ob)
        ob += align(p.out_elems * 4)
    ibuf = torch.zeros(ib, dtype=torch.uint8, device="cuda")
    obuf = torch.empty(ob, dtype=torch.uint8, device="cuda")
    srcs, held = [], []
    for k, (i, o) in enumerate(zip(imgs_np, img_off)):
        t = torch.from_numpy(i)
        if k % 3 == 0:  # pinned host memory
            t = t.pin_memory()
        elif k % 3 == 1:  # device memory elsewhere
            t = t.cuda()
        else:  # already in place
            ibuf[o:o + i.size].copy_(t.reshape(-1))
            t = None
        held.append(t)
        srcs.append(None if t is None else t.data_ptr())
    batch = F.Batch.from_pointers(plans, [ibuf.data_ptr() + o for o in img_off],
                                  [obuf.data_ptr() + o for o in out_off])
    stream = torch.cuda.current_stream()
    batch.copy_images(srcs, stream)
    tables = torch.empty(batch.tables_bytes, dtype=torch.uint8, device="cuda")
    batch.upload(tables, stream)
    batch.run(batch.new_ws(), stream)
    torch.cuda.synchronize()
    for i, p, o in zip(imgs_np, plans, out_off):
        out = obuf[o:o + p.out_elems * 4].view(torch.int32)
        ref = native.hough4_u8(i, 0)
        for q, g in enumerate(p.split_out(out)):
            assert (g.cpu().numpy() == ref[q]).all(), (i.shape, q)
