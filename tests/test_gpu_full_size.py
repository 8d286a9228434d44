"""Parity at the benchmark's full sizes, in the launch configurations bench.py
times: every image of the 64 x 1021x1021 batch (graph replays, and per-image
launches under both per-image schedules), every image of the 512-image ragged
batch, and requests of the serving stream up to 4096 per side, checked on
sampled outputs that the C oracle computes one by one (bit-exact for uint8,
1e-5 of the line's absolute sum for float32)."""
import numpy as np
import pytest
import torch

import paper_2411_07351_amd as F
import workloads as WL
from oracle import native

pytestmark = pytest.mark.gpu


def _samples(plan, rng, k):
    qs = np.array(plan.quadrants, dtype=np.int32)
    q = rng.choice(qs, size=k).astype(np.int32)
    t = np.empty(k, dtype=np.int32)
    s = np.empty(k, dtype=np.int32)
    for i in range(k):
        W, H = plan.shapes[int(q[i])]
        t[i] = rng.integers(0, W)
        s[i] = rng.integers(0, H)
    # always include the extreme slopes and shifts
    for j, qq in enumerate(qs):
        W, H = plan.shapes[int(qq)]
        q = np.append(q, [qq, qq, qq]).astype(np.int32)
        t = np.append(t, [0, W - 1, W // 2]).astype(np.int32)
        s = np.append(s, [0, H - 1, (H * 7) // 11]).astype(np.int32)
    flat = np.array([plan.offsets[int(qq)] + int(tt) * plan.shapes[int(qq)][1] + int(ss)
                     for qq, tt, ss in zip(q, t, s)], dtype=np.int64)
    return q, t, s, flat


def _check_u8(plan, out, img_np, split, rng, k):
    q, t, s, flat = _samples(plan, rng, k)
    got = out[torch.from_numpy(flat).to(out.device)].cpu().numpy()
    ref = native.sample_u8(img_np, split, q, t, s)
    assert (got == ref).all(), np.nonzero(got != ref)[0][:5]


def _check_f32(plan, out, img_np, split, rng, k):
    q, t, s, flat = _samples(plan, rng, k)
    got = out[torch.from_numpy(flat).to(out.device)].double().cpu().numpy()
    ref, ab = native.sample_f64(img_np.astype(np.float64), split, q, t, s)
    assert (np.abs(got - ref) <= 1e-5 * ab + 1e-30).all()


def test_bench_batch_64x1021_graph_every_image():
    n, R, C = 64, 1021, 1021
    imgs_np = WL.edge_maps(WL.rng_for(2), n, R, C)
    imgs = torch.from_numpy(imgs_np).cuda()
    plan = F.Plan(R, C, "u8", "S")
    outs = torch.full((n, plan.out_elems), -1, dtype=torch.int32, device="cuda")
    batch = F.Batch([plan] * n, [imgs[i] for i in range(n)], [outs[i] for i in range(n)])
    ws = batch.new_ws()
    graph = batch.capture(ws)
    graph.replay()
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    for i in range(n):
        _check_u8(plan, outs[i], imgs_np[i], 0, rng, 300)
    # one image in full, against the plain per-image launches
    solo = plan.new_out("cuda")
    plan.forward(imgs[5], solo)
    torch.cuda.synchronize()
    assert torch.equal(solo, outs[5])


def test_bench_plain_schedules_64x1021_every_image():
    # the per-image launches bench.py times, under both of its schedules
    from paper_2411_07351_amd import tuning as T
    n, R, C = 64, 1021, 1021
    imgs_np = WL.edge_maps(WL.rng_for(2), n, R, C)
    imgs = torch.from_numpy(imgs_np).cuda()
    got = {}
    for name, sched in T.PLAIN_SCHEDULES.items():
        plan = F.Plan(R, C, "u8", "S", schedule=sched)
        outs = torch.full((n, plan.out_elems), -1, dtype=torch.int32, device="cuda")
        ws = plan.new_ws("cuda")
        sh = torch.cuda.current_stream().cuda_stream
        for i in range(n):
            for l in range(F.fht_plan_num_launches(plan.handle)):
                F.fht_forward_launch(plan.handle, l, imgs[i].data_ptr(), outs[i].data_ptr(),
                                     ws.data_ptr(), sh)
        torch.cuda.synchronize()
        got[name] = (plan, outs)
    rng = np.random.default_rng(19)
    plan, outs = got["two-pass"]
    assert [F.fht_plan_num_passes(plan.handle, v) for v in (0, 1)] == [2, 2]
    for i in range(n):
        _check_u8(plan, outs[i], imgs_np[i], 0, rng, 200)
    assert torch.equal(outs, got["default"][1])


def test_bench_ragged_512_graph_every_image():
    rng = WL.rng_for(3)
    shapes = WL.ragged_shapes(rng, 512, 32, 2048)
    imgs_np = [WL.edge_map(rng, r, c) for r, c in shapes]
    imgs = [torch.from_numpy(i).cuda() for i in imgs_np]
    cache = {}
    plans = []
    for r, c in shapes:
        if (r, c) not in cache:
            cache[(r, c)] = F.Plan(r, c, "u8", "S")
        plans.append(cache[(r, c)])
    outs = [p.new_out("cuda") for p in plans]
    for o in outs:
        o.fill_(-1)
    batch = F.Batch(plans, imgs, outs)
    ws = batch.new_ws()
    graph = batch.capture(ws)
    graph.replay()
    torch.cuda.synchronize()
    srng = np.random.default_rng(18)
    for p, o, img in zip(plans, outs, imgs_np):
        _check_u8(p, o, img, 0, srng, 40)
    # every output of every image: equal to plain per-image launches, and
    # every slope row of every quadrant sums to the image sum (each line
    # family partitions the pixels, Sec. 3)
    for p, o, img in zip(plans, outs, imgs):
        solo = p.new_out("cuda")
        p.forward(img, solo)
        assert torch.equal(solo, o), (img.shape,)
        total = int(img.sum())
        for g in p.split_out(o):
            assert (g.sum(dim=1, dtype=torch.int64) == total).all(), (img.shape,)
    torch.cuda.synchronize()
    # the smallest images in full
    order = sorted(range(512), key=lambda i: shapes[i][0] * shapes[i][1])[:20]
    for i in order:
        ref = native.hough4_u8(imgs_np[i], 0)
        for q, g in enumerate(plans[i].split_out(outs[i])):
            assert (g.cpu().numpy() == ref[q]).all(), (shapes[i], q)


@pytest.mark.parametrize("kind,shape", [("u8", (4096, 4096)), ("f32", (4096, 1333)),
                                        ("u8", (64, 4096)), ("f32", (3001, 64))])
def test_serving_sizes(kind, shape):
    R, C = shape
    rng = WL.rng_for(5, salt=20)
    img = WL.edge_map(rng, R, C) if kind == "u8" else WL.normal_f32(rng, R, C)
    plan = F.Plan(R, C, kind, "S")
    out = plan.new_out("cuda")
    plan.forward(torch.from_numpy(img).cuda(), out)
    torch.cuda.synchronize()
    srng = np.random.default_rng(19)
    if kind == "u8":
        _check_u8(plan, out, img, 0, srng, 400)
    else:
        _check_f32(plan, out, img, 0, srng, 400)
