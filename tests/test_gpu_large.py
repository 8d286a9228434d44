"""Full-element parity for the widest lane views.

Plans of 2049 lanes and more run three fused passes (up to 8192 lanes: the
last later passes take four tree levels where that saves a pass) or four
(16384 and 65536 lanes, up to the 65536 that fht_plan_create accepts); every
output element is compared, not a sample: with classic Brady-Yong at
4096 x 4096 (Sec. 3: both splits coincide with it at powers of two) and with
the C oracle's direct sums elsewhere.  uint8 bit-exact (int32), float32
within 1e-5 of each line's absolute sum.  Each integer case runs twice and
must repeat bit for bit.
"""
import numpy as np
import pytest
import torch

import paper_2411_07351_amd as F
import workloads as WL
from oracle import fht_oracle as O
from oracle import native

pytestmark = pytest.mark.gpu


def _run(img_np, kind, split, twice=False):
    plan = F.Plan(img_np.shape[0], img_np.shape[1], kind, split)
    img = torch.from_numpy(np.ascontiguousarray(img_np)).cuda()
    out = plan.new_out("cuda")
    plan.forward(img, out)
    torch.cuda.synchronize()
    got = [g.cpu().numpy() for g in plan.split_out(out)]
    if twice:
        out2 = torch.full_like(out, -7)
        plan.forward(img, out2)
        torch.cuda.synchronize()
        assert torch.equal(out, out2), "second run differs"
    return plan, got


def _close(got, ref, ab, tol=1e-5):
    err = np.abs(got.astype(np.float64) - ref)
    bad = err > tol * ab + 1e-30
    assert not bad.any(), f"{int(bad.sum())} elements over tolerance"


@pytest.mark.parametrize("split", ["S", "T"])
def test_4096_u8_every_output_equals_brady_yong(split):
    # S on an edge map, T on uniform 0..255 pixels (the widening pass at full
    # range: sums up to 255 * 4096)
    rng = WL.rng_for(5, salt=30)
    img = WL.edge_map(rng, 4096, 4096) if split == "S" else WL.uniform_u8(rng, 4096, 4096)
    plan, got = _run(img, "u8", split, twice=True)
    assert F.fht_plan_num_passes(plan.handle, 0) >= 3
    for q, (A, sigma) in enumerate(O.quadrant_views(img)):
        assert (got[q] == O.brady_yong(A, sigma)).all(), q


def test_4096_f32_every_output_within_tolerance_of_brady_yong():
    img = WL.normal_f32(WL.rng_for(5, salt=31), 4096, 4096)
    _, got = _run(img, "f32", "S")
    for q, (A, sigma) in enumerate(O.quadrant_views(img.astype(np.float64))):
        _close(got[q], O.brady_yong(A, sigma), O.brady_yong(np.abs(A), sigma))


@pytest.mark.parametrize("kind,shape,split", [
    ("u8", (3001, 64), "S"), ("u8", (64, 3001), "T"),
    ("f32", (3001, 64), "T"), ("f32", (64, 3001), "S"),
    ("u8", (2049, 2049), "T"),
])
def test_non_power_of_two_above_2048_lanes_every_output(kind, shape, split):
    R, C = shape
    rng = WL.rng_for(5, salt=32 + R % 7 + C % 5)
    sp = 0 if split == "S" else 1
    if kind == "u8":
        img = WL.uniform_u8(rng, R, C)
        _, got = _run(img, "u8", split, twice=True)
        ref = native.hough4_u8(img, sp)
        for q in range(4):
            assert (got[q] == ref[q]).all(), q
    else:
        img = WL.normal_f32(rng, R, C)
        _, got = _run(img, "f32", split)
        ref, ab = native.hough4_f64(img.astype(np.float64), sp)
        for q in range(4):
            _close(got[q], ref[q], ab[q])


@pytest.mark.parametrize("kind,shape,split", [
    ("u8", (1, 65536), "S"), ("u8", (65536, 1), "T"),
    ("u8", (8191, 37), "S"), ("u8", (37, 8191), "T"),
    ("f32", (8191, 37), "T"), ("u8", (16384, 3), "S"),
])
def test_sides_above_4096_every_output(kind, shape, split):
    R, C = shape
    rng = WL.rng_for(5, salt=40 + R % 11 + C % 13)
    sp = 0 if split == "S" else 1
    if kind == "u8":
        img = WL.uniform_u8(rng, R, C)
        plan, got = _run(img, "u8", split, twice=True)
        ref = native.hough4_u8(img, sp)
        for q in range(4):
            assert (got[q] == ref[q]).all(), q
    else:
        img = WL.normal_f32(rng, R, C)
        plan, got = _run(img, "f32", split)
        ref, ab = native.hough4_f64(img.astype(np.float64), sp)
        for q in range(4):
            _close(got[q], ref[q], ab[q])
    # 8191 lanes: 13 tree levels in 3 passes (5 + 4 + 4); 16384 and 65536
    # lanes: 4 passes
    assert max(F.fht_plan_num_passes(plan.handle, v) for v in (0, 1)) >= \
        (4 if max(R, C) >= 16384 else 3)
