"""Peak finding on the GPU: equal to a plain NumPy statement of the same
definition on small outputs (bit-exact for integer outputs), valid at full
size, and recovering the planted segments of a 1021 x 1021 edge map."""
import numpy as np
import pytest
import torch

import paper_2411_07351_amd as F
import workloads as WL
from peak_ref import local_maxima_topk, matches, segment_lines

pytestmark = pytest.mark.gpu


def _outs(plan, flat):
    return {q: (flat[plan.offsets[q]:plan.offsets[q] + W * H].reshape(W, H), plan.offsets[q])
            for q, (W, H) in plan.shapes.items()}


def _as_list(recs):
    return [(float(r["value"]), int(r["quadrant"]), int(r["t"]), int(r["s"])) for r in recs]


@pytest.mark.parametrize("case", [("u8", 61, 47, 0, 20, 0.0), ("u8", 61, 47, 1, 40, 6000.0),
                                  ("u8", 64, 33, 3, 25, 0.0), ("f32", 90, 120, 2, 30, -1e9),
                                  ("u8", 5, 3, 4, 10, 0.0)])
def test_peaks_equal_reference(case):
    kind, R, C, radius, k, floor = case
    rng = WL.rng_for(1, salt=radius + 3)
    img = WL.uniform_u8(rng, R, C) if kind == "u8" else WL.normal_f32(rng, R, C)
    plan = F.Plan(R, C, kind, "S")
    out = plan.new_out("cuda")
    plan.forward(torch.from_numpy(img).cuda(), out)
    recs, cands = plan.peaks(out, k=k, radius=radius, min_value=floor)
    ref, ref_cands = local_maxima_topk(_outs(plan, out.cpu().numpy()), k, radius, floor)
    assert cands == ref_cands
    assert _as_list(recs) == ref


@pytest.mark.parametrize("case", [
    # radius 0: every output above the floor is a candidate.  65536 of them:
    # more than the selection sorts at once, so the k-th largest value is
    # found by a radix select first (ties at it included in the sort)
    ("u8", 128, 128, 0, 4096, 0.0),
    # all outputs equal: the tie at the k-th value spans every candidate,
    # which the selection then takes in rounds
    ("zero", 61, 47, 0, 100, 0.0),
    # a few thousand candidates, k at its limit
    ("u8", 100, 90, 1, 4096, 0.0),
])
def test_peaks_many_candidates(case):
    kind, R, C, radius, k, floor = case
    rng = WL.rng_for(1, salt=40 + R)
    img = np.zeros((R, C), dtype=np.uint8) if kind == "zero" else WL.uniform_u8(rng, R, C)
    plan = F.Plan(R, C, "u8", "S")
    out = plan.new_out("cuda")
    plan.forward(torch.from_numpy(img).cuda(), out)
    recs, cands = plan.peaks(out, k=k, radius=radius, min_value=floor, capacity=1 << 17)
    ref, ref_cands = local_maxima_topk(_outs(plan, out.cpu().numpy()), k, radius, floor)
    assert cands == ref_cands
    assert _as_list(recs) == ref


def test_peaks_f64_order_by_exact_value():
    # float64 outputs that round to the same float32 must still be ordered by
    # their own values: integer pixels plus a perturbation far below float32
    # resolution at these magnitudes
    rng = WL.rng_for(1, salt=30)
    R, C = 40, 36
    img = np.round(rng.standard_normal((R, C)) * 3.0) + 1e-9 * rng.standard_normal((R, C))
    plan = F.Plan(R, C, "f64", "S")
    out = plan.new_out("cuda")
    plan.forward(torch.from_numpy(img).cuda(), out)
    recs, cands = plan.peaks(out, k=60, radius=1, min_value=-1e30)
    flat = out.cpu().numpy()
    ref, ref_cands = local_maxima_topk(_outs(plan, flat), 60, 1, -1e30)
    assert cands == ref_cands
    assert _as_list(recs) == ref
    # and some neighbours in that order are equal as float32 but not as float64
    vals = [flat[plan.offsets[q] + t * plan.shapes[q][1] + s] for _, q, t, s in ref]
    assert any(a != b and np.float32(a) == np.float32(b) for a, b in zip(vals, vals[1:]))


def test_peaks_recover_planted_segments():
    R = C = 1021
    img, ends = WL.edge_map_segments(WL.rng_for(2), R, C)
    plan = F.Plan(R, C, "u8", "S")
    out = plan.new_out("cuda")
    plan.forward(torch.from_numpy(img).cuda(), out)
    recs, cands = plan.peaks(out, k=80, radius=8, min_value=120)
    peaks = _as_list(recs)
    flat = out.cpu().numpy()
    outs = _outs(plan, flat)
    # every peak is a strict local maximum above the floor, strongest first
    for v, q, t, s in peaks:
        J = outs[q][0]
        W, H = J.shape
        win = J[max(0, t - 8):t + 9][:, (np.arange(s - 8, s + 9)) % H]
        assert v == J[t, s] >= 120 and (win <= J[t, s]).all()
    assert [p[0] for p in peaks] == sorted((p[0] for p in peaks), reverse=True)
    long_segs = [e for e in ends if max(abs(e[2] - e[0]), abs(e[3] - e[1])) >= 250]
    assert len(long_segs) >= 5
    for r0, c0, r1, c1 in long_segs:
        lines = segment_lines(int(r0), int(c0), int(r1), int(c1), R, C)
        assert any(matches(p, ln) for p in peaks for ln in lines), (r0, c0, r1, c1)


def test_peaks_reject_bad_arguments():
    plan = F.Plan(9, 9, "u8", "S")
    out = plan.new_out("cuda")
    with pytest.raises(F.FhtError):
        plan.peaks(out, k=0)
    with pytest.raises(F.FhtError):
        plan.peaks(out, k=8, capacity=4)
    with pytest.raises(F.FhtError):
        plan.peaks(out, k=8, radius=65)
