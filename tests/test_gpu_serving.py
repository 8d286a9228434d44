"""The serving loop on the GPU: results in the mix equal results alone.

Requests of mixed sizes and dtypes arrive as a Poisson stream fast enough
that batches overlap on two streams.  Every request's four Hough images must
equal the C oracle's (uint8 bit-exact, float32 within 1e-5 of each line's
absolute sum), and equal those of the same image transformed alone
(``Plan.forward``) bit for bit, for uint8 and float32 alike, since both paths
run the same programs.
"""
import numpy as np
import pytest
import torch

import paper_2411_07351_amd as F
from paper_2411_07351_amd import serving as S
import workloads as WL
from oracle import native

pytestmark = pytest.mark.gpu


def _requests(n, seed, qps, lo=64, hi=700):
    rng = WL.rng_for(5, salt=seed)
    items = WL.serving_requests(rng, n, lo, hi)
    arr = WL.poisson_arrivals(rng, n, qps)
    return [S.Request(i, torch.from_numpy(img).pin_memory(), float(t))
            for i, ((kind, img), t) in enumerate(zip(items, arr))]


def _check_oracle(r):
    """The served result of request r against the C oracle (Sec. 3 sums)."""
    img = r.image.numpy()
    got = [g.cpu().numpy() for g in r.result()]
    what = f"request {r.rid} ({r.rows}x{r.cols} {r.kind})"
    if r.kind == "u8":
        ref = native.hough4_u8(img, 0)
        for q in range(4):
            assert got[q].dtype == np.int32 and (got[q] == ref[q]).all(), f"{what} quadrant {q}"
    else:
        ref, ab = native.hough4_f64(img.astype(np.float64), 0)
        for q in range(4):
            err = np.abs(got[q].astype(np.float64) - ref[q])
            assert (err <= 1e-5 * ab[q] + 1e-30).all(), f"{what} quadrant {q}"


def _check_solo(reqs):
    for r in reqs:
        assert r.status == "done", (r.rid, r.status, r.error)
        _check_oracle(r)
        img = r.image.cuda()
        solo = F.Plan(r.rows, r.cols, r.kind, "S").forward(img)
        torch.cuda.synchronize()
        for q, (a, b) in enumerate(zip(r.result(), solo)):
            assert torch.equal(a, b), f"request {r.rid} ({r.rows}x{r.cols} {r.kind}) quadrant {q}"


def _serve(reqs, warm_plans=False, **kw):
    torch.cuda.synchronize()
    srv = S.Server(S.GpuExecutor(streams=kw.pop("streams", 2)), kw.pop("budget", 4 << 30),
                   plan_threads=4, **kw)
    try:
        if warm_plans:  # every plan ready at once: simultaneous arrivals form one batch
            for r in reqs:
                srv.plans.get(r.rows, r.cols, r.kind, r.split).result()
        srv.run(reqs)
    finally:
        srv.close()
    torch.cuda.synchronize()
    return srv


def test_results_in_the_mix_equal_results_alone():
    reqs = _requests(24, seed=10, qps=20000.0)
    srv = _serve(reqs, max_batch_images=6, depth=2)
    assert max(srv.batch_sizes) > 1
    assert {r.kind for r in reqs} == {"u8", "f32"}
    _check_solo(reqs)


def test_small_budget_serialises_and_stays_exact():
    reqs = _requests(8, seed=11, qps=float("inf"), hi=300)
    need = max(S.footprint(F.Plan(r.rows, r.cols, r.kind, "S"), r.kind) for r in reqs)
    srv = _serve(reqs, budget=need)
    assert srv.peak_in_use <= need
    _check_solo(reqs)


def test_injected_enqueue_failure_fails_one_request_only():
    reqs = _requests(8, seed=12, qps=5000.0, hi=300)
    F.fht_debug_fail_next(-4, 1)
    try:
        srv = _serve(reqs, max_batch_images=1)
    finally:
        F.fht_debug_fail_next(0, 0)
    failed = [r for r in reqs if r.status == "failed"]
    assert len(failed) == 1
    _check_solo([r for r in reqs if r.status != "failed"])


def test_injected_failure_of_a_batch_is_retried():
    # the uint8 requests arrive at once with their plans ready, so
    # the first enqueue (the one that fails) is a batch of several requests;
    # its requests are retried one by one and all succeed
    reqs = [r for r in _requests(14, seed=13, qps=float("inf"), hi=300) if r.kind == "u8"]
    F.fht_debug_fail_next(-4, 1)
    try:
        srv = _serve(reqs, warm_plans=True, max_batch_images=len(reqs))
    finally:
        F.fht_debug_fail_next(0, 0)
    assert srv.batch_sizes[0] == 1 and len(srv.batch_sizes) == len(reqs)  # the retries
    _check_solo(reqs)
