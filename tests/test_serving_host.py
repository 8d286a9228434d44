"""Scheduling logic of the serving loop on the CPU.

A fake clock and a fake executor stand in for the GPU: a batch "runs" for a
time proportional to its pixels on the stream it was given, and arrivals
follow a seeded Poisson process on the fake clock, so every test is
deterministic.  Plans are real (the planner is host code).
"""
import time

import numpy as np
import pytest

import paper_2411_07351_amd as F
from paper_2411_07351_amd import serving as S
import workloads as WL


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def idle(self, next_event):
        if next_event is None:
            time.sleep(1e-4)  # waiting for planner threads: real time only
        else:
            self.t = max(self.t, next_event)


class FakeExecutor:
    def __init__(self, clock, streams=2, px_per_s=1e9, overhead=1e-4):
        self.clock, self.px_per_s, self.overhead = clock, px_per_s, overhead
        self.free_at = [0.0] * streams
        self.launched = []
        self.fail = 0

    @property
    def n_streams(self):
        return len(self.free_at)

    def launch(self, reqs, slot):
        if self.fail > 0:
            self.fail -= 1
            raise F.FhtError(-4, "fake enqueue")
        start = max(self.clock.now(), self.free_at[slot])
        end = start + self.overhead + sum(r.pixels for r in reqs) / self.px_per_s
        self.free_at[slot] = end
        h = {"start": start, "end": end, "slot": slot, "rids": [r.rid for r in reqs],
             "kinds": {r.kind for r in reqs}}
        self.launched.append(h)
        return h

    def done(self, h):
        return self.clock.now() >= h["end"]

    def outputs(self, h):
        return None

    def release(self, h):
        pass

    def next_event(self):
        ends = [h["end"] for h in self.launched if h["end"] > self.clock.now()]
        return min(ends) if ends else None


def _requests(n, qps, seed=0, lo=64, hi=512):
    rng = WL.rng_for(5, salt=seed)
    items = WL.serving_requests(rng, n, lo, hi)
    arr = WL.poisson_arrivals(rng, n, qps)
    return [S.Request(i, img, float(t)) for i, ((kind, img), t) in enumerate(zip(items, arr))]


def _serve(reqs, budget=1 << 40, **kw):
    clock = FakeClock()
    ex = FakeExecutor(clock, streams=kw.pop("streams", 2), px_per_s=kw.pop("px_per_s", 1e9))
    srv = S.Server(ex, budget, clock=clock, plan_threads=4, **kw)
    try:
        srv.run(reqs)
    finally:
        srv.close()
    return srv, ex


def test_poisson_stream_all_done_and_latency_bounds():
    reqs = _requests(40, qps=2000.0)
    srv, ex = _serve(reqs)
    assert all(r.status == "done" for r in reqs)
    for r in reqs:
        assert r.arrival <= r.t_admit <= r.t_launch <= r.t_done
        # at least its own share of the batch it ran in
        assert r.latency >= r.pixels / 1e9
    s = S.summarize(reqs)
    assert s["done"] == 40 and s["p50_ms"] <= s["p99_ms"]
    assert s["mpixel_per_s"] > 0


def test_arrivals_are_deterministic():
    a = _requests(30, qps=5000.0, seed=1)
    b = _requests(30, qps=5000.0, seed=1)
    _serve(a)
    _serve(b)
    assert [r.t_done for r in a] == [r.t_done for r in b]
    assert [r.batch for r in a] == [r.batch for r in b]


def test_batches_never_mix_dtypes_and_respect_limits():
    reqs = _requests(60, qps=float("inf"), seed=2)
    srv, ex = _serve(reqs, max_batch_images=5, max_batch_px=400_000)
    by_id = {r.rid: r for r in reqs}
    for h in ex.launched:
        assert len(h["kinds"]) == 1
        assert len(h["rids"]) <= 5
        px = sum(by_id[i].pixels for i in h["rids"])
        assert len(h["rids"]) == 1 or px <= 400_000


def test_continuous_batching_overlaps_batches():
    # requests keep arriving while earlier batches run: later batches are
    # launched before earlier ones complete, on the other stream
    reqs = _requests(40, qps=20000.0, seed=3)
    srv, ex = _serve(reqs, px_per_s=2e8, max_batch_images=4)
    hs = sorted(ex.launched, key=lambda h: h["start"])
    overlaps = sum(1 for a, b in zip(hs, hs[1:]) if b["start"] < a["end"] and a["slot"] != b["slot"])
    assert overlaps >= 1
    assert max(len(h["rids"]) for h in hs) > 1  # queued arrivals joined a batch
    assert all(r.status == "done" for r in reqs)


def test_tiny_budget_serialises_requests():
    rng = WL.rng_for(5, salt=4)
    reqs = [S.Request(i, WL.edge_map(rng, 200, 300), 0.0) for i in range(12)]
    need = S.footprint(F.Plan(200, 300, "u8", "S"), "u8")  # one request, not two
    srv, ex = _serve(reqs, budget=need)
    assert all(r.status == "done" for r in reqs)
    assert srv.peak_in_use <= need
    # admitted one at a time: no two requests were on the device together
    spans = sorted((r.t_launch, r.t_done) for r in reqs)
    assert all(b[0] >= a[1] for a, b in zip(spans, spans[1:]))
    assert srv.peak_running == 1


def test_request_over_budget_is_rejected_and_others_served():
    reqs = _requests(10, qps=1000.0, seed=5)
    small = min(reqs, key=lambda r: r.pixels)
    budget = S.footprint(F.Plan(small.rows, small.cols, small.kind, "S"), small.kind)
    srv, ex = _serve(reqs, budget=budget)
    for r in reqs:
        fp = S.footprint(r.plan, r.kind)
        assert r.status == ("done" if fp <= budget else "rejected")
    assert any(r.status == "rejected" for r in reqs)
    assert small.status == "done"


def test_bad_requests_are_rejected():
    reqs = _requests(4, qps=1000.0, seed=6)
    reqs.append(S.Request(99, np.zeros((8, 8), dtype=np.int16), 0.0))
    _serve(reqs)
    assert reqs[-1].status == "rejected"
    assert all(r.status == "done" for r in reqs[:-1])


def test_failed_batch_is_retried_per_request():
    reqs = _requests(16, qps=float("inf"), seed=7)
    clock = FakeClock()
    ex = FakeExecutor(clock)
    ex.fail = 1
    srv = S.Server(ex, 1 << 40, clock=clock, max_batch_images=8)
    for r in reqs:  # planned up front, so the first (failing) batch holds several requests
        srv.plans.get(r.rows, r.cols, r.kind, r.split).result()
    srv.run(reqs)
    srv.close()
    assert all(r.status == "done" for r in reqs)


def test_failure_of_a_lone_request_fails_only_that_request():
    reqs = _requests(10, qps=1000.0, seed=8)
    clock = FakeClock()
    ex = FakeExecutor(clock)
    ex.fail = 1
    srv = S.Server(ex, 1 << 40, clock=clock, max_batch_images=1)
    srv.run(reqs)
    srv.close()
    failed = [r for r in reqs if r.status == "failed"]
    assert len(failed) == 1 and "FHT_EHIP" in failed[0].error
    assert sum(r.status == "done" for r in reqs) == 9


def test_plan_cache_close_fails_pending_plans_cleanly():
    cache = S.PlanCache(threads=1, capacity=8)
    done = cache.get(64, 80, "u8", "S")
    assert done.result().rows == 64
    pending = [cache.get(3000 + k, 3000, "u8", "S") for k in range(4)]
    cache.close()
    assert done.result().rows == 64  # taken before the close: still valid
    for f in pending:
        try:
            f.result()
        except RuntimeError as e:
            assert "closed" in str(e)
    with pytest.raises(F.FhtError):
        cache.get(70, 70, "u8", "S")


def test_plan_cache_reuses_plans():
    cache = S.PlanCache(threads=2, capacity=2)
    a = cache.get(64, 80, "u8", "S").result()
    b = cache.get(64, 80, "u8", "S").result()
    assert a is b
    cache.get(65, 80, "u8", "S").result()
    cache.get(66, 80, "u8", "S").result()
    assert cache.get(64, 80, "u8", "S").result() is not a  # evicted
    cache.close()


def test_fault_hook_of_the_c_abi():
    # fht_batch_upload returns the injected status before touching any memory
    plan = F.Plan(17, 23, "u8", "S")
    fake = 1 << 40  # never dereferenced: the hook returns first
    b = F.fht_batch_prepare([plan.handle], [fake], [fake])
    try:
        assert F.fht_batch_tables_bytes(b) > 0
        with pytest.raises(F.FhtError) as e:
            F.fht_batch_run(b, fake, None)  # not uploaded yet
        assert e.value.status == -1
        F.fht_debug_fail_next(-5, 2)
        for _ in range(2):
            with pytest.raises(F.FhtError) as e:
                F.fht_batch_upload(b, fake, F.fht_batch_tables_bytes(b), None)
            assert e.value.status == -5
        with pytest.raises(F.FhtError) as e:
            F.fht_batch_upload(b, fake, 1, None)  # too small: argument check first
        assert e.value.status == -1
        with pytest.raises(F.FhtError) as e:  # the staged form needs its host buffer
            F.fht_batch_upload_staged(b, fake, F.fht_batch_tables_bytes(b), 0, None)
        assert e.value.status == -1
    finally:
        F.fht_debug_fail_next(0, 0)
        F.fht_batch_destroy(b)


class _HeldFirstPlans:
    """Plan source whose first request's plan is finished only after every
    other plan has been taken (a large plan still being made), or after 2000
    polls (so that a loop that waited for it in arrival order ends too)."""

    def __init__(self, n):
        self.n, self.taken, self.calls, self.polls = n, 0, 0, 0

    def get(self, rows, cols, kind, split):
        first = self.calls == 0
        self.calls += 1
        src = self

        class Fut:
            def __init__(self):
                self.plan = F.Plan(rows, cols, kind, split)

            def done(self):
                if first:
                    src.polls += 1
                return not first or src.taken >= src.n - 1 or src.polls > 2000

            def result(self):
                if not first:
                    src.taken += 1
                return self.plan

        return Fut()

    def close(self):
        pass


def test_a_plan_still_being_made_holds_up_no_later_request():
    reqs = _requests(12, 1e9, seed=13)
    for r in reqs:
        r.arrival = 0.0
    clock = FakeClock()
    ex = FakeExecutor(clock)
    srv = S.Server(ex, 1 << 40, clock=clock, plan_threads=1)
    srv.plans.close()
    srv.plans = _HeldFirstPlans(len(reqs))
    srv.run(reqs)
    assert all(r.status == "done" for r in reqs)
    first = next(r for r in reqs if r.rid == 0)
    # the other requests were planned, admitted and launched before request 0
    assert all(r.t_launch <= first.t_launch for r in reqs)
    assert 0 not in ex.launched[0]["rids"]
