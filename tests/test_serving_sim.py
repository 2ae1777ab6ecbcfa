"""Scheduler tests of the continuous-batching server on a simulated device
(virtual clock, no GPU): admission against the memory budget and slot
count, arrival-order admission, backfill, failure isolation."""
import pytest

import pfinputs
from paper_1506_01684_amd.serving import (Request, Server, SimBackend, VirtualClock,
                                          request_from_trace, summarize)


def _trace(n=40, rate=20.0, seed=3):
    tr = pfinputs.serving_trace(count=n, rate=rate, seed=seed, lateral=(16, 64), steps=(50, 400))
    return [request_from_trace(d) for d in tr]


def _run(reqs, **kw):
    clock = VirtualClock()
    b = SimBackend(clock, rate=kw.pop("rate", 5e8))
    s = Server(b, clock=clock, sleep=clock.sleep, **kw)
    res = s.run(reqs)
    return s, b, res


def test_every_request_finishes_after_it_arrives():
    reqs = _trace()
    s, b, res = _run(reqs, budget_bytes=5e9, max_slots=8, round_steps=20)
    assert [r.id for r in res] == sorted(r.id for r in reqs)
    for r in res:
        assert r.ok and r.arrival <= r.admitted <= r.finished
    summ = summarize(res)
    assert summ["failed"] == 0 and summ["p99_latency_s"] >= summ["p50_latency_s"] > 0


def test_budget_and_slots_are_never_exceeded():
    reqs = _trace(60)
    budget = 2e9
    s, b, res = _run(reqs, budget_bytes=budget, max_slots=5, round_steps=15)
    live = set()
    for ev, rid, t, used in s.events:
        assert used <= budget
        if ev == "admit":
            live.add(rid)
        else:
            live.discard(rid)
        assert len(live) <= 5


def test_without_backfill_admission_follows_arrival_order():
    reqs = _trace(30)
    s, b, res = _run(reqs, budget_bytes=1.5e9, max_slots=4, round_steps=10, backfill=False)
    order = [rid for ev, rid, t, u in s.events if ev == "admit"]
    arrival = [r.id for r in sorted(reqs, key=lambda r: (r.arrival, r.id))]
    assert order == arrival


def test_backfill_lets_small_requests_pass_a_blocked_head():
    p = pfinputs.p0_params(solid_height=4)
    big = Request(0, 0.0, (64, 64, 64), "fp32", 1000, p, 1, 4, 4)
    blocker = Request(1, 0.0, (64, 64, 64), "fp32", 1000, p, 1, 4, 4)
    small = [Request(2 + i, 0.001, (8, 8, 8), "fp32", 10, p, 1, 4, 4) for i in range(3)]
    reqs = [big, blocker] + small
    one_big = SimBackend(VirtualClock()).required_bytes(big)
    for backfill in (True, False):
        s, b, res = _run(list(reqs), budget_bytes=1.5 * one_big, max_slots=8, round_steps=50,
                         backfill=backfill)
        fin = {r.id: r.finished for r in res}
        if backfill:
            assert all(fin[q.id] < fin[0] for q in small)
        else:
            assert all(fin[q.id] > fin[0] for q in small)


def test_failed_admission_only_fails_that_request():
    reqs = _trace(12)

    class Flaky(SimBackend):
        def open(self, r):
            if r.id == 5:
                raise RuntimeError("device allocation failed")
            super().open(r)

    clock = VirtualClock()
    s = Server(Flaky(clock, rate=5e8), budget_bytes=5e9, max_slots=8, round_steps=20,
               clock=clock, sleep=clock.sleep)
    res = s.run(reqs)
    bad = [r for r in res if not r.ok]
    assert [r.id for r in bad] == [5] and "allocation" in bad[0].error
    assert sum(r.ok for r in res) == 11


def test_oversized_request_is_rejected_up_front():
    p = pfinputs.p0_params(solid_height=4)
    r = Request(0, 0.0, (512, 512, 512), "fp64", 10, p, 1, 4, 4)
    with pytest.raises(ValueError):
        _run([r], budget_bytes=1e6)


def test_sjf_with_cell_target_lowers_median_latency():
    """A burst of requests whose work spans two orders of magnitude: running
    everything at once (processor sharing) makes every request wait for the
    whole burst; admitting the shortest expected jobs first into a pack
    held near the cells that fill the device lets short jobs leave early."""
    reqs = _trace(60, rate=200.0)
    kw = dict(budget_bytes=1e12, max_slots=256, round_steps=10)
    _, _, fifo = _run(reqs, **kw)
    _, _, sjf = _run(reqs, policy="sjf", target_cells=2e5, **kw)
    f, j = summarize(fifo), summarize(sjf)
    assert j["failed"] == 0 and len(sjf) == len(reqs)
    assert j["p50_latency_s"] < 0.7 * f["p50_latency_s"]
    assert j["mean_latency_s"] < f["mean_latency_s"]


def test_sjf_ages_long_jobs_in():
    """A long job arriving first is not starved by a steady stream of short
    ones: its priority improves with the time it has waited."""
    p = pfinputs.p0_params(solid_height=4)
    long_job = Request(0, 0.0, (32, 32, 32), "fp32", 500, p, 1, 4, 4)
    # short jobs (0.4 ms of service each) arrive every 0.2 ms: without aging
    # the long job (33 ms) would wait until the stream has drained
    short = [Request(1 + i, 0.0002 * i, (16, 16, 16), "fp32", 50, p, 1, 4, 4) for i in range(600)]
    s, b, res = _run([long_job] + short, budget_bytes=1e12, max_slots=256, round_steps=10,
                     policy="sjf", target_cells=4096)
    by_id = {r.id: r for r in res}
    assert all(r.ok for r in res)
    last_short = max(r.finished for r in res if r.id != 0)
    assert by_id[0].finished < 0.5 * last_short


def test_unknown_policy_is_rejected():
    with pytest.raises(ValueError):
        Server(SimBackend(VirtualClock()), policy="lifo")


def test_cancelled_requests_leave_queue_and_pack():
    """One request withdrawn while it waits in the queue, one after it was
    admitted: both end as cancelled (the second with the steps it had done),
    the queued one is never opened, their memory is released at once, and
    every other request still finishes."""
    import dataclasses

    reqs = _trace(20)
    reqs[3] = dataclasses.replace(reqs[3], cancel_at=reqs[3].arrival)  # gone on arrival
    s0, _, first = _run(list(_trace(20)), budget_bytes=2e9, max_slots=3, round_steps=20)
    mid = next(r for r in first if r.id == 8)
    reqs[8] = dataclasses.replace(reqs[8], cancel_at=0.5 * (mid.admitted + mid.finished))
    s, b, res = _run(reqs, budget_bytes=2e9, max_slots=3, round_steps=20)
    by = {r.id: r for r in res}
    assert [r.id for r in res] == sorted(r.id for r in reqs)
    assert not by[3].ok and by[3].error == "cancelled" and 3 not in b.opened
    assert not by[8].ok and by[8].error.startswith("cancelled with")
    assert 0 < by[8].steps < reqs[8].steps
    assert all(r.ok for r in res if r.id not in (3, 8))
    ev = [e for e in s.events if e[0] == "cancel"]
    assert [e[1] for e in ev] == [8]
    before = [e for e in s.events if e[2] <= ev[0][2] and e[0] != "cancel"][-1]
    assert ev[0][3] < before[3]  # its bytes were released
    assert b.left == {} and b.cells == {}
