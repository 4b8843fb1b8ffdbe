"""The serving scheduler on the CPU: a fake executor with a simulated clock
checks admission by HBM budget, slot reuse, FIFO order, continuous admission
(no waiting for a batch to finish) and the latency statistics."""
import math

import numpy as np
import pytest

from paper_1709_04488_amd.serve import (FakeExecutor, Request, Scheduler, SimClock, summarize)


def _req(rid, n, arrival, kind="evaluate"):
    return Request(rid, arrival, kind, {"x": np.zeros(n)}, {}, 0)


def _run(reqs, budget, slots, cost):
    clock = SimClock()
    ex = FakeExecutor(clock, cost)
    sched = Scheduler(ex, budget, slots, clock)
    recs = sched.run(reqs)
    return recs, ex, sched


def test_all_complete_and_latency_is_done_minus_arrival():
    reqs = [_req(i, 1000, 0.1 * i) for i in range(10)]
    recs, ex, _ = _run(reqs, 1 << 30, 4, lambda r: 0.05)
    assert all(not r.error for r in recs)
    for r in recs:
        assert r.done >= r.admitted >= r.arrival
        assert r.latency == pytest.approx(0.05)


def test_budget_limits_concurrency():
    # each request needs fixed + 500 B/particle + 168 B/particle arrays
    n = 100_000
    per = (1 << 20) + 500 * n + 168 * n
    reqs = [_req(i, n, 0.0) for i in range(6)]
    recs, ex, sched = _run(reqs, int(2.5 * per), 8, lambda r: 1.0)
    starts = sorted(t for t, _, _ in ex.starts)
    # at most two fit at once: starts come in pairs one second apart
    assert starts == [0.0, 0.0, 1.0, 1.0, 2.0, 2.0]
    assert sched.peak_bytes <= int(2.5 * per)


def test_slots_are_reused_and_capacity_counted():
    reqs = [_req(i, 50_000, 0.0) for i in range(4)]
    recs, ex, sched = _run(reqs, 1 << 30, 2, lambda r: 0.5)
    slots = [s for _, _, s in ex.starts]
    assert sorted(set(slots)) == [0, 1]
    assert max(r.done for r in recs) == pytest.approx(1.0)


def test_continuous_admission_does_not_wait_for_batch():
    # a long request and a stream of short ones: short ones keep flowing through
    # the second slot while the long one runs
    reqs = [_req(0, 1000, 0.0)] + [_req(i, 1000, 0.01 * i) for i in range(1, 6)]
    cost = lambda r: 10.0 if r.rid == 0 else 0.1
    recs, ex, _ = _run(reqs, 1 << 30, 2, cost)
    assert recs[0].done == pytest.approx(10.0)
    assert all(r.done < 1.0 for r in recs[1:])


def test_request_larger_than_budget_is_rejected_not_blocking():
    reqs = [_req(0, 10_000_000, 0.0), _req(1, 1000, 0.0)]
    recs, _, _ = _run(reqs, 64 << 20, 2, lambda r: 0.1)
    assert recs[0].error == "exceeds HBM budget"
    assert not recs[1].error and recs[1].done == pytest.approx(0.1)


def test_fifo_order_of_admission():
    reqs = [_req(i, 1000, 0.0) for i in range(5)]
    recs, ex, _ = _run(reqs, 1 << 30, 1, lambda r: 1.0)
    assert [rid for _, rid, _ in ex.starts] == [0, 1, 2, 3, 4]


def test_summary_percentiles():
    reqs = [_req(i, 1000, float(i)) for i in range(100)]
    recs, _, _ = _run(reqs, 1 << 30, 4, lambda r: 0.01 * (1 + r.rid % 10))
    s = summarize(recs, max(r.done for r in recs))
    lat = sorted(r.latency for r in recs)
    assert s["latency_p50_ms"] == pytest.approx(np.percentile(lat, 50) * 1e3)
    assert s["latency_p99_ms"] == pytest.approx(np.percentile(lat, 99) * 1e3)
    assert s["completed"] == 100


@pytest.mark.timeout(30)
def test_idle_slot_capacity_is_released_when_it_blocks_admission():
    # two large requests leave both slots holding capacity; the next, larger
    # request fits the budget only once that idle capacity is released
    per = lambda n: (1 << 20) + 500 * n + 168 * n  # noqa: E731
    budget = int(1.4e9)
    reqs = [_req(0, 1_000_000, 0.0), _req(1, 1_000_000, 0.0), _req(2, 1_500_000, 5.0)]
    assert 2 * per(1_000_000) <= budget < per(1_500_000) + 2 * (1 << 20) + 500 * 1_000_000 * 2
    recs, ex, sched = _run(reqs, budget, 2, lambda r: 1.0)
    assert all(not r.error for r in recs)
    assert recs[2].admitted == pytest.approx(5.0)
    assert ex.released, "idle capacity was never released"
    assert sched.peak_bytes <= budget


def test_block_integration_requests_carry_the_timeline():
    """integrate_requests(block=True): the same sets, each on block time-steps
    (block_lmax 20, limiter 2), nsteps counting level-0 steps; the global
    variant leaves the setups untouched."""
    from paper_1709_04488_amd import serve as S
    glob = S.integrate_requests(4, 3, n_max_side=6)
    blk = S.integrate_requests(4, 3, n_max_side=6, block=True)
    for g, b in zip(glob, blk):
        assert "block_lmax" not in g.setup
        assert b.setup["block_lmax"] == 20 and b.setup["block_lim"] == 2
        assert b.nsteps == g.nsteps == 3 and b.kind == g.kind == "integrate"
        assert all(np.array_equal(b.arrays[k], g.arrays[k]) for k in g.arrays)
