"""Continuous-batching scheduler on a scripted fake device (no GPU)."""

import numpy as np
import pytest

from paper_1907_06146_amd.serve import FakeDevice, Request, Scheduler, poisson_requests, run, summarize


class SimClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-4  # every look at the clock advances simulated time
        return self.t


def _reqs(sizes, arrivals, L=32, K=4):
    return [Request(i, a, np.zeros((b, 8), np.float32), L, K) for i, (b, a) in enumerate(zip(sizes, arrivals))]


def test_fifo_slots_and_budget():
    clk = SimClock()
    dev = FakeDevice(lambda r: 0.01 * len(r.queries) / 10, clk)
    sch = Scheduler(dev, n_slots=3, inflight_budget=50)
    reqs = _reqs([10, 20, 30, 5, 40, 10, 10], [0.0, 0.0, 0.0, 0.001, 0.002, 0.003, 0.003])
    done = run(reqs, sch, clock=clk)
    assert len(done) == len(reqs)
    order = [rid for _, rid in dev.launched]
    assert order == sorted(order)  # admitted in arrival order
    assert sch.max_running_seen <= 3 and sch.max_inflight_seen <= 50
    assert sch.max_running_seen >= 2  # requests overlapped
    for r in done:
        assert r.arrival <= r.admitted <= r.finished
        assert (r.ids == np.arange(4) + r.rid).all()  # each result went to its own request


def test_oversized_request_runs_alone():
    clk = SimClock()
    dev = FakeDevice(lambda r: 0.005, clk)
    sch = Scheduler(dev, n_slots=4, inflight_budget=16)
    done = run(_reqs([8, 100, 8], [0.0, 0.0, 0.0]), sch, clock=clk)
    assert len(done) == 3
    big = next(r for r in done if len(r.queries) == 100)
    others = [r for r in done if r is not big]
    for o in others:  # never co-running with the oversized one
        assert o.finished <= big.admitted or o.admitted >= big.finished


def test_requests_admitted_while_others_run():
    clk = SimClock()
    dev = FakeDevice(lambda r: 0.02, clk)
    sch = Scheduler(dev, n_slots=4, inflight_budget=1000)
    reqs = _reqs([5, 5, 5], [0.0, 0.005, 0.010])
    done = run(reqs, sch, clock=clk)
    a, b, c = sorted(done, key=lambda r: r.rid)
    assert b.admitted < a.finished and c.admitted < a.finished  # continuous, not a queue drain
    s = summarize(done)
    assert s["requests"] == 3 and s["queries"] == 15 and s["p99_ms"] >= s["p50_ms"] > 0


def test_poisson_generator():
    rng = np.random.default_rng(0)
    pool = np.arange(40, dtype=np.float32).reshape(10, 4)
    reqs, picks = poisson_requests(rng, 200, 1000.0, pool, [32, 64], 10, max_batch=8)
    arr = np.array([r.arrival for r in reqs])
    assert (np.diff(arr) > 0).all()
    assert abs(np.mean(np.diff(arr)) - 1e-3) < 3e-4
    assert all(1 <= len(r.queries) <= 8 and r.L in (32, 64) for r in reqs)
    assert all(np.array_equal(r.queries, pool[p]) for r, p in zip(reqs, picks))


def test_bad_configuration():
    with pytest.raises(ValueError):
        Scheduler(FakeDevice(lambda r: 0, SimClock()), 0, 10)


def test_batch_scheduler_groups_waiting_requests():
    from paper_1907_06146_amd.serve import BatchScheduler, FakeBatchDevice
    clk = SimClock()
    dev = FakeBatchDevice(lambda reqs: 0.002, clk)
    sch = BatchScheduler(dev, n_slots=2, max_batch=64)
    # a burst of requests at t = 0, then stragglers
    sizes = [10, 20, 30, 40, 5, 100, 7, 3]
    arrivals = [0.0] * 6 + [0.01, 0.01]
    reqs = _reqs(sizes, arrivals)
    done = run(reqs, sch, clock=clk)
    assert len(done) == len(reqs)
    batches = [rids for _, rids in dev.launched]
    flat = [rid for b in batches for rid in b]
    assert flat == sorted(flat)  # arrival order kept across batches
    for b in batches:  # each batch fits the budget unless it is one oversized request
        tot = sum(sizes[i] for i in b)
        assert tot <= 64 or len(b) == 1
    assert [5] in batches  # the 100-query request ran alone
    assert sch.max_running_seen <= 2
    for r in done:
        assert r.arrival <= r.admitted <= r.finished
        assert (r.ids == np.arange(4) + r.rid).all() and r.ids.shape == (len(r.queries), 4)


def test_batch_scheduler_rejects_bad_sizes():
    from paper_1907_06146_amd.serve import BatchScheduler, FakeBatchDevice
    with pytest.raises(ValueError):
        BatchScheduler(FakeBatchDevice(lambda r: 0.0, SimClock()), n_slots=0, max_batch=8)
