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
    for b in batches:  # each batch fits the batch size
        assert sum(sizes[i] for i in b) <= 64
    # the 100-query request can never fit a batch: finished at once with an error
    big = next(r for r in done if r.rid == 5)
    assert big.error and big.ids is None and 5 not in flat
    assert sch.max_running_seen <= 2
    for r in done:
        if r.error:
            continue
        assert r.arrival <= r.admitted <= r.finished
        assert (r.ids == np.arange(4) + r.rid).all() and r.ids.shape == (len(r.queries), 4)
    s = summarize(done)
    assert s["rejected"] == 1 and s["requests"] == len(reqs) - 1


def test_batch_scheduler_rejects_bad_sizes():
    from paper_1907_06146_amd.serve import BatchScheduler, FakeBatchDevice
    with pytest.raises(ValueError):
        BatchScheduler(FakeBatchDevice(lambda r: 0.0, SimClock()), n_slots=0, max_batch=8)


def _budget(lds, hbm, per_L=lambda L: 100 * L, per_K=lambda K: 10 * K):
    from paper_1907_06146_amd.serve import DeviceBudget
    return DeviceBudget(lds, hbm, per_L, per_K)


def test_batch_scheduler_queues_until_bytes_free_up():
    """Two requests that do not fit the LDS budget together: the second waits
    for the first to finish although a batch slot is free, and the in-flight
    bytes never pass the budget."""
    from paper_1907_06146_amd.serve import BatchScheduler, FakeBatchDevice
    clk = SimClock()
    dev = FakeBatchDevice(lambda reqs: 0.01, clk)
    bud = _budget(lds=100 * 64 * 30, hbm=10 ** 9)  # 30 queries of L = 64 at a time
    sch = BatchScheduler(dev, n_slots=4, max_batch=1000, budget=bud)
    reqs = _reqs([20, 20, 5], [0.0, 0.0, 0.0], L=64)
    done = run(reqs, sch, clock=clk)
    a, b, c = sorted(done, key=lambda r: r.rid)
    assert all(r.error is None for r in done)
    assert b.admitted >= a.finished  # over budget while a ran: queued
    assert c.admitted >= a.finished  # FIFO: c waits behind b
    assert [rids for _, rids in dev.launched] == [[0], [1, 2]]
    assert sch.budget_waits > 0
    assert sch.max_inflight_seen[0] <= bud.lds_bytes
    assert sch.inflight == [0, 0]  # every admitted byte was released


def test_batch_scheduler_budget_by_pool_size():
    """The LDS price grows with L: small-L requests share the budget that one
    large-L request takes alone."""
    from paper_1907_06146_amd.serve import BatchScheduler, FakeBatchDevice
    clk = SimClock()
    dev = FakeBatchDevice(lambda reqs: 0.005, clk)
    bud = _budget(lds=100 * 512 * 8, hbm=10 ** 9)
    sch = BatchScheduler(dev, n_slots=8, max_batch=1000, budget=bud)
    reqs = [Request(0, 0.0, np.zeros((8, 8), np.float32), 512, 4),
            Request(1, 0.0, np.zeros((8, 8), np.float32), 64, 4),
            Request(2, 0.0, np.zeros((8, 8), np.float32), 64, 4)]
    done = run(reqs, sch, clock=clk)
    assert [rids for _, rids in dev.launched] == [[0], [1, 2]]
    big = next(r for r in done if r.rid == 0)
    assert all(r.admitted >= big.finished for r in done if r.rid)


def test_batch_scheduler_hbm_budget_and_rejections():
    from paper_1907_06146_amd.serve import BatchScheduler, FakeBatchDevice
    clk = SimClock()
    dev = FakeBatchDevice(lambda reqs: 0.003, clk)
    dev.max_queries, dev.max_K = 64, 10
    bud = _budget(lds=10 ** 9, hbm=10 * 10 * 40)  # 40 queries of K = 10 in flight
    sch = BatchScheduler(dev, n_slots=4, max_batch=1000, budget=bud)
    assert sch.max_batch == 64  # capped at what a device slot holds
    reqs = [Request(0, 0.0, np.zeros((30, 8), np.float32), 32, 10),
            Request(1, 0.0, np.zeros((30, 8), np.float32), 32, 10),   # waits for HBM
            Request(2, 0.0, np.zeros((4, 8), np.float32), 32, 11),    # K over the slot
            Request(3, 0.0, np.zeros((41, 8), np.float32), 32, 10),   # over the whole budget
            Request(4, 0.0, np.zeros((65, 8), np.float32), 32, 1)]    # over a batch
    done = run(reqs, sch, clock=clk)
    byid = {r.rid: r for r in done}
    assert byid[1].admitted >= byid[0].finished
    for rid in (2, 3, 4):
        assert byid[rid].error and byid[rid].ids is None
    assert byid[0].error is None and byid[1].error is None
    assert [rids for _, rids in dev.launched] == [[0], [1]]


def test_request_scheduler_rejects_what_a_slot_cannot_hold():
    clk = SimClock()
    dev = FakeDevice(lambda r: 0.002, clk)
    dev.max_queries, dev.max_K = 16, 8
    sch = Scheduler(dev, n_slots=2, inflight_budget=100)
    reqs = [Request(0, 0.0, np.zeros((17, 8), np.float32), 32, 4),
            Request(1, 0.0, np.zeros((4, 8), np.float32), 32, 9),
            Request(2, 0.0, np.zeros((4, 8), np.float32), 32, 4)]
    done = run(reqs, sch, clock=clk)
    byid = {r.rid: r for r in done}
    assert byid[0].error and byid[1].error and byid[2].error is None
    assert [rid for _, rid in dev.launched] == [2]


def test_device_budget_rejects_nonpositive():
    with pytest.raises(ValueError):
        _budget(0, 10)
