"""Serving loop on the GPU: requests admitted while others run overlap on the
device, and every request's result is the same alone and in the mix."""

import numpy as np
import pytest

import synth
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def test_results_identical_alone_and_in_the_mix():
    from paper_1907_06146_amd.serve import GpuDevice, Scheduler, poisson_requests, run, summarize
    cfg = synth.CONFIGS["c2s"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
    tb, tg, te = _dev(base), _dev(g), _dev(entry)
    rng = np.random.default_rng(3)
    reqs, _ = poisson_requests(rng, 80, 20000.0, q, [32, 64, 96, 128], 10, max_batch=64)
    dev = GpuDevice(tb, tg, te, n_slots=6, max_batch=64, max_K=10)
    sch = Scheduler(dev, n_slots=6, inflight_budget=4096)
    done = run(reqs, sch)
    assert len(done) == len(reqs) and sch.max_running_seen >= 2
    s = summarize(done)
    assert s["p99_ms"] >= s["p50_ms"] > 0
    # each request alone, one at a time
    alone_dev = GpuDevice(tb, tg, te, n_slots=1, max_batch=64, max_K=10)
    for r in sorted(done, key=lambda r: r.rid):
        solo = Scheduler(alone_dev, n_slots=1, inflight_budget=4096)
        r2 = type(r)(r.rid, 0.0, r.queries, r.L, r.K)
        out = run([r2], solo)[0]
        assert np.array_equal(out.ids, r.ids) and np.array_equal(out.dists, r.dists)
    # and the results are Alg. 1's (integer data: exact)
    for r in done[:10]:
        oi, od, _, _ = core.search(base, g, entry, r.queries, r.K, r.L)
        assert np.array_equal(r.ids.view(np.uint32), oi)


def test_continuous_batching_matches_single_requests():
    """Requests batched together (each query with its own request's L and K)
    return exactly what each request returns when searched alone."""
    from paper_1907_06146_amd import search
    from paper_1907_06146_amd.serve import BatchScheduler, GpuBatchDevice, poisson_requests, run
    cfg = synth.CONFIGS["c2s"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
    tb, tg, te = _dev(base), _dev(g), _dev(entry)
    rng = np.random.default_rng(5)
    reqs, _ = poisson_requests(rng, 120, 50000.0, q, [32, 64, 96, 128, 200, 300], 10, max_batch=64)
    for i, r in enumerate(reqs):  # mixed result counts too
        r.K = (10, 1, 7)[i % 3]
    dev = GpuBatchDevice(tb, tg, te, n_slots=2, max_batch=512, max_K=10)
    sch = BatchScheduler(dev, n_slots=2, max_batch=512)
    done = run(reqs, sch)
    assert len(done) == len(reqs)
    assert sch.batches < len(reqs)  # requests were grouped
    for r in sorted(done, key=lambda r: r.rid):
        ids, dd = search(tb, tg, te, _dev(r.queries), r.K, r.L)
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy(), r.ids), r.rid
        assert np.array_equal(dd.cpu().numpy(), r.dists), r.rid
    for r in done[:8]:  # and the results are Alg. 1's (integer data: exact)
        oi, _, _, _ = core.search(base, g, entry, r.queries, r.K, r.L)
        assert np.array_equal(r.ids.view(np.uint32), oi)
