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


def test_serving_in_the_serving_workload_form():
    """The serving form of the 5M x 96 workload on a small index of the same
    kind (unit-norm, inner product, R = 32): BF16 storage with an FP32 rerank
    of K = 10, requests of 1..256 queries with L in {32, 48, ..., 256}, 5 %
    of the queries base points, continuous batching admitted by an LDS / HBM
    byte budget tight enough to make requests queue. Each request gets the
    same bits alone and in the mix; the batched results equal the plain
    search; and every row is the oracle's (Alg. 1 on the dequantized
    vectors, FP64, then the FP32 rerank), or differs only by key ties, or
    parts from the oracle's trajectory at a tie."""
    from parity_util import assert_parity, classify

    from oracle import precision as P
    from paper_1907_06146_amd import quantize, search
    from paper_1907_06146_amd.serve import (BatchScheduler, DeviceBudget, GpuBatchDevice,
                                            poisson_requests, run)
    cfg = dict(synth.CONFIGS["c4s"], R=32, knn_k=64, nq_unindexed=1900, nq_indexed=100)
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
    tb, tg, te = _dev(base), _dev(g), _dev(entry)
    qb, _ = quantize(tb, "bf16")
    torch.cuda.synchronize()
    deq = P.bf16_decode(qb.view(torch.int16).cpu().numpy().view(np.uint16))
    rng = np.random.default_rng(17)
    L_choices = list(range(32, 257, 16))
    reqs, picks = poisson_requests(rng, 60, 30000.0, q, L_choices, 10, max_batch=256)
    dev = GpuBatchDevice(qb, tg, te, n_slots=3, max_batch=1024, max_K=10, metric="ip",
                         base_f32=tb, rerank=True)
    full = dev.budget()
    # a budget of about 600 searches of L = 256: requests must wait for bytes
    tight = DeviceBudget(600 * full.lds_of(256), full.hbm_bytes, full.lds_of, full.hbm_of)
    sch = BatchScheduler(dev, n_slots=3, max_batch=1024, budget=tight)
    done = run(reqs, sch)
    assert len(done) == len(reqs) and all(r.error is None for r in done)
    assert sch.budget_waits > 0 and sch.max_inflight_seen[0] <= tight.lds_bytes
    assert sch.batches < len(reqs)  # requests were grouped
    done = sorted(done, key=lambda r: r.rid)
    # alone: each request through its own scheduler, one batch of one request
    solo_dev = GpuBatchDevice(qb, tg, te, n_slots=1, max_batch=256, max_K=10, metric="ip",
                              base_f32=tb, rerank=True)
    T = 4 * 256 + 64
    for r in done:
        r2 = type(r)(r.rid, 0.0, r.queries, r.L, r.K)
        out = run([r2], BatchScheduler(solo_dev, n_slots=1, max_batch=256))[0]
        assert np.array_equal(out.ids, r.ids) and np.array_equal(out.dists, r.dists), r.rid
        # the plain search gives the same bits
        pi, pd, ptr = search(qb, tg, te, _dev(r.queries), r.K, r.L, "ip", base_f32=tb, rerank_k=r.K,
                             trace=T)
        torch.cuda.synchronize()
        assert np.array_equal(pi.cpu().numpy(), r.ids) and np.array_equal(pd.cpu().numpy(), r.dists)
        # and the oracle's rows, row by row
        oi, _ = P.search_precision(base, deq, g, entry, r.queries, r.K, r.L, "ip", rerank=r.K)
        otr = core.search(deq, g, entry, r.queries, r.K, r.L, "ip", trace=T)[4]
        rows = classify(base, r.queries, r.ids.view(np.uint32), oi, "ip", 1e-5, ptr.cpu().numpy(),
                        otr, search_base=deq)
        assert_parity(rows, 0.9, f"request {r.rid}")
    # indexed queries (base points) find themselves first
    ids_idx = synth.indexed_query_ids(cfg)
    first = {int(i): None for i in ids_idx}
    for r, p in zip(done, picks):
        for row, qi in zip(r.ids, p):
            if qi >= cfg["nq_unindexed"]:
                first[int(ids_idx[qi - cfg["nq_unindexed"]])] = int(row[0])
    seen = [k for k, v in first.items() if v is not None]
    assert seen and np.mean([first[k] == k for k in seen]) >= 0.95
