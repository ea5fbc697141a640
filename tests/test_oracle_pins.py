"""Pins of the oracle's helper steps that the search and graph caches rely on.

* ``pair_keys``: the FP64 key of Sec. 2.1's distance (squared) or of the
  negative inner product, checked against exact integer arithmetic (integer
  vectors make every key an integer, computed here in int64) and against the
  independent pure-Python twin.
* ``knn_graph_ivf``: step 1 of Alg. 3 for the large workloads (an
  approximate kNN graph). With every cell probed it must be the exact kNN
  graph; with fewer probes each row must be the exact top K of the points
  in the probed cells, by brute force over exactly those points.
* ``knn_refine``: each output row is the exact top K over the node's list and
  its first J neighbours' lists (brute force over that union), never farther
  than the input row position by position.
* the expansion trace of ``search`` (the order in which Alg. 1 takes the
  first unchecked node), against the pure-Python twin.
"""

import numpy as np
import pytest

import synth
from oracle import core, pyref

SENT = core.SENT


def _int_data(n=1500, nq=40, seed=3):
    cfg = dict(synth.CONFIGS["c2s"], n=n, nq_unindexed=nq, nq_indexed=0, comps=6, seed=seed)
    base = synth.base_vectors(cfg)
    return base, synth.queries(cfg, base)


def _float_data(n=1200, nq=30):
    cfg = dict(synth.CONFIGS["c4s"], n=n, nq_unindexed=nq, comps=5, seed=77)
    base = synth.base_vectors(cfg)
    return base, synth.queries(cfg, base)


def _topk_of(base, x, cand, K, skip=None):
    """Exact top K of point x over the candidate ids (FP64 squared L2 by
    numpy, ties by the smaller id), skip excluded."""
    cand = np.unique(np.asarray([c for c in cand if c != skip and c != SENT], np.int64))
    dd = ((base[cand].astype(np.float64) - x.astype(np.float64)) ** 2).sum(1)
    order = np.lexsort((cand, dd))[:K]
    return cand[order], dd[order]


# ------------------------------------------------------------------ pair_keys
@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_pair_keys_exact_integer_keys(metric):
    base, q = _int_data()
    rng = np.random.default_rng(0)
    ids = rng.integers(0, len(base), (len(q), 17)).astype(np.uint32)
    ids[:, -1] = SENT
    got = core.pair_keys(base, q, ids, metric)
    bi = base.astype(np.int64)
    qi = q.astype(np.int64)
    for r in range(len(q)):
        for t in range(16):
            x = bi[ids[r, t]]
            want = int(((qi[r] - x) ** 2).sum()) if metric == "l2" else -int((qi[r] * x).sum())
            assert got[r, t] == want
            assert got[r, t] == pyref._key(q[r], base[ids[r, t]], metric)
    assert np.isinf(got[:, -1]).all()


def test_pair_keys_float_data_match_python_twin_and_search():
    base, q = _float_data()
    rng = np.random.default_rng(1)
    ids = rng.integers(0, len(base), (len(q), 9)).astype(np.uint32)
    for metric in ("l2", "ip"):
        got = core.pair_keys(base, q, ids, metric)
        for r in range(len(q)):
            assert got[r].tolist() == [pyref._key(q[r], base[v], metric) for v in ids[r]]
    # the keys Alg. 1 returns are the same function of the same pairs
    knn, _ = core.knn_graph(base, 12)
    g = core.nssg_prune(base, knn, 24, 10)
    entry = np.arange(0, len(base), 97, dtype=np.uint32)
    si, sd, _, _ = core.search(base, g, entry, q, 8, 20, "ip")
    assert np.array_equal(core.pair_keys(base, q, si, "ip"), sd)


# ------------------------------------------------------------------ IVF kNN graph
@pytest.mark.parametrize("kind", ["int", "float"])
def test_ivf_with_every_cell_probed_is_the_exact_knn_graph(kind):
    base, _ = _int_data(n=1200) if kind == "int" else _float_data(n=1000)
    K = 15
    ei, ed = core.knn_graph(base, K)
    ii, idd = core.knn_graph_ivf(base, K, nlist=8, nprobe=8, seed=5, sample=600)
    assert np.array_equal(ii, ei)
    assert np.array_equal(idd, ed)


def test_ivf_rows_are_exact_over_the_probed_cells():
    base, _ = _int_data(n=1600)
    K, nlist, nprobe, seed = 12, 10, 3, 9
    lab, probe, cent = core.ivf_partition(base, nlist, nprobe, seed, sample=800)
    # the partition: every point in the cell of a nearest centroid (up to
    # fp32 rounding of the scores), probe lists = the nprobe nearest centroids
    c64 = cent.astype(np.float64)
    d2 = ((base.astype(np.float64)[:, None, :] - c64[None]) ** 2).sum(-1)
    best = d2.min(1)
    scale = (base.astype(np.float64) ** 2).sum(1) + (c64 ** 2).sum(1).max()
    assert (d2[np.arange(len(base)), lab] <= best + 1e-5 * scale).all()
    cd = ((c64[:, None, :] - c64[None]) ** 2).sum(-1)
    for c in range(nlist):
        kth = np.sort(cd[c])[nprobe - 1]
        assert len(set(probe[c].tolist())) == nprobe
        assert (cd[c, probe[c]] <= kth * (1 + 1e-9) + 1e-6).all()
        assert c in probe[c]
    ids, dd = core.knn_graph_ivf(base, K, nlist, nprobe, seed, sample=800)
    members = [np.nonzero(lab == c)[0] for c in range(nlist)]
    for i in range(0, len(base), 7):
        cand = np.concatenate([members[c] for c in probe[lab[i]]])
        wi, wd = _topk_of(base, base[i], cand, K, skip=i)
        m = len(wi)
        assert ids[i, :m].tolist() == wi.tolist(), i
        assert np.array_equal(dd[i, :m], wd)
        assert (ids[i, m:] == SENT).all()


# ------------------------------------------------------------------ refinement
def test_knn_refine_is_exact_over_the_neighbour_lists():
    base, _ = _int_data(n=1400)
    K, J = 10, 4
    rng = np.random.default_rng(4)
    # a deliberately poor start: the exact list of a random other point
    exact, _ = core.knn_graph(base, K)
    start = exact[rng.permutation(len(base))].copy()
    for i in range(len(base)):  # no self ids
        start[i][start[i] == i] = exact[i][0]
        _, first = np.unique(start[i], return_index=True)
        keep = np.zeros(K, bool)
        keep[first] = True
        start[i][~keep] = SENT
        start[i] = np.concatenate([start[i][keep], start[i][~keep]])
    out = core.knn_refine(base, start, J, rounds=1)
    b64 = base.astype(np.float64)
    for i in range(len(base)):
        cand = [v for v in start[i]]
        for a in range(J):
            if start[i, a] != SENT:
                cand += list(start[start[i, a]])
        wi, _ = _topk_of(base, base[i], cand, K, skip=i)
        assert out[i, :len(wi)].tolist() == wi.tolist(), i
        assert (out[i, len(wi):] == SENT).all()
        # never farther than the input row, position by position
        din = np.where(start[i] != SENT, ((b64[start[i].astype(np.int64) % len(base)] - b64[i]) ** 2).sum(1),
                       np.inf)
        dout = np.where(out[i] != SENT, ((b64[out[i].astype(np.int64) % len(base)] - b64[i]) ** 2).sum(1),
                        np.inf)
        assert (dout <= np.sort(din)).all()


def test_knn_refine_keeps_an_exact_graph():
    base, _ = _float_data(n=900)
    exact, _ = core.knn_graph(base, 8)
    assert np.array_equal(core.knn_refine(base, exact, 8, rounds=2), exact)


# ------------------------------------------------------------------ expansion trace
def test_search_trace_matches_python_twin():
    rng = np.random.default_rng(12)
    for trial in range(6):
        n, d, R = int(rng.integers(20, 80)), int(rng.integers(2, 9)), int(rng.integers(2, 7))
        base = rng.integers(0, 9, (n, d)).astype(np.float32)
        g = np.full((n, R), SENT, np.uint32)
        for i in range(n):
            k = int(rng.integers(0, R + 1))
            g[i, :k] = rng.choice(np.delete(np.arange(n), i), size=k, replace=False)
        entry = rng.choice(n, size=int(rng.integers(1, 5)), replace=False).astype(np.uint32)
        q = rng.integers(0, 9, (5, d)).astype(np.float32)
        K, L = 4, int(rng.integers(1, 12))
        cap = n + 2
        ci, cd, cn, ch, ct = core.search(base, g, entry, q, K, L, trace=cap)
        for r in range(len(q)):
            pi, pk, pn, ph, order = pyref.search(base, g, entry, q[r], K, L, trace=True)
            assert ct[r, :ch[r]].tolist() == order
            assert (ct[r, ch[r]:] == SENT).all()
            assert len(set(order)) == len(order)  # a node is expanded at most once
        # a shorter record is the prefix of the full one
        _, _, _, _, short = core.search(base, g, entry, q, K, L, trace=2)
        assert np.array_equal(short, ct[:, :2])


def test_search_does_not_depend_on_the_order_of_a_row():
    """Alg. 1 takes every neighbour of the expanded node and re-sorts the pool
    by (distance, id): permuting the ids within each adjacency row changes no
    result, no expansion count and no expansion record."""
    rng = np.random.default_rng(8)
    base = rng.integers(0, 40, (600, 16)).astype(np.float32)
    knn, _ = core.knn_graph(base, 20)
    entry = rng.choice(600, 5, replace=False).astype(np.uint32)
    g = core.nssg_build(base, knn, 30, 12, 60.0, entry)["graph"]
    perm = g.copy()
    for r in range(len(perm)):
        k = int((perm[r] != core.SENT).sum())
        perm[r, :k] = rng.permutation(perm[r, :k])
    assert not np.array_equal(perm, g)
    q = rng.integers(0, 40, (50, 16)).astype(np.float32)
    a = core.search(base, g, entry, q, 10, 40, trace=200)
    b = core.search(base, perm, entry, q, 10, 40, trace=200)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
