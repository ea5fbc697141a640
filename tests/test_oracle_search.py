"""Pins of the oracle's Alg. 1 (search) against facts fixed outside its code.

* a hand-traced trajectory (golden fixture, Alg. 1 on a path graph);
* complete graph => exact brute-force top-K (special case of Alg. 1);
* L >= number of reachable nodes => exact top-K (Sec. 4.2, "worst case");
* the independent pure-Python twin gives the same ids, keys, NDC and hops;
* permuting graph rows changes nothing (set semantics of the add-then-sort step);
* forgetting nodes once they leave the pool changes no result;
* (dist, id) tie order (the tie rule used in the proof of Theorem 3);
* on a unit-norm base, inner-product search follows the L2 trajectory
  (algebraic identity |q - x|^2 = |q|^2 + 1 - 2<q, x>).
"""

import json
import math
import os

import numpy as np
import pytest

from oracle import core, pyref

HERE = os.path.dirname(os.path.abspath(__file__))
SENT = core.SENT


def _golden():
    with open(os.path.join(HERE, "golden", "alg1_line.json")) as f:
        return json.load(f)


def _pad_rows(rows, R):
    g = np.full((len(rows), R), SENT, np.uint32)
    for i, r in enumerate(rows):
        g[i, :len(r)] = r
    return g


@pytest.mark.parametrize("case", range(4))
def test_hand_traced_path_graph(case):
    gd = _golden()
    c = gd["cases"][case]
    base = np.array(gd["points"], np.float32)
    g = _pad_rows(gd["graph"], 2)
    q = np.array([gd["query"]], np.float32)
    ids, dd, ndc, hops = core.search(base, g, gd["entry"], q, c["K"], c["L"])
    assert ids[0].tolist() == c["ids"]
    want = [math.inf if k == "inf" else k for k in c["keys"]]
    assert dd[0].tolist() == want
    assert int(ndc[0]) == c["ndc"] and int(hops[0]) == c["hops"]
    pi, pk, pn, ph = pyref.search(base, g, gd["entry"], q[0], c["K"], c["L"])
    assert pi == c["ids"] and pk == want and pn == c["ndc"] and ph == c["hops"]


def _random_graph(rng, n, R, fill=0.7):
    g = np.full((n, R), SENT, np.uint32)
    for i in range(n):
        k = rng.integers(1, R + 1) if rng.random() < fill else R
        nb = rng.choice(np.delete(np.arange(n), i), size=k, replace=False)
        g[i, :k] = nb
    return g


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_c_oracle_matches_python_twin(seed, metric):
    rng = np.random.default_rng(seed)
    n, d, R = 80, int(rng.integers(2, 9)), int(rng.integers(2, 9))
    base = rng.standard_normal((n, d)).astype(np.float32)
    if seed % 2:  # integer data: many exact ties, exercises the id tie-break
        base = np.rint(base * 2).astype(np.float32)
    g = _random_graph(rng, n, R)
    entry = rng.choice(n, size=5, replace=False).astype(np.uint32)
    Q = rng.standard_normal((12, d)).astype(np.float32)
    for L, K in [(1, 1), (3, 5), (8, 4), (20, 20), (100, 10)]:
        ids, dd, ndc, hops = core.search(base, g, entry, Q, K, L, metric)
        for r in range(len(Q)):
            pi, pk, pn, ph = pyref.search(base, g, entry, Q[r], K, L, metric)
            assert ids[r].tolist() == pi
            assert dd[r].tolist() == pk
            assert int(ndc[r]) == pn and int(hops[r]) == ph


def _int_data(rng, n, d):
    return rng.integers(0, 16, size=(n, d)).astype(np.float32)


@pytest.mark.parametrize("seed", range(4))
def test_complete_graph_gives_exact_topk(seed):
    rng = np.random.default_rng(100 + seed)
    n, d = 60, 4
    base = _int_data(rng, n, d)
    g = np.array([[j for j in range(n) if j != i] for i in range(n)], np.uint32)
    Q = _int_data(rng, 10, d)
    entry = np.array([int(rng.integers(n))], np.uint32)
    for K, L in [(1, 1), (5, 5), (10, 30), (10, 60)]:
        ids, dd, _, _ = core.search(base, g, entry, Q, K, L)
        # brute force with numpy on exact integer distances, ties by id
        d2 = ((Q[:, None, :].astype(np.int64) - base[None].astype(np.int64)) ** 2).sum(-1)
        for r in range(len(Q)):
            order = np.lexsort((np.arange(n), d2[r]))[:K]
            assert ids[r].tolist() == order.tolist()
            assert dd[r].tolist() == d2[r, order].astype(float).tolist()


def test_pool_as_large_as_graph_is_exact(c1_graph):
    base, q, g, entry, gt_i, gt_d = c1_graph
    n = base.shape[0]
    ids, dd, _, hops = core.search(base, g, entry, q, 10, n)
    assert np.array_equal(ids, gt_i[:, :10])
    assert np.array_equal(dd, gt_d[:, :10])
    assert (hops == n).all()  # every node is reachable from every navigating node


@pytest.mark.parametrize("seed", range(3))
def test_row_permutation_invariance(c1_graph, seed):
    base, q, g, entry, _, _ = c1_graph
    rng = np.random.default_rng(seed)
    gp = g.copy()
    for i in range(len(gp)):
        k = int((gp[i] != SENT).sum())
        gp[i, :k] = rng.permutation(gp[i, :k])
    a = core.search(base, g, entry, q, 10, 50)
    b = core.search(base, gp, entry, q, 10, 50)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_forgetting_evicted_nodes_is_result_neutral(c1_graph):
    base, q, g, entry, _, _ = c1_graph
    for L in (1, 10, 50, 200):
        a_i, a_d, a_n, a_h = core.search(base, g, entry, q, 10, L)
        b_i, b_d, b_n, b_h = core.search(base, g, entry, q, 10, L, forget=True)
        assert np.array_equal(a_i, b_i) and np.array_equal(a_d, b_d)
        assert np.array_equal(a_h, b_h)
        assert (b_n >= a_n).all()


def test_tie_break_by_smaller_id():
    # two nodes at the same distance from the query: the smaller id ranks first
    base = np.array([[0, 0], [1, 0], [-1, 0], [0, 5]], np.float32)
    g = _pad_rows([[3, 2, 1], [0], [0], [0]], 3)
    q = np.array([[0, 0.0]], np.float32)
    ids, dd, _, _ = core.search(base, g, [3], q, 3, 3)
    assert ids[0].tolist() == [0, 1, 2]
    assert dd[0].tolist() == [0.0, 1.0, 1.0]


def test_nearest_navigating_node_is_the_seed():
    # isolated nodes: the search can only return its seed
    base = np.array([[0, 0], [10, 0], [3, 0], [2, 0]], np.float32)
    g = np.full((4, 2), SENT, np.uint32)
    q = np.array([[2.4, 0]], np.float32)
    ids, dd, ndc, hops = core.search(base, g, [0, 1, 2, 3], q, 2, 5)
    assert ids[0].tolist() == [3, SENT] and ndc[0] == 4 and hops[0] == 1
    # equal distance to two navigating nodes: the smaller id seeds the pool
    q = np.array([[2.5, 0]], np.float32)
    ids, _, _, _ = core.search(base, g, [2, 3], q, 1, 5)
    assert ids[0, 0] == 2


def test_indexed_queries_find_themselves_on_exact_graph(c1_graph):
    base, q, g, entry, gt_i, _ = c1_graph
    # indexed queries are the last 20 rows; with L = n they are exact
    ids, dd, _, _ = core.search(base, g, entry, q[-20:], 1, base.shape[0])
    assert (dd[:, 0] == 0).all()


def test_bad_arguments_raise():
    base = np.zeros((4, 2), np.float32)
    g = np.full((4, 2), SENT, np.uint32)
    with pytest.raises(ValueError):
        core.search(base, g, [7], base[:1], 1, 1)  # entry id out of range
    with pytest.raises(ValueError):
        core.search(base, g, [0], base[:1], 0, 1)  # K < 1


def test_inner_product_on_unit_norm_base_equals_l2(c1_graph):
    """On a unit-norm base, |q - x|^2 = |q|^2 + 1 - 2<q, x>, so L2 and -IP
    order the candidates alike: Alg. 1 follows the same trajectory and the
    returned keys satisfy that identity (pins the IP key's sign and form)."""
    base, q, g, entry, _, _ = c1_graph
    b = base.astype(np.float64)
    b /= np.linalg.norm(b, axis=1, keepdims=True)
    b = b.astype(np.float32)
    i2, d2, n2, h2 = core.search(b, g, entry, q, 10, 50, "l2")
    ii, di, ni, hi = core.search(b, g, entry, q, 10, 50, "ip")
    same = (i2 == ii).all(1)
    assert same.mean() > 0.99
    qq = (q.astype(np.float64) ** 2).sum(1)[:, None]
    xx = (b.astype(np.float64) ** 2).sum(1)  # 1 up to the fp32 rounding of the rows
    # dists of the IP search, converted with the identity, agree with the
    # L2 search's (rows that differ may only do so through near-equal keys)
    conv = qq + xx[ii.astype(np.int64)] + 2.0 * di
    assert np.allclose(conv[same], d2[same], rtol=1e-12, atol=1e-12)
    assert np.allclose(np.sort(d2[~same], 1), np.sort(qq[~same] + 1.0 + 2.0 * di[~same], 1),
                       rtol=1e-6, atol=1e-6)
    assert np.array_equal(h2[same], hi[same])
