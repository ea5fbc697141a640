"""Pins of the oracle's indexing side (Alg. 2, Alg. 3) and of its kNN step.

* the 60-degree boundary is exact and is not a conflict (integer 3-D vectors);
* Lemma 1: an exact SSG at 60 degrees has out-degree <= kissing number
  (6 in 2-D, 12 in 3-D);
* Theorem 1: on an exact SSG, greedy search with pool 1 reaches any indexed
  query from any start;
* the C pruning equals the pure-Python twin;
* alpha = 0 disables pruning, which exposes the candidate set of Alg. 3 and of
  reverse-neighbour checking so they can be compared with a direct reading;
* NSSG invariants: degree <= R, angles >= alpha except DFS edges, no
  duplicates or self loops, every node reachable from every navigating node;
* kNN by coarse pass + certificate equals a full brute-force scan.
"""

import numpy as np
import pytest

import synth
from oracle import core, pyref

SENT = core.SENT


def _angle_ok(base, i, a, b, alpha):
    u = base[a].astype(np.float64) - base[i]
    v = base[b].astype(np.float64) - base[i]
    c = u @ v / np.sqrt((u @ u) * (v @ v))
    return c <= np.cos(np.radians(alpha)) + 1e-9


def test_exact_sixty_degrees_is_not_a_conflict():
    # |a| = |b| = sqrt(2), <a, b> = 1  =>  angle exactly 60 degrees
    base = np.array([[0, 0, 0], [1, 1, 0], [1, 0, 1], [2, 1, 1]], np.float32)
    adj, deg = core.ssg_exact(base[:3], 60.0)
    assert sorted(adj[0, :deg[0]].tolist()) == [1, 2]
    # (2,1,1) is 30 degrees from (1,1,0) and longer: pruned from node 0
    adj, deg = core.ssg_exact(base, 60.0)
    assert 3 not in adj[0, :deg[0]].tolist()
    assert pyref.ssg_prune(base, 0, [1, 2, 3], 60.0) == [1, 2]


@pytest.mark.parametrize("d,bound", [(2, 6), (3, 12)])
def test_lemma1_degree_bound(d, bound):
    rng = np.random.default_rng(d)
    base = rng.standard_normal((400, d)).astype(np.float32)
    _, deg = core.ssg_exact(base, 60.0)
    assert deg.max() <= bound
    # smaller alpha -> denser graph (Sec. 3.2)
    _, deg30 = core.ssg_exact(base, 30.0)
    assert deg30.mean() > deg.mean()


@pytest.mark.parametrize("d", [2, 3, 8])
@pytest.mark.parametrize("alpha", [30.0, 45.0, 60.0])
def test_theorem1_greedy_reaches_indexed_query(d, alpha):
    rng = np.random.default_rng(int(alpha) + d)
    n = 300
    base = rng.standard_normal((n, d)).astype(np.float32)
    adj, deg = core.ssg_exact(base, alpha)
    targets = rng.choice(n, size=40, replace=False)
    for t in targets:
        start = int(rng.integers(n))
        ids, dd, _, _ = core.search(base, adj, [start], base[t:t + 1], 1, 1)
        assert ids[0, 0] == t and dd[0, 0] == 0.0


@pytest.mark.parametrize("seed", range(3))
def test_c_pruning_matches_python_twin(seed):
    rng = np.random.default_rng(seed)
    n, d = 70, 5
    base = rng.standard_normal((n, d)).astype(np.float32)
    if seed == 1:
        base = np.rint(base * 3).astype(np.float32)  # ties and exact zeros
    for alpha in (30.0, 60.0):
        adj, deg = core.ssg_exact(base, alpha)
        for i in range(n):
            assert adj[i, :deg[i]].tolist() == pyref.ssg_prune(base, i, range(n), alpha)


def _literal_candidates(knn, i, l):
    P = []
    seen = {i}
    for nb in knn[i]:
        for v in [nb] + list(knn[nb]):
            if v not in seen:
                seen.add(v)
                P.append(int(v))
        if len(P) >= l:
            break
    return P


def test_expansion_rule_and_reverse_candidates():
    rng = np.random.default_rng(7)
    n, d, K, l = 200, 6, 5, 12
    base = rng.standard_normal((n, d)).astype(np.float32)
    knn, _ = core.knn_graph(base, K)
    R = 64
    g1 = core.nssg_prune(base, knn, l, R, alpha=0.0)  # alpha 0: nothing conflicts
    for i in range(n):
        P = _literal_candidates(knn, i, l)
        want = sorted(P, key=lambda v: (float(((base[v].astype(np.float64) - base[i]) ** 2).sum()), v))
        got = g1[i][g1[i] != SENT].tolist()
        assert got == want[:R]
        assert pyref.ssg_prune(base, i, P, 0.0, R) == got
    g2 = core.nssg_reverse(base, g1, alpha=0.0)
    rev = [set() for _ in range(n)]
    for i in range(n):
        for v in g1[i][g1[i] != SENT]:
            rev[v].add(i)
    for j in range(n):
        cand = set(g1[j][g1[j] != SENT].tolist()) | rev[j]
        want = sorted(cand, key=lambda v: (float(((base[v].astype(np.float64) - base[j]) ** 2).sum()), v))
        assert g2[j][g2[j] != SENT].tolist() == want[:R]


def _reachable(g, root):
    seen = np.zeros(len(g), bool)
    seen[root] = True
    st = [int(root)]
    while st:
        v = st.pop()
        for w in g[v]:
            if w == SENT:
                break
            if not seen[w]:
                seen[w] = True
                st.append(int(w))
    return seen


@pytest.mark.parametrize("name", ["c1", "c2s"])
def test_nssg_invariants(name):
    cfg = synth.CONFIGS[name]
    base = synth.base_vectors(cfg)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    res = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)
    g, added = res["graph"], res["dfs_edges"]
    n, R = g.shape
    assert R == cfg["R"]
    dfs = set(map(tuple, added.tolist()))
    rng = np.random.default_rng(0)
    for i in range(n):
        row = g[i]
        k = int((row != SENT).sum())
        assert (row[k:] == SENT).all() and (row[:k] < n).all()
        ids = row[:k].tolist()
        assert len(set(ids)) == k and i not in ids
    # angle invariant on a sample of nodes (all pairs of non-DFS out-edges)
    for i in rng.choice(n, size=300, replace=False):
        ids = [v for v in g[i][g[i] != SENT].tolist() if (i, v) not in dfs]
        for x in range(len(ids)):
            for y in range(x + 1, len(ids)):
                assert _angle_ok(base, i, ids[x], ids[y], cfg["alpha"])
    for e in entry:
        assert _reachable(g, e).all()


def test_dfs_spanning_connects_components():
    # two far-apart groups with no edge between them; one root in group A
    rng = np.random.default_rng(3)
    a = rng.standard_normal((30, 2)).astype(np.float32)
    b = (rng.standard_normal((30, 2)) + 100).astype(np.float32)
    base = np.concatenate([a, b])
    knn = np.empty((60, 5), np.uint32)
    for grp in (range(0, 30), range(30, 60)):
        idx = np.array(list(grp))
        for i in grp:
            d2 = ((base[idx] - base[i]) ** 2).sum(1)
            order = [int(idx[j]) for j in np.lexsort((idx, d2)) if idx[j] != i][:5]
            knn[i] = order
    g = core.nssg_reverse(base, core.nssg_prune(base, knn, 10, 8))
    g2, added = core.dfs_connect(base, g, [0], 20)
    assert _reachable(g2, 0).all()
    assert len(added) >= 1
    for w, u in added:
        assert g2[w].tolist().count(u) == 1


@pytest.mark.parametrize("metric", ["l2", "ip"])
def test_knn_and_ground_truth_equal_full_scan(metric):
    rng = np.random.default_rng(11)
    base = rng.standard_normal((3000, 24)).astype(np.float32)
    q = rng.standard_normal((50, 24)).astype(np.float32)
    a = core.topk(base, q, 20, metric, margin=0, col_block=700)  # forces fallbacks
    b = core.bruteforce(base, q, 20, metric)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    ki, kd = core.knn_graph(base[:800], 15, col_block=300)
    bi, bd = core.bruteforce(base[:800], base[:800], 15, skip=np.arange(800))
    assert np.array_equal(ki, bi) and np.array_equal(kd, bd)
    # and against an independent pure-Python scan
    for r in range(3):
        pi, pk = pyref.bruteforce(base[:300], q[r], 5, metric)
        ci, cd = core.bruteforce(base[:300], q[r:r + 1], 5, metric)
        assert ci[0].tolist() == pi and cd[0].tolist() == pk


def test_recall_definition():
    gt = np.array([[1, 2, 3], [4, 5, 6]], np.uint32)
    r = np.array([[3, 2, 9], [SENT, 6, 4]], np.uint32)
    assert core.recall_at(r, gt, 3) == 4 / 6
