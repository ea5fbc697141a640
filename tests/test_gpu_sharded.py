"""Partitioned search (Sec. 6.5: random shards, one graph each, every query
searched in all shards, results aggregated) against the oracle composed the
same way: per-shard Alg. 1 in FP64, ids mapped back, merged by (distance,
global id)."""

import numpy as np
import pytest

import synth
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
SENT = 0xFFFFFFFF


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def _oracle_sharded(parts, bases, graphs, entries, q, K, L, K_out, metric="l2"):
    cand = [[] for _ in range(len(q))]
    for gids, b, g, e in zip(parts, bases, graphs, entries):
        oi, od, _, _ = core.search(b, g, e, q, K, L, metric)
        for r in range(len(q)):
            for i, dist in zip(oi[r], od[r]):
                if i != SENT:
                    cand[r].append((dist, int(gids[i])))
    ids = np.full((len(q), K_out), SENT, np.uint32)
    dd = np.full((len(q), K_out), np.inf)
    for r, c in enumerate(cand):
        c.sort()
        for t, (dist, gid) in enumerate(c[:K_out]):
            ids[r, t], dd[r, t] = gid, dist
    return ids, dd


@pytest.mark.parametrize("S,combined", [(2, True), (4, True), (4, False)])
def test_sharded_search_matches_oracle(S, combined):
    from paper_1907_06146_amd.sharded import ShardedIndex, partition
    cfg = synth.CONFIGS["c2s"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)[:64]
    parts = partition(len(base), S, seed=7)
    bases, graphs, entries = [], [], []
    for s, gids in enumerate(parts):
        b = base[gids]
        knn, _ = core.knn_graph(b, 40)
        e = np.random.default_rng(100 + s).choice(len(b), 10, replace=False).astype(np.uint32)
        graphs.append(core.nssg_build(b, knn, 60, 32, 60.0, e)["graph"])
        bases.append(b)
        entries.append(e)
    idx = ShardedIndex([_dev(b) for b in bases], [_dev(g) for g in graphs],
                       [_dev(e) for e in entries], parts, combined=combined)
    for K, L, K_out in [(10, 40, 10), (20, 32, 30)]:
        gi, gd = idx.search(_dev(q), K, L, K_out)
        torch.cuda.synchronize()
        oi, od = _oracle_sharded(parts, bases, graphs, entries, q, K, L, K_out)
        # integer data: FP32 distances are exact, so the merge must agree exactly
        assert np.array_equal(gi.cpu().numpy().view(np.uint32), oi)
        assert np.array_equal(gd.cpu().numpy().astype(np.float64), od)
    # BF16 shards hold these integers exactly: the same results
    idx16 = ShardedIndex([_dev(b).to(torch.bfloat16) for b in bases], [_dev(g) for g in graphs],
                         [_dev(e) for e in entries], parts, combined=combined)
    gi16, gd16 = idx16.search(_dev(q), 10, 40, 10)
    torch.cuda.synchronize()
    oi, od = _oracle_sharded(parts, bases, graphs, entries, q, 10, 40, 10)
    assert np.array_equal(gi16.cpu().numpy().view(np.uint32), oi)
    assert np.array_equal(gd16.cpu().numpy().astype(np.float64), od)
    # one index's rerank vectors or FP8 scale cannot describe S shards
    for kw in (dict(base_f32=_dev(bases[0])), dict(dim_scale=_dev(np.ones(128, np.float32))),
               dict(rerank_k=5)):
        with pytest.raises(ValueError):
            idx.search(_dev(q), 10, 40, **kw)


def test_merge_ties_and_padding():
    """Equal distances in different shards are ordered by global id; lists
    shorter than K leave padding; K_out above the real results pads."""
    from paper_1907_06146_amd import _lib
    from paper_1907_06146_amd.binding import _ptr
    import ctypes
    S, nq, K = 3, 2, 4
    loc = np.array([[[0, 1, SENT, SENT], [2, 0, 1, SENT]],
                    [[0, 1, 2, 3], [SENT, SENT, SENT, SENT]],
                    [[1, 0, SENT, SENT], [0, SENT, SENT, SENT]]], np.uint32)
    dist = np.array([[[1.0, 2.0, np.inf, np.inf], [0.5, 3.0, 3.0, np.inf]],
                     [[1.0, 1.0, 2.0, 9.0], [np.inf] * 4],
                     [[0.25, 2.0, np.inf, np.inf], [3.0, np.inf, np.inf, np.inf]]], np.float32)
    maps = [np.array([10, 4, 7]), np.array([3, 11, 5, 8]), np.array([6, 2])]
    idmap = np.concatenate(maps).astype(np.uint32)
    off = np.array([0, 3, 7], np.int64)
    K_out = 8
    oi = torch.empty((nq, K_out), dtype=torch.int32, device="cuda")
    od = torch.empty((nq, K_out), dtype=torch.float32, device="cuda")
    tl, td, tm, to = _dev(loc), _dev(dist), _dev(idmap), _dev(off)
    rc = _lib.lib().ssg_merge_shards(_ptr(tl), _ptr(td), S, nq, K, _ptr(tm), _ptr(to), len(idmap), K_out, _ptr(oi),
                                     _ptr(od), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(rc)
    torch.cuda.synchronize()
    gi, gd = oi.cpu().numpy().view(np.uint32), od.cpu().numpy()
    # expected: all real (dist, gid) pairs sorted, then padding
    for r in range(nq):
        real = sorted((float(dist[s, r, i]), int(maps[s][loc[s, r, i]]))
                      for s in range(S) for i in range(K) if loc[s, r, i] != SENT)
        exp_i = [g for _, g in real] + [SENT] * (K_out - len(real))
        exp_d = [d for d, _ in real] + [np.inf] * (K_out - len(real))
        assert gi[r].tolist() == exp_i[:K_out]
        assert np.array_equal(gd[r], np.array(exp_d[:K_out], np.float32))


def test_merge_treats_ids_outside_the_map_as_padding():
    """A local id whose map index falls outside [0, map_len) is never read
    through; it is padding."""
    from paper_1907_06146_amd import _lib
    from paper_1907_06146_amd.binding import _ptr
    import ctypes
    S, nq, K = 2, 1, 3
    loc = np.array([[[0, 5, SENT]], [[1, 0, 2]]], np.uint32)     # 5 and 2 are past their maps
    dist = np.array([[[1.0, 0.5, np.inf]], [[2.0, 3.0, 0.1]]], np.float32)
    idmap = np.array([40, 41, 50, 51], np.uint32)                 # shard 0: 40, 41; shard 1: 50, 51
    off = np.array([0, 2], np.int64)
    K_out = 6
    oi = torch.empty((nq, K_out), dtype=torch.int32, device="cuda")
    od = torch.empty((nq, K_out), dtype=torch.float32, device="cuda")
    tl, td, tm, to = _dev(loc), _dev(dist), _dev(idmap), _dev(off)
    rc = _lib.lib().ssg_merge_shards(_ptr(tl), _ptr(td), S, nq, K, _ptr(tm), _ptr(to), len(idmap), K_out,
                                     _ptr(oi), _ptr(od), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(rc)
    torch.cuda.synchronize()
    gi, gd = oi.cpu().numpy().view(np.uint32)[0], od.cpu().numpy()[0]
    # shard 0 local 5 -> index 5 >= 4: padding; shard 1 local 2 -> index 4 >= 4: padding
    assert gi.tolist() == [40, 51, 50, SENT, SENT, SENT]
    assert gd[:3].tolist() == [1.0, 2.0, 3.0] and np.isinf(gd[3:]).all()
