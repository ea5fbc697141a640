"""ctypes wrapper over the FP64 C oracle (test infrastructure only).

Functions follow the paper's steps:
  knn_graph       step 1 of Alg. 3: exact kNN graph (brute force)
  ground_truth    exact top-K of queries (the G set of Eq. 1)
  nssg_build      Alg. 3: expansion, SSG pruning, reverse-neighbour checking,
                  navigating nodes and DFS spanning
  search          Alg. 1 from the nearest navigating node (Sec. 4.1)
  ssg_exact       Alg. 2 over all pairs (tiny n)
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssg_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

SENT = 0xFFFFFFFF
METRICS = {"l2": 0, "ip": 1}


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (portable x86-64, no contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        cmd = ["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
               "-shared", "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB)
            P = ctypes.c_void_p
            i64, i32, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_double
            L.orc_bruteforce.argtypes = [P, i64, i32, P, i64, P, i32, i32, P, P]
            L.orc_rerank.argtypes = [P, i64, i32, P, i64, P, P, i32, i32, i32, P, P]
            L.orc_nssg_prune.argtypes = [P, i64, i32, P, i32, i32, i32, f64, i32, P]
            L.orc_nssg_reverse.argtypes = [P, i64, i32, P, i32, f64, P]
            L.orc_dfs_connect.argtypes = [P, i64, i32, P, i32, P, i32, i32, P, i64]
            L.orc_dfs_connect.restype = i64
            L.orc_threads.argtypes = [i32]
            L.orc_threads.restype = i32
            L.orc_search.argtypes = [P, i64, i32, P, i32, P, i32, P, i64, i32, i32, P, P, i32,
                                     i32, P, P, P, P, P, i32]
            L.orc_ssg_exact.argtypes = [P, i64, i32, f64, i32, P, P]
            L.orc_pair_keys.argtypes = [P, i64, i32, P, i64, P, i32, i32, P]
            L.orc_knn_refine.argtypes = [P, i64, i32, P, i32, i32, P]
            _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def cos2(alpha_deg: float) -> float:
    """cos^2(alpha); exactly 0.25 for 60 degrees (exact conflict boundary)."""
    if alpha_deg == 60.0:
        return 0.25
    return math.cos(math.radians(alpha_deg)) ** 2


# ------------------------------------------------------------------ brute force
def bruteforce(base, Q, K: int, metric: str = "l2", skip=None):
    """Exact top-K of every row of Q over base by full scan, FP64 keys,
    (dist, id) order. ``skip`` gives one id per row to leave out."""
    base, Q = _f32(base), _f32(Q)
    n, d = base.shape
    nq = Q.shape[0]
    ids = np.empty((nq, K), np.uint32)
    dd = np.empty((nq, K), np.float64)
    sk = None if skip is None else np.ascontiguousarray(skip, dtype=np.int64)
    rc = lib().orc_bruteforce(_p(base), n, d, _p(Q), nq, _p(sk), K, METRICS[metric], _p(ids), _p(dd))
    if rc:
        raise ValueError(f"orc_bruteforce rc={rc}")
    return ids, dd


def _exact_from_scores_is_safe(base: np.ndarray) -> bool:
    """fp32 score arithmetic is exact for integer vectors in [0, 255] with
    d <= 128: every product, partial sum and squared norm is an integer below
    2^24, so the coarse pass orders exactly like FP64."""
    d = base.shape[1]
    if d > 128:
        return False
    return bool(np.all(base >= 0) and np.all(base <= 255) and np.all(np.rint(base) == base))


def topk(base, Q, K: int, metric: str = "l2", exclude_self: bool = False,
         margin: int = 28, block: int = 2048, col_block: int = 262144, verbose: bool = False):
    """Exact top-K (FP64 keys, (dist, id) order) of every row of Q over base.

    A coarse fp32 pass (a library matmul, then a library top-k) keeps K+margin
    candidates per row; the C oracle recomputes their exact FP64 keys and
    selects K. A row is certified when the (K+margin)-th coarse score, minus a
    bound on the fp32 rounding error, is still above the exact K-th key:
    then no point outside the candidates can belong to the top K. Rows that
    fail the certificate are recomputed by a full FP64 scan.
    With exclude_self, row r is base row r and r itself is excluded.
    """
    import torch

    base, Q = _f32(base), _f32(Q)
    n, d = base.shape
    nq = Q.shape[0]
    C = min(n, K + margin + (1 if exclude_self else 0))
    tb = torch.from_numpy(base)
    exact = _exact_from_scores_is_safe(base) and _exact_from_scores_is_safe(Q)
    if metric == "l2":
        ny = (tb.double() ** 2).sum(1).float()
    u = 2.0 ** -24
    maxnorm2 = float((base.astype(np.float64) ** 2).sum(1).max())
    cand = np.empty((nq, C), np.int64)
    cth = np.empty(nq, np.float64)  # C-th coarse score (lower bound for non-candidates)
    for lo in range(0, nq, block):
        hi = min(nq, lo + block)
        tq = torch.from_numpy(Q[lo:hi])
        best_v = None
        best_i = None
        for clo in range(0, n, col_block):
            chi = min(n, clo + col_block)
            cb = tb[clo:chi]
            if metric == "l2":
                s = torch.addmm(ny[clo:chi].unsqueeze(0).expand(hi - lo, -1), tq, cb.t(),
                                beta=1.0, alpha=-2.0)
            else:
                s = -(tq @ cb.t())
            kk = min(C, chi - clo)
            v, i = torch.topk(s, kk, dim=1, largest=False, sorted=False)
            i = i + clo
            if best_v is None:
                best_v, best_i = v, i
            else:
                v = torch.cat([best_v, v], 1)
                i = torch.cat([best_i, i], 1)
                best_v, sel = torch.topk(v, min(C, v.shape[1]), dim=1, largest=False, sorted=False)
                best_i = torch.gather(i, 1, sel)
        cand[lo:hi] = best_i.numpy()
        cth[lo:hi] = best_v.max(1).values.double().numpy()
        if verbose:
            print(f"  coarse {hi}/{nq}", flush=True)
    skip = np.arange(nq, dtype=np.int64) if exclude_self else None
    ids = np.empty((nq, K), np.uint32)
    dd = np.empty((nq, K), np.float64)
    rc = lib().orc_rerank(_p(base), n, d, _p(Q), nq, _p(skip), _p(cand), C, K, METRICS[metric],
                          _p(ids), _p(dd))
    if rc:
        raise ValueError(f"orc_rerank rc={rc}")
    if C >= n:  # every point was a candidate: nothing to certify
        return ids, dd
    qn2 = (Q.astype(np.float64) ** 2).sum(1)
    if exact:
        err = np.zeros(nq)
    else:
        g = 4.0 * (d + 4) * u
        if metric == "l2":
            err = g * (maxnorm2 + 2.0 * np.sqrt(qn2 * maxnorm2)) + g * maxnorm2
        else:
            err = g * np.sqrt(qn2 * maxnorm2)
    lower = cth - err + (qn2 if metric == "l2" else 0.0)
    kth = dd[:, K - 1]
    bad = np.nonzero(~(lower > kth))[0]
    if len(bad):
        if verbose:
            print(f"  {len(bad)} rows fall back to a full scan", flush=True)
        bi, bd = bruteforce(base, Q[bad], K, metric, skip=None if skip is None else skip[bad])
        ids[bad] = bi
        dd[bad] = bd
    return ids, dd


def knn_graph(base, K: int, **kw):
    """Exact K-nearest-neighbour graph (step 1 of Alg. 3, built by brute force
    instead of nn-descent): row i lists the K nearest other points of i in
    (squared L2, id) order."""
    return topk(base, base, K, "l2", exclude_self=True, **kw)


def ivf_partition(base, nlist: int, nprobe: int, seed: int, iters: int = 6,
                  sample: int = 100_000):
    """Cells and probe lists of the IVF candidate pass of ``knn_graph_ivf``.

    k-means (Lloyd iterations on a seeded sample of at most ``sample`` rows)
    gives nlist centroids; every point is assigned to its nearest centroid
    (fp32 scores); cell c probes the nprobe cells whose centroids are nearest
    to c's centroid (FP64 scores). Returns (labels[n] int64,
    probe[nlist, nprobe] int64, centroids float32 [nlist, d])."""
    import torch

    base = _f32(base)
    n, d = base.shape
    tb = torch.from_numpy(base)
    rng = np.random.default_rng(seed)
    samp = tb[torch.from_numpy(np.sort(rng.choice(n, size=min(sample, n), replace=False)))]
    cent = samp[torch.from_numpy(rng.choice(len(samp), size=nlist, replace=False))].clone()

    def assign(x):
        out = torch.empty(len(x), dtype=torch.int64)
        cn = (cent.double() ** 2).sum(1).float()
        for lo in range(0, len(x), 65536):
            s = torch.addmm(cn.unsqueeze(0).expand(min(65536, len(x) - lo), -1), x[lo:lo + 65536],
                            cent.t(), beta=1.0, alpha=-2.0)
            out[lo:lo + 65536] = s.argmin(1)
        return out

    for _ in range(iters):
        a = assign(samp)
        sums = torch.zeros_like(cent).index_add_(0, a, samp)
        cnt = torch.bincount(a, minlength=nlist).float()
        keep = cnt > 0
        cent[keep] = sums[keep] / cnt[keep, None]
    lab = assign(tb).numpy()
    cn = (cent.double() ** 2).sum(1)
    cd = cn[:, None] + cn[None, :] - 2.0 * (cent.double() @ cent.double().t())
    probe = torch.topk(cd, min(nprobe, nlist), dim=1, largest=False).indices.numpy()
    return lab, probe, cent.numpy()


def knn_graph_ivf(base, K: int, nlist: int, nprobe: int, seed: int, iters: int = 6,
                  sample: int = 100_000, margin: int = 16, verbose: bool = False):
    """Approximate K-nearest-neighbour graph for the large workloads (step 1
    of Alg. 3 asks only for an approximate kNN graph; the paper uses
    nn-descent, or an IVF index in Alg. 4).

    The base set is split into cells by ``ivf_partition``. The candidates of
    every point of cell c are the points of the cells c probes; a coarse fp32
    pass keeps K + margin + 1 of them and the C oracle picks the K nearest
    other points by exact FP64 keys, in (dist, id) order. Points outside the
    probed cells are the only source of error (``knn_accuracy`` measures it
    against a full scan); with nprobe = nlist the result is the exact kNN
    graph whenever the coarse pass keeps the true K nearest (always, for
    integer data, where the fp32 scores are exact).
    """
    import torch

    base = _f32(base)
    n, d = base.shape
    tb = torch.from_numpy(base)
    lab, probe, _ = ivf_partition(base, nlist, nprobe, seed, iters, sample)
    order = np.argsort(lab, kind="stable")
    starts = np.searchsorted(lab[order], np.arange(nlist + 1))
    ny = (tb.double() ** 2).sum(1).float()
    C = K + margin + 1
    cand = np.full((n, C), -1, np.int64)
    for c in range(nlist):
        pts = order[starts[c]:starts[c + 1]]
        if len(pts) == 0:
            continue
        cid = np.concatenate([order[starts[j]:starts[j + 1]] for j in probe[c]])
        ti = torch.from_numpy(cid)
        k = min(C, len(cid))
        cand_t = tb[ti].t().contiguous()
        rows = max(256, (1 << 28) // max(1, len(cid)))  # bound the score block to ~1 GiB
        for lo in range(0, len(pts), rows):
            p = pts[lo:lo + rows]
            s = torch.addmm(ny[ti].unsqueeze(0).expand(len(p), -1), tb[torch.from_numpy(p)],
                            cand_t, beta=1.0, alpha=-2.0)
            idx = torch.topk(s, k, dim=1, largest=False).indices.numpy()
            cand[p, :k] = cid[idx]
        if verbose and c % 200 == 0:
            print(f"  ivf cell {c}/{nlist}", flush=True)
    skip = np.arange(n, dtype=np.int64)
    ids = np.empty((n, K), np.uint32)
    dd = np.empty((n, K), np.float64)
    rc = lib().orc_rerank(_p(base), n, d, _p(base), n, _p(skip), _p(cand), C, K, 0, _p(ids), _p(dd))
    if rc:
        raise ValueError(f"orc_rerank rc={rc}")
    return ids, dd


def knn_refine(base, knn, J: int, rounds: int = 1):
    """Neighbour-of-neighbour refinement of an approximate kNN graph: each
    node's candidates are its list plus its first J neighbours' lists; exact
    FP64 keys keep the K nearest. Never loses a closer neighbour it had."""
    base = _f32(base)
    cur = np.ascontiguousarray(knn, dtype=np.uint32)
    n, d = base.shape
    for _ in range(rounds):
        out = np.empty_like(cur)
        rc = lib().orc_knn_refine(_p(base), n, d, _p(cur), cur.shape[1], J, _p(out))
        if rc:
            raise ValueError(f"orc_knn_refine rc={rc}")
        cur = out
    return cur


def knn_accuracy(base, knn, sample: int = 500, seed: int = 0):
    """1-NN and K-NN accuracy of a kNN graph against a full FP64 scan on a
    sample of rows (the two accuracy columns of Table 5)."""
    n, K = knn.shape
    rows = np.sort(np.random.default_rng(seed).choice(n, size=min(sample, n), replace=False))
    ex, _ = bruteforce(base, base[rows], K, "l2", skip=rows.astype(np.int64))
    one = float(np.mean(knn[rows, 0] == ex[:, 0]))
    kk = float(np.mean([len(set(a.tolist()) & set(b.tolist())) / K for a, b in zip(knn[rows], ex)]))
    return one, kk


def ground_truth(base, Q, K: int, metric: str = "l2", **kw):
    """Exact top-K answer set of every query (the G of Eq. 1)."""
    return topk(base, Q, K, metric, exclude_self=False, **kw)


# ------------------------------------------------------------------ Alg. 3
def nssg_prune(base, knn, l: int, R: int, alpha: float = 60.0, expand: str = "literal"):
    """First loop of Alg. 3: candidates from the kNN graph (neighbours and
    neighbours' neighbours until |P| >= l), then SSG angular pruning to at
    most R edges."""
    base = _f32(base)
    knn = np.ascontiguousarray(knn, dtype=np.uint32)
    n, d = base.shape
    out = np.empty((n, R), np.uint32)
    rc = lib().orc_nssg_prune(_p(base), n, d, _p(knn), knn.shape[1], l, R, cos2(alpha),
                              {"literal": 0, "hop1first": 1}[expand], _p(out))
    if rc:
        raise ValueError(f"orc_nssg_prune rc={rc}")
    return out


def nssg_reverse(base, G1, alpha: float = 60.0):
    """Second loop of Alg. 3 (reverse-neighbour checking)."""
    base = _f32(base)
    G1 = np.ascontiguousarray(G1, dtype=np.uint32)
    n, d = base.shape
    R = G1.shape[1]
    out = np.empty_like(G1)
    rc = lib().orc_nssg_reverse(_p(base), n, d, _p(G1), R, cos2(alpha), _p(out))
    if rc:
        raise ValueError(f"orc_nssg_reverse rc={rc}")
    return out


def dfs_connect(base, graph, roots, l: int):
    """Last loop of Alg. 3: DFS spanning from each navigating node. Modifies
    a copy of ``graph``; returns (graph, added_edges[k, 2])."""
    base = _f32(base)
    g = np.ascontiguousarray(graph, dtype=np.uint32).copy()
    roots = np.ascontiguousarray(roots, dtype=np.uint32)
    n, d = base.shape
    cap = 2 * n + 16
    added = np.empty((cap, 2), np.uint32)
    k = lib().orc_dfs_connect(_p(base), n, d, _p(g), g.shape[1], _p(roots), len(roots), l,
                              _p(added), cap)
    if k < 0:
        raise ValueError(f"orc_dfs_connect rc={k}")
    return g, added[:k].copy()


def nssg_build(base, knn, l: int, R: int, alpha: float, entry_ids, expand: str = "literal"):
    """Alg. 3 end to end. Returns dict(graph, entry_ids, dfs_edges, g1)."""
    g1 = nssg_prune(base, knn, l, R, alpha, expand)
    g2 = nssg_reverse(base, g1, alpha)
    g3, added = dfs_connect(base, g2, entry_ids, l)
    return dict(graph=g3, entry_ids=np.asarray(entry_ids, np.uint32), dfs_edges=added, g1=g1)


# ------------------------------------------------------------------ Alg. 1
def threads(n: int = 0) -> int:
    """Set the oracle's thread count (n >= 1) and return the count in use."""
    return int(lib().orc_threads(int(n)))


def search(base, graph, entry_ids, Q, K: int, L: int, metric: str = "l2", forget: bool = False,
           seed_all: bool = False, L_arr=None, K_arr=None, trace: int = 0):
    """Alg. 1 (Search-on-Graph) from the navigating node nearest each query.

    Returns (ids[nq, K] uint32, dists[nq, K] float64, ndc[nq], hops[nq]);
    rows hold the first min(K, |S|) pool entries, padded with 0xFFFFFFFF and
    +inf. With per-query ``L_arr``/``K_arr`` the output stride is K = max.
    trace > 0 appends trace[nq, trace] uint32: the ids of the first `trace`
    expanded nodes of each query in expansion order, padded with 0xFFFFFFFF.
    """
    base, Q = _f32(base), _f32(Q)
    graph = np.ascontiguousarray(graph, dtype=np.uint32)
    entry = np.ascontiguousarray(entry_ids, dtype=np.uint32)
    n, d = base.shape
    nq = Q.shape[0]
    La = None if L_arr is None else np.ascontiguousarray(L_arr, dtype=np.int32)
    Ka = None if K_arr is None else np.ascontiguousarray(K_arr, dtype=np.int32)
    ids = np.empty((nq, K), np.uint32)
    dd = np.empty((nq, K), np.float64)
    ndc = np.empty(nq, np.int64)
    hops = np.empty(nq, np.int64)
    flags = (1 if forget else 0) | (2 if seed_all else 0)
    tr = np.empty((nq, trace), np.uint32) if trace > 0 else None
    rc = lib().orc_search(_p(base), n, d, _p(graph), graph.shape[1], _p(entry), len(entry), _p(Q),
                          nq, K, L, _p(La), _p(Ka), METRICS[metric], flags, _p(ids), _p(dd),
                          _p(ndc), _p(hops), _p(tr), int(trace))
    if rc:
        raise ValueError(f"orc_search rc={rc}")
    if tr is not None:
        return ids, dd, ndc, hops, tr
    return ids, dd, ndc, hops


def pair_keys(base, Q, ids, metric: str = "l2"):
    """Exact FP64 keys of the given (query, id) pairs (+inf for padding)."""
    base, Q = _f32(base), _f32(Q)
    ids = np.ascontiguousarray(ids, dtype=np.uint32)
    n, d = base.shape
    out = np.empty(ids.shape, np.float64)
    rc = lib().orc_pair_keys(_p(base), n, d, _p(Q), ids.shape[0], _p(ids), ids.shape[1],
                             METRICS[metric], _p(out))
    if rc:
        raise ValueError(f"orc_pair_keys rc={rc}")
    return out


# ------------------------------------------------------------------ Alg. 2
def ssg_exact(base, alpha: float = 60.0, cap: int | None = None):
    """Exact SSG (Alg. 2) over all pairs; returns (adjacency[n, cap], degree)."""
    base = _f32(base)
    n, d = base.shape
    cap = cap or (n - 1)
    out = np.empty((n, cap), np.uint32)
    deg = np.empty(n, np.int32)
    rc = lib().orc_ssg_exact(_p(base), n, d, cos2(alpha), cap, _p(out), _p(deg))
    if rc:
        raise ValueError(f"orc_ssg_exact rc={rc}")
    return out, deg


def recall_at(ids, gt_ids, k: int) -> float:
    """precision(R) = |R and G| / |G| (Eq. 1) averaged over queries, with R
    the first k returned ids and G the first k ground-truth ids."""
    ids = np.asarray(ids)[:, :k]
    gt = np.asarray(gt_ids)[:, :k]
    hit = 0
    for a, b in zip(ids, gt):
        hit += len(set(a.tolist()) & set(b.tolist()) - {SENT})
    return hit / float(gt.shape[0] * k)
