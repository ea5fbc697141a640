"""PyTorch-facing wrapper of ``ssg_search`` (device memory and streams only).

``search`` takes torch tensors that already live on the GPU, passes their raw
pointers and the current HIP stream to the C ABI and returns torch tensors.
All work is done by the library's kernels, asynchronously on the stream.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib

_DTYPES = {torch.float32: _lib.SSG_F32, torch.bfloat16: _lib.SSG_BF16, torch.uint8: _lib.SSG_FP8E4M3}
_METRICS = {"l2": _lib.SSG_L2, "ip": _lib.SSG_IP}


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need_cuda(name, t, dtypes=None):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA (HIP) tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if dtypes is not None and t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")


_VISITED = {"auto": 0, "hash": 1, "cache": 2}


def search(base, graph, entry_ids, queries, K: int, L: int, metric: str = "l2",
           dim_scale=None, exact_visited: bool = False, stats: bool = False,
           waves_per_block: int = 0, hash_log2: int = 0, gather_variant: int = 0,
           base_f32=None, rerank_k: int = 0, out=None, stream=None, entry_group_size: int = 0,
           visited: str = "auto", trace: int = 0, queries_per_wave: int = 0):
    """Alg. 1 from the nearest navigating node for every row of ``queries``.

    base       [n, d] float32 | bfloat16 | uint8 (FP8 E4M3 codes, with dim_scale)
    graph      [n, R] int32 (or uint32 bits); padding -1 (= 0xFFFFFFFF)
    entry_ids  [s] int32 navigating nodes
    queries    [nq, d] float32
    Returns (ids [nq, K] int32 with -1 padding, dists [nq, K] float32) and,
    with stats=True, also (ndc [nq] int32, hops [nq] int32); with trace = T > 0
    the last element is the expansion record [nq, T] int32 (ids of the first T
    expanded nodes in expansion order, -1 after the last).
    base_f32   optional [n, d] float32: rerank the first max(rerank_k, K)
               pool entries (capped at L) exactly in FP32 before writing the K
               results.
    entry_group_size  > 0: entry_ids is [G, s] and queries g*size .. (g+1)*size-1
               start from row g (several shards stored as one block-diagonal
               graph, searched in one launch).
    visited    "auto" | "hash" | "cache": form of the LDS visited set (ignored
               with exact_visited); every form gives the same results.
    queries_per_wave  1: one search per 64-lane wavefront; 2: two searches of
               32 lanes each (L <= 256, tag-cache visited set, d = 96 or 128);
               0: the library's choice. Same results either way.
    """
    _need_cuda("base", base, tuple(_DTYPES))
    _need_cuda("graph", graph, (torch.int32, torch.uint32))
    _need_cuda("entry_ids", entry_ids, (torch.int32, torch.uint32))
    _need_cuda("queries", queries, (torch.float32,))
    if base.dim() != 2 or graph.dim() != 2 or queries.dim() != 2:
        raise ValueError("base, graph and queries must be 2-D")
    n, d = base.shape
    if graph.shape[0] != n:
        raise ValueError("graph must have one row per base vector")
    if queries.shape[1] != d:
        raise ValueError("queries and base differ in dimension")
    dtype = _DTYPES[base.dtype]
    if dtype == _lib.SSG_FP8E4M3:
        _need_cuda("dim_scale", dim_scale, (torch.float32,))
    if base_f32 is not None:
        _need_cuda("base_f32", base_f32, (torch.float32,))
        if tuple(base_f32.shape) != (n, d):
            raise ValueError("base_f32 must have the shape of base")
    nq = queries.shape[0]
    dev = base.device
    if out is None:
        ids = torch.empty((nq, K), dtype=torch.int32, device=dev)
        dd = torch.empty((nq, K), dtype=torch.float32, device=dev)
    else:
        ids, dd = out
    ndc = hops = None
    if stats:
        ndc = torch.empty(nq, dtype=torch.int32, device=dev)
        hops = torch.empty(nq, dtype=torch.int32, device=dev)
    n_entry = entry_ids.numel()
    if entry_group_size > 0:
        if entry_ids.dim() != 2 or entry_ids.shape[0] * entry_group_size < nq:
            raise ValueError("entry_group_size needs entry_ids of shape [groups, s] covering every query")
        n_entry = entry_ids.shape[1]
    if visited not in _VISITED:
        raise ValueError(f"visited must be one of {sorted(_VISITED)}, not {visited!r}")
    tr = torch.empty((nq, trace), dtype=torch.int32, device=dev) if trace > 0 else None
    opts = _lib.SearchOpts(1 if exact_visited else 0, hash_log2, waves_per_block,
                           None if ndc is None else ndc.data_ptr(),
                           None if hops is None else hops.data_ptr(), gather_variant,
                           None if base_f32 is None else base_f32.data_ptr(), rerank_k,
                           entry_group_size, _VISITED[visited],
                           None if tr is None else tr.data_ptr(), max(0, int(trace)),
                           int(queries_per_wave))
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc = _lib.lib().ssg_search_ex(
        _ptr(base), n, d, dtype, _ptr(dim_scale) if dtype == _lib.SSG_FP8E4M3 else None,
        _ptr(graph), graph.shape[1], _ptr(entry_ids), n_entry, _ptr(queries), nq, K, L,
        _METRICS[metric], _ptr(ids), _ptr(dd), ctypes.byref(opts), ctypes.c_void_p(st.cuda_stream))
    _lib.check(rc)
    res = (ids, dd, ndc, hops) if stats else (ids, dd)
    return res + (tr,) if tr is not None else res


def quantize(base_f32, dtype: str, stream=None):
    """Reduced-precision copy of FP32 base vectors, built by the library's
    kernels. dtype "bf16" -> (bfloat16 [n, d], None); "fp8" -> (uint8 E4M3
    codes [n, d], per-dimension scale float32 [d])."""
    _need_cuda("base_f32", base_f32, (torch.float32,))
    n, d = base_f32.shape
    dev = base_f32.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    if dtype == "bf16":
        out = torch.empty((n, d), dtype=torch.bfloat16, device=dev)
        rc = _lib.lib().ssg_quantize(_ptr(base_f32), n, d, _lib.SSG_BF16, None, _ptr(out),
                                     ctypes.c_void_p(st.cuda_stream))
        _lib.check(rc)
        return out, None
    if dtype == "fp8":
        out = torch.empty((n, d), dtype=torch.uint8, device=dev)
        scale = torch.empty(d, dtype=torch.float32, device=dev)
        rc = _lib.lib().ssg_quantize(_ptr(base_f32), n, d, _lib.SSG_FP8E4M3, _ptr(scale), _ptr(out),
                                     ctypes.c_void_p(st.cuda_stream))
        _lib.check(rc)
        return out, scale
    raise ValueError(f"unknown storage dtype {dtype}")


def knn_graph(base, K: int, stream=None):
    """Exact K-nearest-neighbour graph of the rows of ``base`` (float32
    [n, d] on the GPU) by brute force on the matrix cores: row i lists the K
    nearest other points in ascending (squared L2, id) order. Returns
    (ids int32 [n, K], dists float32 [n, K], stats dict). Synchronous."""
    _need_cuda("base", base, (torch.float32,))
    n, d = base.shape
    dev = base.device
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    L = _lib.lib()
    nbytes = L.ssg_knn_workspace_bytes(n, d, K)
    if nbytes == 0:
        raise ValueError(f"invalid kNN shape n={n} d={d} K={K}")
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
    off = (-ws.data_ptr()) % 256
    ids = torch.empty((n, K), dtype=torch.int32, device=dev)
    dd = torch.empty((n, K), dtype=torch.float32, device=dev)
    stats = (ctypes.c_int64 * 4)()
    rc = L.ssg_knn_graph(_ptr(base), n, d, K, _ptr(ids), _ptr(dd), ctypes.c_void_p(ws.data_ptr() + off),
                         nbytes, stats, ctypes.c_void_p(st.cuda_stream))
    _lib.check(rc)
    del ws
    return ids, dd, {"exact_path": bool(stats[0]), "rescanned_rows": int(stats[1]),
                     "candidates": int(stats[2])}


def cos2(alpha_deg: float) -> float:
    """cos^2 of the minimum edge angle; exactly 0.25 at 60 degrees."""
    import math
    return 0.25 if alpha_deg == 60.0 else math.cos(math.radians(alpha_deg)) ** 2


def nssg_prune(base, knn, l: int, R: int, alpha: float = 60.0, stream=None):
    """First loop of Alg. 3 on the GPU: candidates from the kNN graph
    (int32 [n, Kk], -1 padding) and the SSG angular rule; returns int32 [n, R]."""
    _need_cuda("base", base, (torch.float32,))
    _need_cuda("knn", knn, (torch.int32,))
    n, d = base.shape
    st = stream if stream is not None else torch.cuda.current_stream(base.device)
    out = torch.empty((n, R), dtype=torch.int32, device=base.device)
    rc = _lib.lib().ssg_nssg_prune(_ptr(base), n, d, _ptr(knn), knn.shape[1], l, R, cos2(alpha),
                                   _ptr(out), ctypes.c_void_p(st.cuda_stream))
    _lib.check(rc)
    return out


def nssg_reverse(base, g1, alpha: float = 60.0, stream=None):
    """Second loop of Alg. 3 (reverse-neighbour checking) on the GPU."""
    _need_cuda("base", base, (torch.float32,))
    _need_cuda("g1", g1, (torch.int32,))
    n, d = base.shape
    R = g1.shape[1]
    st = stream if stream is not None else torch.cuda.current_stream(base.device)
    L = _lib.lib()
    nbytes = L.ssg_nssg_reverse_workspace_bytes(n, R)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=base.device)
    off = (-ws.data_ptr()) % 256
    out = torch.empty((n, R), dtype=torch.int32, device=base.device)
    rc = L.ssg_nssg_reverse(_ptr(base), n, d, _ptr(g1), R, cos2(alpha), _ptr(out),
                            ctypes.c_void_p(ws.data_ptr() + off), nbytes, ctypes.c_void_p(st.cuda_stream))
    _lib.check(rc)
    st.synchronize()  # the workspace is released on return
    return out


def nssg_graph(base, knn_k: int, l: int, R: int, alpha: float = 60.0):
    """kNN graph, forward pruning and reverse checking of Alg. 3, all on the
    GPU. Returns (g2 int32 [n, R], kNN ids int32 [n, knn_k])."""
    ids, _, _ = knn_graph(base, knn_k)
    g1 = nssg_prune(base, ids, l, R, alpha)
    return nssg_reverse(base, g1, alpha), ids


def exact_ssg(base, alpha: float = 60.0, cap: int | None = None, stream=None):
    """Exact satellite system graph (Alg. 2) on the GPU. Returns (adjacency
    int32 [n, cap] truncated at cap (default: n - 1, the whole graph), and
    the untruncated out-degrees int32 [n]). Synchronous."""
    _need_cuda("base", base, (torch.float32,))
    n, d = base.shape
    cap = cap or (n - 1)
    st = stream if stream is not None else torch.cuda.current_stream(base.device)
    L = _lib.lib()
    nbytes = L.ssg_exact_ssg_workspace_bytes(n)
    ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=base.device)
    off = (-ws.data_ptr()) % 256
    out = torch.empty((n, cap), dtype=torch.int32, device=base.device)
    deg = torch.empty(n, dtype=torch.int32, device=base.device)
    rc = L.ssg_exact_ssg(_ptr(base), n, d, cos2(alpha), cap, _ptr(out), _ptr(deg),
                         ctypes.c_void_p(ws.data_ptr() + off), nbytes, ctypes.c_void_p(st.cuda_stream))
    _lib.check(rc)
    st.synchronize()
    return out, deg
