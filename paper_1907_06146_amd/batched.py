"""Mixed-workload batched search: per-query pool size L_i and result count
K_i in one launch (a captured HIP graph of persistent bucket kernels).

Queries are grouped into buckets by L (pool capacities 64, 128, 256, 512);
inside a bucket the longest searches are queued first so the persistent
wavefronts finish together. Each bucket's launch shape comes from the
autotuner (``autotune.py``) or the library defaults.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .binding import _DTYPES, _METRICS, _VISITED, _need_cuda

BUCKET_BOUNDS = (64, 128, 256, 512)


def plan_buckets(L_host: np.ndarray, bounds=BUCKET_BOUNDS):
    """Split query indices by pool size: returns [(max_L, qidx int32)], qidx
    ordered by decreasing L (ties by index)."""
    L_host = np.asarray(L_host, np.int64)
    out = []
    lo = 0
    for hi in bounds:
        sel = np.nonzero((L_host > lo) & (L_host <= hi))[0]
        lo = hi
        if len(sel) == 0:
            continue
        order = sel[np.lexsort((sel, -L_host[sel]))]
        out.append((int(L_host[sel].max()), order.astype(np.int32)))
    if (L_host > bounds[-1]).any() or (L_host < 1).any():
        raise ValueError(f"every L must be in [1, {bounds[-1]}]")
    return out


class BatchedSearch:
    """Holds device buffers and (optionally) the captured graph for one
    mixed batch; ``run()`` enqueues it on the current stream.

    base / base_f32 / dim_scale as in ``search``; L, K: int32 [nq] (host or
    device); rerank: 0 none, -m the first m * K_i entries (1 <= m <= 16),
    > 0 a fixed count (at least K_i).
    no_alloc: run through ssg_search_batched_noalloc (the work-queue counters
    in the library's per-device array; calls on one device must not overlap).
    shapes: {max_L bucket capacity: dict(gather_variant, hash_log2,
    waves_per_block, blocks, visited, queries_per_wave)} from the autotuner
    (visited: "auto", "hash" or "cache", the form of the LDS visited set;
    queries_per_wave: searches per wavefront, 0 = the library's choice).
    """

    def __init__(self, base, graph, entry_ids, queries, L, K, metric="l2", dim_scale=None,
                 base_f32=None, rerank=0, shapes=None, kstride=None, stats=False, use_graph=True,
                 bounds=BUCKET_BOUNDS, trace=0, no_alloc=False):
        _need_cuda("base", base, tuple(_DTYPES))
        _need_cuda("graph", graph, (torch.int32, torch.uint32))
        _need_cuda("entry_ids", entry_ids, (torch.int32, torch.uint32))
        _need_cuda("queries", queries, (torch.float32,))
        dev = base.device
        L_host = L.cpu().numpy() if isinstance(L, torch.Tensor) else np.asarray(L)
        K_host = K.cpu().numpy() if isinstance(K, torch.Tensor) else np.asarray(K)
        self.nq = queries.shape[0]
        self.kstride = int(kstride or K_host.max())
        self.L = torch.as_tensor(L_host, dtype=torch.int32).to(dev)
        self.K = torch.as_tensor(K_host, dtype=torch.int32).to(dev)
        self.plan = plan_buckets(L_host, bounds)
        self.qlists = [torch.from_numpy(q).to(dev) for _, q in self.plan]
        self.out_ids = torch.empty((self.nq, self.kstride), dtype=torch.int32, device=dev)
        self.out_d = torch.empty((self.nq, self.kstride), dtype=torch.float32, device=dev)
        self.ndc = torch.empty(self.nq, dtype=torch.int32, device=dev) if stats else None
        self.hops = torch.empty(self.nq, dtype=torch.int32, device=dev) if stats else None
        self.trace = torch.empty((self.nq, trace), dtype=torch.int32, device=dev) if trace > 0 else None
        nb = len(self.plan)
        if no_alloc:  # the counters live in the library's own array
            self.ws, wsp, self._ws = None, 0, (0, 0)
        else:
            self.ws = torch.empty(_lib.lib().ssg_batch_workspace_bytes(nb) + 256, dtype=torch.uint8,
                                  device=dev)
            wsp = (self.ws.data_ptr() + 255) & ~255
            self._ws = (wsp, _lib.lib().ssg_batch_workspace_bytes(nb))
        self._keep = (base, graph, entry_ids, queries, dim_scale, base_f32)
        dtype = _DTYPES[base.dtype]
        self.desc = _lib.BatchDesc(
            base.data_ptr(), base.shape[0], base.shape[1], dtype, _METRICS[metric],
            None if dim_scale is None else dim_scale.data_ptr(),
            None if base_f32 is None else base_f32.data_ptr(), rerank, graph.data_ptr(),
            graph.shape[1], entry_ids.data_ptr(), entry_ids.numel(), queries.data_ptr(), self.nq,
            self.L.data_ptr(), self.K.data_ptr(), self.kstride, self.out_ids.data_ptr(),
            self.out_d.data_ptr(), None if self.ndc is None else self.ndc.data_ptr(),
            None if self.hops is None else self.hops.data_ptr(),
            None if self.trace is None else self.trace.data_ptr(), max(0, int(trace)))
        shapes = shapes or {}
        arr = (_lib.Bucket * nb)()
        for i, ((mL, q), ql) in enumerate(zip(self.plan, self.qlists)):
            cap = next(b for b in bounds if mL <= b)
            sh = shapes.get(cap, {})
            arr[i] = _lib.Bucket(ql.data_ptr(), len(q), mL, sh.get("gather_variant", 0),
                                 sh.get("hash_log2", 0), sh.get("waves_per_block", 0),
                                 sh.get("blocks", 0), _VISITED[sh.get("visited", "auto")],
                                 sh.get("queries_per_wave", 0))
        self.buckets = arr
        self.graph = None
        self.no_alloc = no_alloc
        if use_graph and not no_alloc:
            g = ctypes.c_void_p()
            _lib.check(_lib.lib().ssg_batch_graph_create(ctypes.byref(g), ctypes.byref(self.desc),
                                                         self.buckets, nb, ctypes.c_void_p(wsp),
                                                         self._ws[1]))
            self.graph = g

    def run(self, stream=None):
        st = stream if stream is not None else torch.cuda.current_stream()
        if self.no_alloc:  # counters in the library's own array: nothing allocated per call
            rc = _lib.lib().ssg_search_batched_noalloc(ctypes.byref(self.desc), self.buckets,
                                                       len(self.plan), ctypes.c_void_p(st.cuda_stream))
        elif self.graph is not None:
            rc = _lib.lib().ssg_batch_graph_launch(self.graph, ctypes.c_void_p(st.cuda_stream))
        else:
            rc = _lib.lib().ssg_search_batched(ctypes.byref(self.desc), self.buckets,
                                               len(self.plan), ctypes.c_void_p(self._ws[0]),
                                               self._ws[1], ctypes.c_void_p(st.cuda_stream))
        _lib.check(rc)
        return self.out_ids, self.out_d

    def close(self):
        if self.graph is not None:
            torch.cuda.synchronize()  # no replay may still be running
            _lib.lib().ssg_batch_graph_destroy(self.graph)
            self.graph = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
