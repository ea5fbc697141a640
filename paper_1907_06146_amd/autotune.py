"""Launch-shape autotuner for the batched search.

For every L bucket it times candidate shapes -- gather variant (lanes per
candidate and loads in flight), visited-set size, wavefronts per workgroup
-- on a sample of that bucket's queries and keeps the fastest. Results are
cached in a JSON file keyed by device, storage type, dimension, metric, row
width, bucket capacity and rerank mode.
"""

from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import _lib
from .batched import BUCKET_BOUNDS, BatchedSearch


def candidate_shapes(dtype: torch.dtype, d: int, cap: int = 512):
    """Launch shapes worth timing for a storage type and dimension: gather
    variants x visited-cache size (default 4,096 entries, or 2,048, which
    lets low-register shapes hold more wavefronts) x wavefronts per
    workgroup, and two queries per wavefront where a grouped kernel exists
    (d = 96 or 128, pool capacity <= 256)."""
    variants = (0,)
    if d == 128 and dtype == torch.float32:
        variants = (0, 1, 2, 3)
    elif d == 128 and dtype == torch.bfloat16:
        variants = (0, 2, 7, 8)
    elif d == 128 and dtype == torch.uint8:
        variants = (0, 3)
    elif d == 96 and dtype == torch.bfloat16:
        variants = (0, 4)
    out = [dict(gather_variant=v, hash_log2=h, waves_per_block=w, queries_per_wave=1)
           for v in variants for h in (0, 11) for w in (1, 2)]
    if d in (96, 128) and cap <= 256:
        out += [dict(gather_variant=0, hash_log2=0, waves_per_block=w, queries_per_wave=2) for w in (1, 2)]
    return out


def _key(base, metric, R, cap, rerank):
    dev = torch.cuda.get_device_name(base.device)
    return f"{dev}|{base.dtype}|d{base.shape[1]}|{metric}|R{R}|cap{cap}|rerank{rerank}"


def tune(base, graph, entry_ids, queries, L, K, metric="l2", dim_scale=None, base_f32=None,
         rerank=0, sample=4096, reps=3, cache_path=None, seed=0, log=None):
    """Returns {bucket capacity: shape dict} for this workload."""
    L_host = L.cpu().numpy() if isinstance(L, torch.Tensor) else np.asarray(L)
    K_host = K.cpu().numpy() if isinstance(K, torch.Tensor) else np.asarray(K)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    shapes = {}
    rng = np.random.default_rng(seed)
    lo = 0
    for cap in BUCKET_BOUNDS:
        sel = np.nonzero((L_host > lo) & (L_host <= cap))[0]
        lo = cap
        if len(sel) == 0:
            continue
        key = _key(base, metric, graph.shape[1], cap, rerank)
        if key in cache:
            shapes[cap] = cache[key]["shape"]
            continue
        sub = np.sort(rng.choice(sel, size=min(sample, len(sel)), replace=False))
        q = queries[torch.from_numpy(sub).to(queries.device)].contiguous()
        best = None
        for sh in candidate_shapes(base.dtype, base.shape[1], cap):
            try:
                bs = BatchedSearch(base, graph, entry_ids, q, L_host[sub], K_host[sub], metric,
                                   dim_scale, base_f32, rerank, shapes={cap: sh}, use_graph=False)
                bs.run()
            except _lib.SSGError:  # a shape this bucket cannot run
                continue
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                bs.run()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            if log:
                log(f"autotune cap={cap} {sh}: {ms:.3f} ms for {len(sub)} queries")
            if best is None or ms < best[0]:
                best = (ms, sh)
        shapes[cap] = best[1]
        cache[key] = {"shape": best[1], "ms": best[0], "queries": int(len(sub))}
    if cache_path:
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    return shapes


def tune_search(base, graph, entry_ids, queries, K: int, L: int, metric="l2", dim_scale=None,
                base_f32=None, rerank_k: int = 0, reps: int = 3, log=None):
    """Fastest launch shape of the plain search for these queries: every
    candidate shape is timed on them (HIP events on the current stream) and
    (shape, ms per launch, all timings) is returned. The shape dict holds
    ``search`` keyword arguments. Every shape gives the same results."""
    from .binding import search
    st = torch.cuda.current_stream(queries.device)
    rows = []
    for sh in candidate_shapes(base.dtype, base.shape[1], 64 * -(-L // 64)):
        kw = dict(sh, dim_scale=dim_scale, base_f32=base_f32, rerank_k=rerank_k)
        try:
            search(base, graph, entry_ids, queries, K, L, metric, **kw)
        except _lib.SSGError:
            continue
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        for _ in range(reps):
            search(base, graph, entry_ids, queries, K, L, metric, **kw)
        e1.record(st)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        rows.append((ms, sh))
        if log:
            log(f"tune_search {sh}: {ms:.4f} ms for {queries.shape[0]} queries")
    best = min(rows, key=lambda r: r[0])
    return best[1], best[0], rows
