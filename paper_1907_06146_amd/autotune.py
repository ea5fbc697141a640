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

from .batched import BUCKET_BOUNDS, BatchedSearch


def candidate_shapes(dtype: torch.dtype, d: int):
    variants = (0,)
    if d == 128 and dtype == torch.float32:
        variants = (0, 1, 2, 3)
    elif d == 128 and dtype == torch.bfloat16:
        variants = (0, 3)
    return [dict(gather_variant=v, hash_log2=h, waves_per_block=w)
            for v in variants for h in (0, 11) for w in (1, 2)]


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
        for sh in candidate_shapes(base.dtype, base.shape[1]):
            bs = BatchedSearch(base, graph, entry_ids, q, L_host[sub], K_host[sub], metric,
                               dim_scale, base_f32, rerank, shapes={cap: sh}, use_graph=False)
            bs.run()
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
