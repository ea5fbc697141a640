"""Partitioned search on one GPU (Sec. 6.5): the data set is split at random
into S shards of (nearly) equal size, each shard gets its own graph, every
query is searched in all shards (one launch per shard, on S streams), and the
per-shard top-K lists are merged on the device by (distance, global id)
(``ssg_merge_shards``).

By default the shards are stored as one block-diagonal index (shard s's rows
at an offset, its graph's ids shifted by it) and all S x nq searches run in
one launch, each query group starting from its own shard's navigating nodes
(``entry_group_size``); a graph edge never leaves its shard, so each search
stays inside its shard. ``combined=False`` instead launches one ordinary
search per shard on S streams. Either way the shards may be stored in FP32 or
BF16 and the launch-shape options apply to every shard. Arguments that belong
to one index's vectors (an FP8 per-dimension scale, FP32 rerank vectors) are
rejected: a single value cannot describe S shards.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from .binding import _need_cuda, _ptr, search


def partition(n: int, S: int, seed: int) -> list[np.ndarray]:
    """Random split of range(n) into S shards of sizes differing by at most
    one; each shard's global ids in ascending order."""
    if S < 1 or S > n:
        raise ValueError("need 1 <= S <= n")
    perm = np.random.default_rng(seed).permutation(n)
    return [np.sort(p).astype(np.int64) for p in np.array_split(perm, S)]


class ShardedIndex:
    """S shard indexes resident on one GPU.

    bases:    list of S [n_s, d] device tensors (shard rows)
    graphs:   list of S [n_s, R] int32 device tensors (shard-local ids)
    entries:  list of S navigating-node id tensors (shard-local)
    id_maps:  list of S int arrays: local id -> global id
    """

    def __init__(self, bases, graphs, entries, id_maps, metric: str = "l2", combined: bool = True):
        if not (len(bases) == len(graphs) == len(entries) == len(id_maps)) or not bases:
            raise ValueError("one base, graph, entry set and id map per shard")
        for t in bases:
            _need_cuda("shard base", t)
        self.S = len(bases)
        self.bases, self.graphs, self.entries = bases, graphs, entries
        self.metric = metric
        self.combined = combined
        dev = bases[0].device
        sizes = [len(m) for m in id_maps]
        starts = np.concatenate([[0], np.cumsum(sizes)[:-1]]).astype(np.int64)
        self.map = torch.from_numpy(np.concatenate(id_maps).astype(np.uint32).view(np.int32)).to(dev)
        self.off = torch.tensor(starts, dtype=torch.int64, device=dev)
        if combined:
            if len({e.numel() for e in entries}) != 1:
                raise ValueError("combined mode needs the same number of navigating nodes per shard")
            self.cbase = torch.cat(list(bases), 0).contiguous()
            rows = []
            for g, o in zip(graphs, starts):
                g = g.to(torch.int32)
                rows.append(torch.where(g >= 0, g + int(o), g))
            self.cgraph = torch.cat(rows, 0).contiguous()
            self.centry = torch.stack([e.to(torch.int32).reshape(-1) + int(o)
                                       for e, o in zip(entries, starts)]).contiguous()
            self.zero_off = torch.zeros(self.S, dtype=torch.int64, device=dev)
        else:
            self.streams = [torch.cuda.Stream(device=dev) for _ in range(self.S)]  # default priority

    def search(self, queries, K: int, L: int, K_out: int | None = None, **kw):
        """Search every shard with pool size L, keep K per shard, merge to
        K_out (default K) by (distance, global id). Returns (ids, dists)."""
        K_out = K_out or K
        for k in ("dim_scale", "base_f32", "rerank_k"):
            v = kw.get(k)
            if v is not None and not (isinstance(v, int) and v == 0):
                raise ValueError(f"{k} describes one index's vectors and cannot be applied to "
                                 f"{self.S} shards")
        nq = queries.shape[0]
        dev = queries.device
        main = torch.cuda.current_stream(dev)
        if self.combined:
            tq = queries.repeat(self.S, 1).contiguous()
            ids, dd = search(self.cbase, self.cgraph, self.centry, tq, K, L, self.metric,
                             entry_group_size=nq, **kw)
            return self._merge(ids, dd, nq, K, K_out, self.map, self.zero_off, main)
        ids = torch.empty((self.S, nq, K), dtype=torch.int32, device=dev)
        dd = torch.empty((self.S, nq, K), dtype=torch.float32, device=dev)
        for s in range(self.S):
            st = self.streams[s]
            st.wait_stream(main)  # queries and outputs are ready on the caller's stream
            search(self.bases[s], self.graphs[s], self.entries[s], queries, K, L, self.metric,
                   out=(ids[s], dd[s]), stream=st, **kw)
        for st in self.streams:
            main.wait_stream(st)
        return self._merge(ids, dd, nq, K, K_out, self.map, self.off, main)

    def _merge(self, ids, dd, nq, K, K_out, idmap, off, main):
        dev = ids.device
        out_i = torch.empty((nq, K_out), dtype=torch.int32, device=dev)
        out_d = torch.empty((nq, K_out), dtype=torch.float32, device=dev)
        rc = _lib.lib().ssg_merge_shards(_ptr(ids), _ptr(dd), self.S, nq, K, _ptr(idmap),
                                         _ptr(off), idmap.numel(), K_out, _ptr(out_i), _ptr(out_d),
                                         ctypes.c_void_p(main.cuda_stream))
        _lib.check(rc)
        # the shard buffers stay alive until the merge has read them
        self._last = (ids, dd)
        return out_i, out_d
