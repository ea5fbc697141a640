"""Loader of NSSG graph caches into HBM.

A cache directory holds the graph in compressed rows (``graph_off.npy``, int64
[n+1], and ``graph_ids.npy``, uint32: row i is ids[off[i]:off[i+1]]), which the
loader expands into the fixed-width n x R matrix the kernels read (ids, then
0xFFFFFFFF padding: the n x m layout of Sec. 6.2),
``entry_ids.npy`` (uint32 [s], the navigating nodes) and ``meta.json`` (build
parameters and checksums). Arrays are read with numpy's pickle-free loader.
"""

from __future__ import annotations

import hashlib
import json
import os

import numpy as np


def default_root() -> str:
    return os.environ.get("SSG_DATA", os.path.join(os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))), "data"))


def _digest(a: np.ndarray) -> str:
    h = hashlib.sha1()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(np.ascontiguousarray(a).view(np.uint8).reshape(-1).data)
    return h.hexdigest()[:16]


def load(name: str, root: str | None = None, verify: bool = True) -> dict:
    """Read a cache: returns dict(graph, entry_ids, meta) as numpy arrays."""
    d = os.path.join(root or default_root(), name)
    if not os.path.isdir(d):
        raise FileNotFoundError(f"graph cache {d} not found (built by the oracle's cache script)")
    with open(os.path.join(d, "meta.json")) as f:
        meta = json.load(f)
    off = np.load(os.path.join(d, "graph_off.npy"), allow_pickle=False)
    ids = np.load(os.path.join(d, "graph_ids.npy"), allow_pickle=False)
    R = int(meta["R"])
    n = len(off) - 1
    graph = np.full((n, R), 0xFFFFFFFF, np.uint32)
    for_row = np.repeat(np.arange(n), np.diff(off))
    slot = np.arange(len(ids)) - off[for_row]
    if len(ids) and (slot.max() >= R or ids.max() >= n):
        raise ValueError(f"corrupt graph rows in {d}")
    graph[for_row, slot] = ids
    entry = np.load(os.path.join(d, "entry_ids.npy"), allow_pickle=False)
    if graph.dtype != np.uint32 or graph.ndim != 2:
        raise ValueError("graph must be a 2-D uint32 array")
    if verify and "graph_sha" in meta and _digest(graph) != meta["graph_sha"]:
        raise ValueError(f"graph checksum mismatch in {d}")
    return dict(graph=graph, entry_ids=entry.astype(np.uint32), meta=meta)


def to_device(arr: np.ndarray, device="cuda"):
    """Move a numpy array into HBM as a torch tensor (uint32 -> int32 bits)."""
    import torch
    if arr.dtype == np.uint32:
        arr = arr.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)
