"""Loader of NSSG graph caches into HBM.

A cache directory holds the graph in compressed rows, which the loader
expands into the fixed-width n x R matrix the kernels read (ids, then
0xFFFFFFFF padding: the n x m layout of Sec. 6.2). Row lengths are
``graph_off.npy`` (int64 [n+1], row i is ids[off[i]:off[i+1]]) or
``graph_deg.npy`` (uint8 [n]); the ids are ``graph_ids.npy`` (uint32) or
``graph_bits.npy``: each id in ``meta["graph_bits"]`` bits, 64 ids to a block
of that many uint64 words, id j of a block at bit j * bits of the block read
as one little-endian bit string. Search-only caches may instead hold rows
sorted by id in Elias-Fano form (``graph_efl.npy``: low parts packed like
graph_bits at l bits; ``graph_efh.npy``: bytes of one bit stream, least
significant bit first, where row r owns deg_r + H bits and its i-th id sets
bit (id >> l) + i of them; meta["graph_ef"] = dict(l, H, sorted_sha)): the
search gives the same results for any order of a row.
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


def unpack_bits(words: np.ndarray, bits: int, count: int, chunk: int = 1 << 20) -> np.ndarray:
    """The first ``count`` ids of a ``graph_bits`` stream, as uint32."""
    if not 1 <= bits <= 25:
        raise ValueError("ids must take 1..25 bits")
    raw = np.ascontiguousarray(words, dtype="<u8").view(np.uint8)
    blk = bits * 8  # bytes per block of 64 ids
    if raw.size % blk or count > raw.size // blk * 64:
        raise ValueError("graph_bits stream does not hold the ids")
    raw = np.concatenate([raw, np.zeros(4, np.uint8)])  # a value may end in the last byte
    bitpos = np.arange(64, dtype=np.int64) * bits
    out = np.empty(count, np.uint32)
    mask = np.uint32((1 << bits) - 1)
    for v0 in range(0, count, chunk * 64):
        v1 = min(count, v0 + chunk * 64)
        v = np.arange(v0, v1, dtype=np.int64)
        pos = (v >> 6) * blk * 8 + bitpos[v & 63]  # bit offset in the stream
        at = pos >> 3
        word = (raw[at].astype(np.uint32) | raw[at + 1].astype(np.uint32) << np.uint32(8)
                | raw[at + 2].astype(np.uint32) << np.uint32(16)
                | raw[at + 3].astype(np.uint32) << np.uint32(24))
        out[v0:v1] = (word >> (pos & 7).astype(np.uint32)) & mask
    return out


def decode_ef_rows(low: np.ndarray, high: np.ndarray, l: int, H: int, deg: np.ndarray) -> np.ndarray:
    """Ids of Elias-Fano rows (row order, ascending within a row) as uint32."""
    deg = np.asarray(deg, dtype=np.int64)
    total = int(deg.sum())
    width = deg + H
    ends = np.cumsum(width)
    ones = np.flatnonzero(np.unpackbits(np.asarray(high, np.uint8), bitorder="little"))
    ones = ones[ones < (ends[-1] if len(ends) else 0)]
    if len(ones) != total:
        raise ValueError("Elias-Fano stream does not match the row lengths")
    row = np.searchsorted(ends, ones, side="right")  # the field each set bit falls in
    first = np.concatenate([[0], np.cumsum(deg)[:-1]])  # index of each row's first id
    rank = np.arange(total, dtype=np.int64) - first[row]
    hi = ones - (ends[row] - width[row]) - rank
    lo = unpack_bits(low, l, total).astype(np.int64) if l > 0 else np.zeros(total, np.int64)
    return ((hi << l) | lo).astype(np.uint32)


def load(name: str, root: str | None = None, verify: bool = True) -> dict:
    """Read a cache: returns dict(graph, entry_ids, meta) as numpy arrays."""
    d = os.path.join(root or default_root(), name)
    if not os.path.isdir(d):
        raise FileNotFoundError(f"graph cache {d} not found (built by the oracle's cache script)")
    with open(os.path.join(d, "meta.json")) as f:
        meta = json.load(f)
    if os.path.exists(os.path.join(d, "graph_off.npy")):
        off = np.load(os.path.join(d, "graph_off.npy"), allow_pickle=False)
    else:
        deg = np.load(os.path.join(d, "graph_deg.npy"), allow_pickle=False)
        off = np.concatenate([[0], np.cumsum(deg, dtype=np.int64)])
    sha = meta.get("graph_sha")
    if os.path.exists(os.path.join(d, "graph_ids.npy")):
        ids = np.load(os.path.join(d, "graph_ids.npy"), allow_pickle=False)
    elif os.path.exists(os.path.join(d, "graph_bits.npy")):
        ids = unpack_bits(np.load(os.path.join(d, "graph_bits.npy"), allow_pickle=False),
                          int(meta["graph_bits"]), int(off[-1]))
    else:
        ef = meta["graph_ef"]
        ids = decode_ef_rows(np.load(os.path.join(d, "graph_efl.npy"), allow_pickle=False),
                             np.load(os.path.join(d, "graph_efh.npy"), allow_pickle=False),
                             int(ef["l"]), int(ef["H"]), np.diff(off))
        sha = ef["sorted_sha"]
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
    if verify and sha is not None and _digest(graph) != sha:
        raise ValueError(f"graph checksum mismatch in {d}")
    return dict(graph=graph, entry_ids=entry.astype(np.uint32), meta=meta)


def to_device(arr: np.ndarray, device="cuda"):
    """Move a numpy array into HBM as a torch tensor (uint32 -> int32 bits)."""
    import torch
    if arr.dtype == np.uint32:
        arr = arr.view(np.int32)
    return torch.from_numpy(np.ascontiguousarray(arr)).to(device)
