"""Writer and reader of the graph cache directories (test infrastructure).

A cache directory ``data/<workload>/`` holds plain ``.npy`` arrays and a
``meta.json`` with the build parameters, the readings used and checksums:

  graph_off.npy  int64 [n+1]   NSSG rows in compressed form: row i is
  graph_ids.npy  uint32 [nnz]   graph_ids[graph_off[i]:graph_off[i+1]]; the
                                fixed-width [n, R] matrix (ids, then
                                0xFFFFFFFF) is rebuilt on load, R = meta["R"]
  entry_ids.npy  uint32 [s]     navigating nodes
  dfs_edges.npy  uint32 [k, 2]  edges added by DFS spanning (w, u)
  gt_ids.npy     uint32 [nq, Kg] exact ground truth, (dist, id) order
  gt_d.npy       float64 [nq, Kg]
  oracle_L<L>_{ids,d,ndc,hops}.npy  Alg. 1 results of the oracle at pool L
  sweep.json     per-L recall / NDC / hops / CPU time of the oracle

Compact copies for shipping (written by ``oracle/pack_cache.py``; the loader
uses them when the plain files are absent):
  graph_deg.npy   uint8 [n]        row lengths (replaces graph_off)
  graph_bits.npy  uint64 [words]   graph_ids at meta["graph_bits"] bits per
                                   id, 64 ids per block of graph_bits words
  gt10_ids.npy    uint32 [nq, 10]  the first 10 columns of gt_ids

The base vectors and queries are not stored: they are regenerated from the
seed by ``synth`` and checked against the recorded checksums.
"""

from __future__ import annotations

import json
import os

import numpy as np

FORMAT_VERSION = 1


def data_root() -> str:
    return os.environ.get("SSG_DATA", os.path.join(os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))), "data"))


def path(name: str) -> str:
    return os.path.join(data_root(), name)


SENT = 0xFFFFFFFF


def _to_csr(g: np.ndarray):
    valid = g != SENT
    off = np.zeros(g.shape[0] + 1, np.int64)
    np.cumsum(valid.sum(1), out=off[1:])
    return off, g[valid].astype(np.uint32)


def _from_csr(off: np.ndarray, ids: np.ndarray, R: int) -> np.ndarray:
    n = len(off) - 1
    deg = np.diff(off)
    g = np.full((n, R), SENT, np.uint32)
    col = np.arange(len(ids)) - np.repeat(off[:-1], deg)
    g[np.repeat(np.arange(n), deg), col] = ids
    return g


def save(name: str, arrays: dict, meta: dict) -> str:
    d = path(name)
    os.makedirs(d, exist_ok=True)
    for k, v in arrays.items():
        if k == "graph":
            off, ids = _to_csr(v)
            np.save(os.path.join(d, "graph_off.npy"), off)
            np.save(os.path.join(d, "graph_ids.npy"), ids)
            continue
        np.save(os.path.join(d, k + ".npy"), v)
    m = dict(meta)
    m["format_version"] = FORMAT_VERSION
    old = load_meta(name) or {}
    old.update(m)
    with open(os.path.join(d, "meta.json"), "w") as f:
        json.dump(old, f, indent=1, sort_keys=True)
    return d


def load_meta(name: str):
    p = os.path.join(path(name), "meta.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        return json.load(f)


def pack_ids(ids: np.ndarray, bits: int) -> np.ndarray:
    """Pack uint32 values below 2^bits into a uint64 stream, 64 values per
    block of ``bits`` words (value j of a block at bit offset j * bits)."""
    ids = np.ascontiguousarray(ids, dtype=np.uint64)
    nb = -(-len(ids) // 64)
    v = np.zeros((nb, 64), np.uint64)
    v.reshape(-1)[:len(ids)] = ids
    w = np.zeros((nb, bits + 1), np.uint64)
    for j in range(64):
        off = j * bits
        k, sh = off // 64, off % 64
        w[:, k] |= v[:, j] << np.uint64(sh)
        if sh + bits > 64:
            w[:, k + 1] |= v[:, j] >> np.uint64(64 - sh)
    return np.ascontiguousarray(w[:, :bits]).reshape(-1)


def unpack_ids(words: np.ndarray, bits: int, count: int) -> np.ndarray:
    """Inverse of ``pack_ids``: the first ``count`` values as uint32."""
    w = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1, bits)
    w = np.concatenate([w, np.zeros((len(w), 1), np.uint64)], axis=1)
    mask = np.uint64((1 << bits) - 1)
    out = np.empty((len(w), 64), np.uint64)
    for j in range(64):
        off = j * bits
        k, sh = off // 64, off % 64
        x = w[:, k] >> np.uint64(sh)
        if sh + bits > 64:
            x |= w[:, k + 1] << np.uint64(64 - sh)
        out[:, j] = x & mask
    return out.reshape(-1)[:count].astype(np.uint32)


def ef_decode(low: np.ndarray, high: np.ndarray, l: int, H: int, deg: np.ndarray, n: int) -> np.ndarray:
    """Ids of Elias-Fano coded rows (see oracle.pack_cache.ef_encode), in row
    order, each row ascending."""
    deg = np.asarray(deg, np.int64)
    nnz = int(deg.sum())
    field = np.zeros(len(deg) + 1, np.int64)
    np.cumsum(deg + H, out=field[1:])
    pos = np.flatnonzero(np.unpackbits(high, bitorder="little")[:field[-1]])
    if len(pos) != nnz:
        raise ValueError("Elias-Fano high bits do not match the row lengths")
    row = np.repeat(np.arange(len(deg)), deg)
    start = np.zeros(len(deg) + 1, np.int64)
    np.cumsum(deg, out=start[1:])
    hi = pos - field[row] - (np.arange(nnz) - start[row])
    lo = unpack_ids(low, max(l, 1), nnz).astype(np.int64) if l else 0
    out = (hi << l) | lo
    if nnz and (out.max() >= n or hi.min() < 0):
        raise ValueError("Elias-Fano rows out of range")
    return out.astype(np.uint32)


def load(name: str, key: str, mmap: bool = False):
    if key == "graph":
        d = path(name)
        R = load_meta(name)["R"]
        ef = load_meta(name).get("graph_ef")
        if ef and not os.path.exists(os.path.join(d, "graph_ids.npy")) and \
                not os.path.exists(os.path.join(d, "graph_bits.npy")):
            deg = np.load(os.path.join(d, "graph_deg.npy"), allow_pickle=False)
            off = np.zeros(len(deg) + 1, np.int64)
            np.cumsum(deg, out=off[1:])
            ids = ef_decode(np.load(os.path.join(d, "graph_efl.npy"), allow_pickle=False),
                            np.load(os.path.join(d, "graph_efh.npy"), allow_pickle=False),
                            ef["l"], ef["H"], deg, load_meta(name)["n"])
            return _from_csr(off, ids, R)
        if os.path.exists(os.path.join(d, "graph_off.npy")):
            off = np.load(os.path.join(d, "graph_off.npy"), allow_pickle=False)
        else:
            deg = np.load(os.path.join(d, "graph_deg.npy"), allow_pickle=False)
            off = np.zeros(len(deg) + 1, np.int64)
            np.cumsum(deg, out=off[1:])
        if os.path.exists(os.path.join(d, "graph_ids.npy")):
            ids = np.load(os.path.join(d, "graph_ids.npy"), allow_pickle=False)
        else:
            words = np.load(os.path.join(d, "graph_bits.npy"), allow_pickle=False)
            ids = unpack_ids(words, load_meta(name)["graph_bits"], int(off[-1]))
        return _from_csr(off, ids, R)
    rg = (load_meta(name) or {}).get("ragged", {}).get(key)
    if rg and not os.path.exists(os.path.join(path(name), key + ".npy")):
        # first K_i ids of each row, padded with SENT to the stored width
        Kq = np.load(os.path.join(path(name), "mixed_K.npy"), allow_pickle=False).astype(np.int64)
        vals = unpack_ids(np.load(os.path.join(path(name), key + "_bits.npy"), allow_pickle=False),
                          rg["bits"], int(Kq.sum()))
        vals[vals == load_meta(name)["n"]] = SENT  # an empty slot
        out = np.full((len(Kq), rg["width"]), SENT, np.uint32)
        out[np.arange(rg["width"])[None, :] < Kq[:, None]] = vals
        return out
    if key == "gt10_ids" and not os.path.exists(os.path.join(path(name), "gt10_ids.npy")):
        return np.ascontiguousarray(load(name, "gt_ids")[:, :10])
    p = os.path.join(path(name), key + ".npy")
    return np.load(p, mmap_mode="r" if mmap else None, allow_pickle=False)


def exists(name: str, key: str) -> bool:
    if key == "graph":
        return any(os.path.exists(os.path.join(path(name), k + ".npy")) for k in ("graph_off", "graph_deg"))
    if key == "gt10_ids" and exists(name, "gt_ids"):
        return True
    if key in (load_meta(name) or {}).get("ragged", {}):
        return True
    return os.path.exists(os.path.join(path(name), key + ".npy"))
