"""Writer and reader of the graph cache directories (test infrastructure).

A cache directory ``data/<workload>/`` holds plain ``.npy`` arrays and a
``meta.json`` with the build parameters, the readings used and checksums:

  graph.npy      uint32 [n, R]  NSSG rows: neighbour ids, then 0xFFFFFFFF
  entry_ids.npy  uint32 [s]     navigating nodes
  dfs_edges.npy  uint32 [k, 2]  edges added by DFS spanning (w, u)
  gt_ids.npy     uint32 [nq, Kg] exact ground truth, (dist, id) order
  gt_d.npy       float64 [nq, Kg]
  oracle_L<L>_{ids,d,ndc,hops}.npy  Alg. 1 results of the oracle at pool L
  sweep.json     per-L recall / NDC / hops / CPU time of the oracle

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


def save(name: str, arrays: dict, meta: dict) -> str:
    d = path(name)
    os.makedirs(d, exist_ok=True)
    for k, v in arrays.items():
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


def load(name: str, key: str, mmap: bool = False):
    p = os.path.join(path(name), key + ".npy")
    return np.load(p, mmap_mode="r" if mmap else None, allow_pickle=False)


def exists(name: str, key: str) -> bool:
    return os.path.exists(os.path.join(path(name), key + ".npy"))
