"""Write the compact copies of a workload cache that GPU runs load.

    python -m oracle.pack_cache c2 c5 ...

For each cache: row lengths as uint8 (graph_deg), the neighbour ids packed
at ceil(log2 n) bits each (graph_bits; meta["graph_bits"]), and the first 10
ground-truth columns (gt10_ids). Every packed array is unpacked again and
compared with the original before it is kept. Only files the oracle wrote
are read; nothing here computes a result.
"""

from __future__ import annotations

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

from oracle import cache  # noqa: E402


def pack(name: str) -> None:
    d = cache.path(name)
    meta = cache.load_meta(name)
    off = np.load(os.path.join(d, "graph_off.npy"), allow_pickle=False)
    ids = np.load(os.path.join(d, "graph_ids.npy"), allow_pickle=False)
    deg = np.diff(off)
    if deg.max() > 255:
        raise SystemExit(f"{name}: a row is longer than 255")
    bits = max(1, int(meta["n"] - 1).bit_length())
    words = cache.pack_ids(ids, bits)
    if not np.array_equal(cache.unpack_ids(words, bits, len(ids)), ids):
        raise SystemExit(f"{name}: packed ids do not round-trip")
    np.save(os.path.join(d, "graph_deg.npy"), deg.astype(np.uint8))
    np.save(os.path.join(d, "graph_bits.npy"), words)
    if os.path.exists(os.path.join(d, "gt_ids.npy")):
        gt = np.load(os.path.join(d, "gt_ids.npy"), allow_pickle=False)
        np.save(os.path.join(d, "gt10_ids.npy"), np.ascontiguousarray(gt[:, :10]))
    cache.save(name, {}, {"graph_bits": bits})
    print(f"{name}: {len(ids)} ids at {bits} bits: {words.nbytes / 2**20:.1f} MiB "
          f"(from {ids.nbytes / 2**20:.1f}); degrees {deg.nbytes / 8 / 2**20:.1f} MiB", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        pack(nm)
