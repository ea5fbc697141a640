"""Write the compact copies of a workload cache that GPU runs load.

    python -m oracle.pack_cache c2 c5 ...

For each cache: row lengths as uint8 (graph_deg), the neighbour ids packed
at ceil(log2 n) bits each (graph_bits; meta["graph_bits"]), and the first 10
ground-truth columns (gt10_ids). Workloads with a per-query result count K_i
also get the first K_i ids of every row of the mixed oracle result and of the
ground truth, packed the same way at bit_length(n) bits with n standing for
an empty slot (``<key>_bits``, row lengths ``mixed_K``; meta["ragged"][key] =
dict(bits, width)). The search-only workloads (EF_WORKLOADS) also get their
rows sorted by id and Elias-Fano coded (graph_efl, graph_efh; meta["graph_ef"],
with the checksum of the row-sorted graph): Alg. 1 gives the same results for
any order of a row, and sorted rows code in about log2(n / degree) + 2 bits
per id. Every packed array is unpacked again and
compared with the original before it is kept. Only files the oracle wrote
are read; nothing here computes a result.
"""

from __future__ import annotations

import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402
from oracle import cache  # noqa: E402


# workloads whose graphs ship as Elias-Fano rows (search-only caches: Alg. 1
# does not depend on the order of a row, so its ids are stored sorted)
EF_WORKLOADS = ("c3", "c4", "c5")


def ef_encode(off: np.ndarray, ids: np.ndarray, n: int):
    """Elias-Fano code of every row of a CSR graph, the row's ids sorted.

    One low-bit width l = floor(log2(n / mean degree)) for all rows. Low
    parts (id & (2^l - 1)) in row order, packed like graph_bits at l bits.
    High parts: row r owns a field of deg_r + H bits, H = ((n - 1) >> l) + 1,
    fields back to back from bit 0; its i-th sorted id sets bit (id >> l) + i
    of the field. The bit stream is stored as bytes, least significant bit
    first. Returns (low words, high bytes, l, H)."""
    deg = np.diff(off).astype(np.int64)
    nnz = int(off[-1])
    srt = ids.copy()
    for r0 in range(0, len(deg), 1 << 16):  # sort each row
        r1 = min(len(deg), r0 + (1 << 16))
        a, b = int(off[r0]), int(off[r1])
        row = np.repeat(np.arange(r0, r1), deg[r0:r1])
        order = np.lexsort((ids[a:b], row))
        srt[a:b] = ids[a:b][order]
    mean = max(1.0, nnz / max(1, len(deg)))
    l = max(0, int(np.floor(np.log2(max(1.0, n / mean)))))
    H = ((n - 1) >> l) + 1
    low = cache.pack_ids((srt & np.uint32((1 << l) - 1)) if l else np.zeros(nnz, np.uint32), max(l, 1))
    field = np.zeros(len(deg) + 1, np.int64)
    np.cumsum(deg + H, out=field[1:])
    row = np.repeat(np.arange(len(deg)), deg)
    i = np.arange(nnz, dtype=np.int64) - off[row]
    pos = field[row] + (srt.astype(np.int64) >> l) + i
    bitsarr = np.zeros(int(field[-1]), np.uint8)
    bitsarr[pos] = 1
    high = np.packbits(bitsarr, bitorder="little")
    return low, high, l, H, srt


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
    ragged = {}
    if "K_choices" in synth.CONFIGS.get(name, {}) and os.path.exists(os.path.join(d, "oracle_mixed_ids.npy")):
        _, Kq = synth.query_params(name)
        np.save(os.path.join(d, "mixed_K.npy"), Kq.astype(np.uint8))
        mask = np.arange(int(Kq.max()))[None, :] < Kq[:, None]
        for key in ("oracle_mixed_ids", "gt_ids"):
            full = np.load(os.path.join(d, key + ".npy"), allow_pickle=False)
            vals = np.ascontiguousarray(full[:, :mask.shape[1]][mask])
            # a row may hold fewer than K_i ids (L_i < K_i): SENT is stored as n
            rb = max(1, int(meta["n"]).bit_length())
            codes = np.where(vals == cache.SENT, np.uint32(meta["n"]), vals)
            w = cache.pack_ids(codes, rb)
            if not np.array_equal(cache.unpack_ids(w, rb, len(vals)), codes):
                raise SystemExit(f"{name}: packed {key} does not round-trip")
            np.save(os.path.join(d, key + "_bits.npy"), w)
            ragged[key] = dict(bits=rb, width=int(full.shape[1]))
            print(f"{name}: {key} first K_i ids: {w.nbytes / 2**20:.1f} MiB (from {full.nbytes / 2**20:.1f})")
    extra = {}
    if name in EF_WORKLOADS:  # rows sorted by id, Elias-Fano coded
        low, high, l, H, srt = ef_encode(off, ids, int(meta["n"]))
        back = cache.ef_decode(low, high, l, H, deg, int(meta["n"]))
        if not np.array_equal(back, srt):
            raise SystemExit(f"{name}: Elias-Fano rows do not round-trip")
        np.save(os.path.join(d, "graph_efl.npy"), low)
        np.save(os.path.join(d, "graph_efh.npy"), high)
        extra["graph_ef"] = dict(l=int(l), H=int(H),
                                 sorted_sha=synth.checksum(cache._from_csr(off, srt, int(meta["R"]))))
        print(f"{name}: Elias-Fano rows {(low.nbytes + high.nbytes) / 2**20:.1f} MiB "
              f"({8 * (low.nbytes + high.nbytes) / len(ids):.2f} bits per id, l = {l})", flush=True)
    cache.save(name, {}, {"graph_bits": bits, **({"ragged": ragged} if ragged else {}), **extra})
    print(f"{name}: {len(ids)} ids at {bits} bits: {words.nbytes / 2**20:.1f} MiB "
          f"(from {ids.nbytes / 2**20:.1f}); degrees {deg.nbytes / 8 / 2**20:.1f} MiB", flush=True)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        pack(nm)
