"""The compact cache format (bit-packed ids, uint8 row lengths) round-trips
exactly, and a cache loads the same graph from either form."""

import os
import shutil

import numpy as np
import pytest

from oracle import cache


@pytest.mark.parametrize("bits", [1, 7, 20, 23, 31, 32])
def test_pack_round_trip(bits):
    rng = np.random.default_rng(bits)
    for n in (0, 1, 63, 64, 65, 1000):
        v = rng.integers(0, 2 ** bits, n, dtype=np.uint64).astype(np.uint32)
        w = cache.pack_ids(v, bits)
        assert w.dtype == np.uint64 and len(w) == -(-n // 64) * bits
        assert np.array_equal(cache.unpack_ids(w, bits, n), v)


def test_packed_graph_loads_identically(tmp_path, monkeypatch):
    from oracle import pack_cache
    monkeypatch.setenv("SSG_DATA", str(tmp_path))
    rng = np.random.default_rng(0)
    n, R = 700, 9
    g = np.full((n, R), cache.SENT, np.uint32)
    for i in range(n):
        k = int(rng.integers(0, R + 1))
        g[i, :k] = rng.choice(n, k, replace=False)
    cache.save("t", dict(graph=g, gt_ids=rng.integers(0, n, (5, 12)).astype(np.uint32)),
               dict(n=n, R=R))
    pack_cache.pack("t")
    d = cache.path("t")
    for f in ("graph_off", "graph_ids"):
        os.remove(os.path.join(d, f + ".npy"))
    assert np.array_equal(cache.load("t", "graph"), g)
    assert np.array_equal(cache.load("t", "gt10_ids"), cache.load("t", "gt_ids")[:, :10])
    assert cache.load_meta("t")["graph_bits"] == 10
    shutil.rmtree(d)


@pytest.mark.parametrize("bits", [1, 9, 20, 23, 25])
def test_library_loader_reads_the_packed_stream(bits):
    """The package's own reader of the packed ids (used to load graphs into
    HBM) reads what the cache writer packed, in small chunks too."""
    from paper_1907_06146_amd import graph_io
    rng = np.random.default_rng(100 + bits)
    for n in (0, 1, 63, 64, 65, 4097):
        v = rng.integers(0, 2 ** bits, n, dtype=np.uint64).astype(np.uint32)
        w = cache.pack_ids(v, bits)
        assert np.array_equal(graph_io.unpack_bits(w, bits, n), v)
        assert np.array_equal(graph_io.unpack_bits(w, bits, n, chunk=1), v)


def test_library_loader_loads_the_packed_graph(tmp_path, monkeypatch):
    from oracle import pack_cache
    from paper_1907_06146_amd import graph_io
    monkeypatch.setenv("SSG_DATA", str(tmp_path))
    rng = np.random.default_rng(1)
    n, R = 900, 11
    g = np.full((n, R), cache.SENT, np.uint32)
    for i in range(n):
        k = int(rng.integers(0, R + 1))
        g[i, :k] = rng.choice(n, k, replace=False)
    cache.save("u", dict(graph=g, entry_ids=np.arange(4, dtype=np.uint32)), dict(n=n, R=R))
    pack_cache.pack("u")
    d = cache.path("u")
    for f in ("graph_off", "graph_ids"):
        os.remove(os.path.join(d, f + ".npy"))
    out = graph_io.load("u", root=str(tmp_path), verify=False)
    assert np.array_equal(out["graph"], g)
    with pytest.raises(ValueError):
        graph_io.unpack_bits(np.zeros(3, np.uint64), 20, 10)
    shutil.rmtree(d)


def _random_csr(rng, n, R, empty_rows=True):
    deg = rng.integers(0 if empty_rows else 1, R + 1, n)
    off = np.concatenate([[0], np.cumsum(deg)]).astype(np.int64)
    ids = np.concatenate([rng.choice(n, k, replace=False) for k in deg] or [np.zeros(0)]).astype(np.uint32)
    return off, ids


@pytest.mark.parametrize("n,R", [(2, 1), (50, 7), (3000, 40), (70_000, 20)])
def test_elias_fano_rows_round_trip(n, R):
    """Rows of a CSR graph, sorted and Elias-Fano coded: the oracle's decoder
    and the package's own decoder both give the sorted rows back."""
    from oracle import pack_cache
    from paper_1907_06146_amd import graph_io
    rng = np.random.default_rng(n)
    off, ids = _random_csr(rng, n, R)
    low, high, l, H, srt = pack_cache.ef_encode(off, ids, n)
    deg = np.diff(off)
    for r in range(min(n, 200)):  # each row sorted, same set of ids
        a, b = off[r], off[r + 1]
        assert np.array_equal(srt[a:b], np.sort(ids[a:b]))
    assert np.array_equal(cache.ef_decode(low, high, l, H, deg, n), srt)
    assert np.array_equal(graph_io.decode_ef_rows(low, high, l, H, deg), srt)
    if len(ids) > 1000:  # close to log2(n / degree) + 2 bits per id
        assert 8 * (low.nbytes + high.nbytes) / len(ids) < np.log2(n / deg.mean()) + 3


def test_elias_fano_cache_loads_sorted_rows(tmp_path, monkeypatch):
    from oracle import pack_cache
    from paper_1907_06146_amd import graph_io
    monkeypatch.setenv("SSG_DATA", str(tmp_path))
    monkeypatch.setattr(pack_cache, "EF_WORKLOADS", ("v",))
    rng = np.random.default_rng(2)
    n, R = 1200, 13
    off, ids = _random_csr(rng, n, R)
    g = cache._from_csr(off, ids, R)
    cache.save("v", dict(graph=g, entry_ids=np.arange(3, dtype=np.uint32)), dict(n=n, R=R))
    pack_cache.pack("v")
    d = cache.path("v")
    for f in ("graph_off", "graph_ids", "graph_bits"):
        os.remove(os.path.join(d, f + ".npy"))
    want = np.sort(g, axis=1)  # SENT (the largest value) stays at the end of each row
    assert np.array_equal(cache.load("v", "graph"), want)
    out = graph_io.load("v", root=str(tmp_path))  # verifies the sorted-graph checksum
    assert np.array_equal(out["graph"], want)
    shutil.rmtree(d)
