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
