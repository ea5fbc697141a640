"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before any device work (no GPU needed)."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_1907_06146_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "ssg.h")).read()
    return sorted(set(re.findall(r"\b(ssg_[a-z_]+)\s*\(", txt)) - {"ssg_search_opts"})


def test_header_and_binding_agree():
    assert sorted(_lib.EXPORTS) == _declared()


def test_library_exports_every_symbol():
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
    assert L.ssg_version().decode().startswith("libssg")
    assert L.ssg_search_workspace_bytes(10, 10, 10, 10, 0) == 0


def _fake(n_bytes=1 << 12):
    buf = np.zeros(n_bytes, np.uint8)
    addr = buf.ctypes.data
    addr = (addr + 255) & ~255
    return buf, addr


BASE = dict(n=100, d=32, dtype=0, R=8, n_entry=2, nq=4, K=10, L=20, metric=0)


def _call(**kw):
    a = dict(BASE)
    a.update(kw)
    keep, p = _fake()
    ptr = kw.get("ptr", p)
    return _lib.lib().ssg_search(ptr, a["n"], a["d"], a["dtype"], None, ptr, a["R"], ptr,
                                 a["n_entry"], ptr, a["nq"], a["K"], a["L"], a["metric"], ptr,
                                 ptr, None, 0, None)


@pytest.mark.parametrize("kw,code", [
    (dict(K=0), _lib.SSG_EINVAL),
    (dict(L=0), _lib.SSG_EINVAL),
    (dict(d=0), _lib.SSG_EINVAL),
    (dict(R=0), _lib.SSG_EINVAL),
    (dict(n_entry=0), _lib.SSG_EINVAL),
    (dict(nq=-1), _lib.SSG_EINVAL),
    (dict(n=0), _lib.SSG_EINVAL),
    (dict(n=2 ** 31), _lib.SSG_EINVAL),
    (dict(metric=7), _lib.SSG_EINVAL),
    (dict(dtype=9), _lib.SSG_EINVAL),
    (dict(dtype=2), _lib.SSG_EINVAL),  # FP8 without a scale vector
    (dict(ptr=None), _lib.SSG_EINVAL),
    (dict(L=513), _lib.SSG_EUNSUPPORTED),
    (dict(R=65), _lib.SSG_EUNSUPPORTED),
    (dict(K=5000), _lib.SSG_EUNSUPPORTED),
    (dict(d=30), _lib.SSG_EUNSUPPORTED),
    (dict(dtype=1, d=36), _lib.SSG_EUNSUPPORTED),
])
def test_argument_errors(kw, code):
    assert _call(**kw) == code
    assert len(_lib.last_error()) > 0


def test_misaligned_base_is_rejected():
    keep, p = _fake()
    L = _lib.lib()
    rc = L.ssg_search(p + 4, 100, 32, 0, None, p, 8, p, 2, p, 4, 10, 20, 0, p, p, None, 0, None)
    assert rc == _lib.SSG_EINVAL and "aligned" in _lib.last_error()


def _validate(g):
    g = np.ascontiguousarray(g, np.uint32)
    return _lib.lib().ssg_validate_graph(g.ctypes.data_as(ctypes.c_void_p), g.shape[0], g.shape[1])


def test_validate_graph():
    S = 0xFFFFFFFF
    assert _validate([[1, 2, S], [0, S, S], [0, 1, S]]) == 0
    assert _validate([[1, S, 2], [0, S, S], [0, 1, S]]) == _lib.SSG_EINVAL  # id after padding
    assert "row 0" in _lib.last_error()
    assert _validate([[1, 1, S], [0, S, S], [0, 1, S]]) == _lib.SSG_EINVAL  # duplicate
    assert _validate([[0, S, S], [0, S, S], [0, 1, S]]) == _lib.SSG_EINVAL  # self loop
    assert _validate([[1, 3, S], [0, S, S], [0, 1, S]]) == _lib.SSG_EINVAL  # id >= n


def test_validate_oracle_graphs():
    """Graphs the oracle builds meet the search's preconditions: a small
    NSSG built here, and every stored full-size graph that is present."""
    import synth
    from oracle import cache, core
    cfg = dict(synth.CONFIGS["c2s"], n=3000)
    base = synth.base_vectors(cfg)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, 40)
    g = core.nssg_build(base, knn, 60, 32, 60.0, entry)["graph"]
    assert _validate(g) == 0
    for name in ("c2", "c3", "c4"):
        if cache.exists(name, "graph"):
            assert _validate(cache.load(name, "graph")) == 0, name


@pytest.mark.parametrize("n,d,K", [(1, 8, 1), (100, 0, 5), (100, 8, 0), (100, 8, 101), (10, 8, 10),
                                   ((1 << 25) + 1, 8, 5)])
def test_knn_rejects_bad_shapes_on_host(n, d, K):
    keep, p = _fake()
    rc = _lib.lib().ssg_knn_graph(p, n, d, K, p, p, p, 1 << 40, None, None)
    assert rc == _lib.SSG_EINVAL
    assert "ssg_knn_graph" in _lib.last_error()


def test_knn_rejects_small_or_misaligned_workspace():
    keep, p = _fake()
    need = _lib.lib().ssg_knn_workspace_bytes(1000, 32, 10)
    assert need > 1000 * 32 * 4
    assert _lib.lib().ssg_knn_graph(p, 1000, 32, 10, p, p, p, need - 1, None, None) == _lib.SSG_EINVAL
    assert _lib.lib().ssg_knn_graph(p, 1000, 32, 10, p, p, p + 8, need, None, None) == _lib.SSG_EINVAL
    assert _lib.lib().ssg_knn_workspace_bytes(1, 32, 10) == 0


def test_build_steps_reject_bad_arguments_on_host():
    keep, p = _fake()
    L = _lib.lib()
    assert L.ssg_nssg_prune(p, 100, 8, p, 10, 20, 65, 0.25, p, None) == _lib.SSG_EINVAL  # R > 64
    assert L.ssg_nssg_prune(p, 100, 8, p, 600, 500, 16, 0.25, p, None) == _lib.SSG_EUNSUPPORTED
    assert L.ssg_nssg_prune(p, 100, 8, p, 10, 20, 16, 1.5, p, None) == _lib.SSG_EINVAL
    assert L.ssg_nssg_prune(None, 100, 8, p, 10, 20, 16, 0.25, p, None) == _lib.SSG_EINVAL
    need = L.ssg_nssg_reverse_workspace_bytes(1000, 16)
    assert need > 1000 * 16 * 4
    assert L.ssg_nssg_reverse(p, 1000, 8, p, 16, 0.25, p, p, need - 1, None) == _lib.SSG_EINVAL
    assert L.ssg_nssg_reverse(p, 1000, 8, p, 16, 0.25, p, p + 8, need, None) == _lib.SSG_EINVAL
    assert "ssg_nssg_reverse" in _lib.last_error()


def test_merge_shards_rejects_bad_arguments_on_host():
    keep, p = _fake()
    L = _lib.lib()
    assert L.ssg_merge_shards(p, p, 0, 10, 5, p, p, 100, 5, p, p, None) == _lib.SSG_EINVAL
    assert L.ssg_merge_shards(p, p, 50, 10, 100, p, p, 100, 5, p, p, None) == _lib.SSG_EUNSUPPORTED
    assert L.ssg_merge_shards(p, p, 2, 10, 5, p, p, 100, 11, p, p, None) == _lib.SSG_EINVAL
    assert L.ssg_merge_shards(p, p, 2, 10, 5, p, p, -1, 5, p, p, None) == _lib.SSG_EINVAL
    assert L.ssg_merge_shards(None, p, 2, 10, 5, p, p, 100, 5, p, p, None) == _lib.SSG_EINVAL
    assert L.ssg_merge_shards(None, None, 2, 0, 5, None, None, 0, 5, None, None, None) == _lib.SSG_OK


def _call_ex(n=100, **opts):
    keep, p = _fake()
    o = _lib.SearchOpts()
    for k, v in opts.items():
        setattr(o, k, v)
    return _lib.lib().ssg_search_ex(p, n, 32, 0, None, p, 8, p, 2, p, 4, 10, 20, 0, p, p,
                                    ctypes.byref(o), None)


@pytest.mark.parametrize("n,opts,code", [
    (100, dict(visited_kind=4), _lib.SSG_EINVAL),
    (100, dict(visited_kind=-1), _lib.SSG_EINVAL),
    (100, dict(hash_log2=3), _lib.SSG_EINVAL),
    (100, dict(hash_log2=16), _lib.SSG_EINVAL),
    # a 16-bit tag cannot hold ids of 2^30 nodes with 1,024 sets: the cache
    # form is refused when asked for explicitly (the default falls back to the hash)
    (1 << 30, dict(visited_kind=2, hash_log2=12), _lib.SSG_EUNSUPPORTED),
    (1 << 20, dict(exact_visited=1), _lib.SSG_EUNSUPPORTED),
    (100, dict(entry_group_size=-1), _lib.SSG_EINVAL),
])
def test_search_options_rejected_on_host(n, opts, code):
    assert _call_ex(n, **opts) == code
    assert len(_lib.last_error()) > 0


def test_query_lds_bytes_on_host():
    """The per-search LDS figure serving admits by: grows with the pool's
    bucket, is 0 for shapes the search rejects, and leaves the last error
    message alone."""
    L = _lib.lib()
    f = L.ssg_query_lds_bytes
    b64 = f(64, 50, 128, _lib.SSG_F32, 1_000_000, 0, 0)
    b128 = f(100, 50, 128, _lib.SSG_F32, 1_000_000, 0, 0)
    b512 = f(512, 50, 128, _lib.SSG_F32, 1_000_000, 0, 0)
    assert 0 < b64 < b128 < b512 <= 64 * 1024
    assert f(33, 50, 128, _lib.SSG_F32, 10 ** 6, 0, 0) == b64  # one bucket, one size
    assert b64 % 16 == 0
    # a 4096-entry 16-bit tag cache (8 KB) and the merge stage are in it
    assert b64 >= 8192 + 64 * 8
    assert f(513, 50, 128, _lib.SSG_F32, 10 ** 6, 0, 0) == 0
    assert f(64, 65, 128, _lib.SSG_F32, 10 ** 6, 0, 0) == 0
    assert f(64, 50, 100, _lib.SSG_BF16, 10 ** 6, 0, 0) == 0  # d not a multiple of 8
    assert f(64, 50, 128, 7, 10 ** 6, 0, 0) == 0
    assert L.ssg_validate_graph(None, 1, 1) == _lib.SSG_EINVAL
    msg = _lib.last_error()
    f(64, 50, 128, _lib.SSG_F32, 10 ** 6, 0, 99)  # a bad visited size: 0, message kept
    assert f(64, 50, 128, _lib.SSG_F32, 10 ** 6, 0, 99) == 0
    assert _lib.last_error() == msg


def _batch(rerank):
    keep, p = _fake(1 << 14)
    d = _lib.BatchDesc(p, 100, 32, 0, 0, None, p, rerank, p, 8, p, 2, p, 4, p, p, 10, p, p,
                       None, None, None, 0)
    b = (_lib.Bucket * 1)()
    b[0] = _lib.Bucket(p, 4, 64, 0, 0, 0, 0, 0, 0)
    return keep, p, d, b


def test_batched_rerank_multiple_rejected_on_host():
    """rerank = -m reranks m * K_i entries for 1 <= m <= 16; below -16 the
    call is refused before anything reaches the device."""
    keep, p, d, b = _batch(-17)
    rc = _lib.lib().ssg_search_batched(ctypes.byref(d), b, 1, ctypes.c_void_p(p), 1 << 12, None)
    assert rc == _lib.SSG_EINVAL and "rerank" in _lib.last_error()


def test_no_alloc_entry_rejects_bucket_counts_on_host():
    keep, p, d, b = _batch(0)
    for nb in (0, 65):
        assert _lib.lib().ssg_search_batched_noalloc(ctypes.byref(d), b, nb, None) == _lib.SSG_EINVAL
        assert "64" in _lib.last_error()
