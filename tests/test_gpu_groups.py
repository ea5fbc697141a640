"""GPU parity of the search with two queries per wavefront (32 lanes each).

The grouped kernel computes Alg. 1 per query exactly like the one-query
kernel: on integer data (exact FP32 sums) ids, distances and expansion
counts equal the oracle's; on float data every row is the oracle's, or
differs by key ties, or parts from the oracle's trajectory at a tie. Cases:
odd query counts (a wavefront with one idle group), pool sizes at each
register capacity (64, 96, 128, 256) and between, a visited cache small
enough to evict (the duplicate check), FP32 rerank, BF16 / FP8 storage,
inner product on 96-d data, per-shard entry sets, and the persistent
batched form with mixed L and K.
"""

import numpy as np
import pytest

import synth
from oracle import core, precision as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
SENT = core.SENT


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def _gpu(base, g, entry, q, K, L, metric="l2", **kw):
    from paper_1907_06146_amd import search
    out = search(base if isinstance(base, torch.Tensor) else _dev(base), _dev(g), _dev(entry),
                 _dev(q), K, L, metric, stats=True, queries_per_wave=2, **kw)
    torch.cuda.synchronize()
    out = [t.cpu().numpy() for t in out]
    out[0] = out[0].view(np.uint32)
    return out


@pytest.fixture(scope="module")
def c2s():
    cfg = synth.CONFIGS["c2s"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
    return base, q, g, entry


@pytest.mark.parametrize("L,K", [(1, 1), (10, 10), (33, 100), (64, 64), (65, 10), (96, 100),
                                 (97, 20), (128, 128), (129, 50), (256, 100)])
def test_integer_data_bit_exact(c2s, L, K):
    base, q, g, entry = c2s
    oi, od, ondc, ohops, otr = core.search(base, g, entry, q, K, L, trace=L + 64)
    gi, gd, gndc, ghops, gtr = _gpu(base, g, entry, q, K, L, trace=L + 64)
    assert np.array_equal(gi, oi)
    assert np.array_equal(gd.astype(np.float64), od)
    assert np.array_equal(ghops, ohops)
    assert np.array_equal(gtr.view(np.uint32), otr)
    assert (gndc >= ondc).all()


@pytest.mark.parametrize("nq", [1, 2, 3, 63, 65])
def test_odd_query_counts(c2s, nq):
    base, q, g, entry = c2s
    q = q[:nq]
    oi, od, _, ohops = core.search(base, g, entry, q, 20, 48)
    gi, gd, _, ghops = _gpu(base, g, entry, q, 20, 48)
    assert np.array_equal(gi, oi) and np.array_equal(gd.astype(np.float64), od)
    assert np.array_equal(ghops, ohops)


@pytest.mark.parametrize("hash_log2", [4, 6, 8])
def test_evicting_cache_is_result_neutral(c2s, hash_log2):
    """A cache of 16 to 256 entries evicts pool members: the duplicate check
    must drop every returning copy."""
    base, q, g, entry = c2s
    K, L = 50, 200
    oi, od, ondc, ohops = core.search(base, g, entry, q, K, L)
    gi, gd, gndc, ghops = _gpu(base, g, entry, q, K, L, hash_log2=hash_log2)
    assert np.array_equal(gi, oi) and np.array_equal(gd.astype(np.float64), od)
    assert np.array_equal(ghops, ohops)
    assert (gndc > ondc).mean() > 0.5  # most queries recomputed something


def test_same_results_as_one_query_per_wave(c2s):
    from paper_1907_06146_amd import search
    base, q, g, entry = c2s
    tb = _dev(base)
    for dt in (torch.float32, torch.bfloat16):
        bb = tb.to(dt)
        for L, K in ((80, 100), (200, 10)):
            a = search(bb, _dev(g), _dev(entry), _dev(q), K, L, queries_per_wave=1)
            b = search(bb, _dev(g), _dev(entry), _dev(q), K, L, queries_per_wave=2)
            c = search(bb, _dev(g), _dev(entry), _dev(q), K, L, queries_per_wave=2, base_f32=tb,
                       rerank_k=L)
            d = search(bb, _dev(g), _dev(entry), _dev(q), K, L, queries_per_wave=1, base_f32=tb,
                       rerank_k=L)
            torch.cuda.synchronize()
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
            assert torch.equal(c[0], d[0]) and torch.equal(c[1], d[1])


def test_entry_groups(c2s):
    """Per-shard entry sets (the block-diagonal partitioned search)."""
    base, q, g, entry = c2s
    rng = np.random.default_rng(3)
    groups = np.stack([rng.choice(len(base), 10, replace=False) for _ in range(4)]).astype(np.uint32)
    qq = q[:64]
    gi, gd, _, _ = _gpu(base, g, groups, qq, 10, 40, entry_group_size=16)
    for s in range(4):
        oi, od, _, _ = core.search(base, g, groups[s], qq[16 * s:16 * s + 16], 10, 40)
        assert np.array_equal(gi[16 * s:16 * s + 16], oi)


@pytest.fixture(scope="module")
def c4s():
    cfg = synth.CONFIGS["c4s"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)[:600]
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
    return cfg, base, q, g, entry


@pytest.mark.parametrize("fmt", ["f32", "bf16", "fp8"])
def test_float_data_inner_product(c4s, fmt):
    from parity_util import assert_parity, classify

    from paper_1907_06146_amd import quantize
    cfg, base, q, g, entry = c4s
    tb = _dev(base)
    if fmt == "f32":
        codes, scale, deq = tb, None, base
    else:
        codes, scale = quantize(tb, fmt)
        torch.cuda.synchronize()
        deq = (P.bf16_decode(codes.view(torch.int16).cpu().numpy().view(np.uint16)) if fmt == "bf16"
               else P.fp8_dequantize(codes.cpu().numpy(), scale.cpu().numpy()))
    for L, K in ((16, 1), (96, 10), (256, 100)):
        T = 4 * L + 64
        oi, od, _, _, otr = core.search(deq, g, entry, q, K, L, "ip", trace=T)
        gi, gd, _, _, gtr = _gpu(codes, g, entry, q, K, L, "ip", dim_scale=scale, trace=T)
        rows = classify(deq, q, gi, oi, "ip", 1e-5, gtr, otr)
        assert_parity(rows, 0.99, f"{fmt} L={L} K={K}")


def test_batched_mixed_lk_grouped(c4s):
    from parity_util import assert_parity, classify

    from paper_1907_06146_amd.batched import BatchedSearch
    cfg, base, q, g, entry = c4s
    rng = np.random.default_rng(11)
    Lq = rng.choice(np.arange(16, 257, 16), size=len(q)).astype(np.int32)
    Kq = rng.choice([1, 10, 100], size=len(q)).astype(np.int32)
    T = 4 * 256 + 64
    shapes = {cap: {"queries_per_wave": 2} for cap in (64, 128, 256)}
    bs = BatchedSearch(_dev(base), _dev(g), _dev(entry), _dev(q), Lq, Kq, "ip", shapes=shapes,
                       stats=True, trace=T)
    ids, dd = bs.run()
    torch.cuda.synchronize()
    oi, od, _, _, otr = core.search(base, g, entry, q, 100, 256, "ip", L_arr=Lq, K_arr=Kq, trace=T)
    gi = ids.cpu().numpy().view(np.uint32)
    rows = classify(base, q, gi, oi, "ip", 1e-5, bs.trace.cpu().numpy(), otr)
    assert_parity(rows, 0.99, "grouped mixed batch")
    dd = dd.cpu().numpy()
    for r in range(len(q)):  # padding past each K_i
        assert (gi[r, Kq[r]:] == SENT).all() and np.isinf(dd[r, Kq[r]:]).all()
    bs.close()


def test_grouped_shape_rejected_when_it_cannot_run(c2s):
    from paper_1907_06146_amd import _lib, search
    base, q, g, entry = c2s
    with pytest.raises(_lib.SSGError):  # L above 256
        search(_dev(base), _dev(g), _dev(entry), _dev(q[:4]), 10, 300, queries_per_wave=2)
    with pytest.raises(_lib.SSGError):  # exact visited set
        search(_dev(base), _dev(g), _dev(entry), _dev(q[:4]), 10, 64, queries_per_wave=2,
               exact_visited=True)
    with pytest.raises(_lib.SSGError):  # d = 32 has no compiled grouped shape
        search(_dev(base[:, :32].copy()), _dev(g), _dev(entry), _dev(q[:4, :32].copy()), 10, 64,
               queries_per_wave=2)
