"""Pins of the precision-form oracle: number formats from their definitions.

FP8 E4M3 (OCP): largest finite 448, smallest normal 2^-6, smallest subnormal
2^-9, one NaN pattern per sign and no infinities. bfloat16: the upper half of
a binary32, so the integers 0..256 are exact (8 significant bits).
"""

import numpy as np

from oracle import core, precision as P


def test_fp8_table_landmarks():
    t = P.fp8_table()
    assert t[0x7E] == 448.0 and t[0xFE] == -448.0
    assert t[0x08] == 2.0 ** -6 and t[0x01] == 2.0 ** -9 and t[0x07] == 7 * 2.0 ** -9
    assert t[0x38] == 1.0 and t[0x39] == 1.125
    assert np.isnan(t[0x7F]) and np.isnan(t[0xFF])
    assert t[0x00] == 0.0 and np.signbit(t[0x80])
    fin = t[np.isfinite(t)]
    assert len(fin) == 254 and np.isinf(t).sum() == 0


def test_fp8_encode_roundtrip_ties_and_saturation():
    codes = np.array([c for c in range(256) if c not in (0x7F, 0xFF)], np.uint8)
    assert np.array_equal(P.fp8_encode(P.fp8_decode(codes)), codes)
    # midpoints go to the even code
    assert P.fp8_encode(np.array([1.0625]))[0] == 0x38       # between 1.0 and 1.125
    assert P.fp8_encode(np.array([1.1875]))[0] == 0x3A       # between 1.125 and 1.25
    assert P.fp8_encode(np.array([2.0 ** -10]))[0] == 0x00   # half the smallest subnormal
    assert P.fp8_encode(np.array([3 * 2.0 ** -10]))[0] == 0x02
    assert P.fp8_encode(np.array([1000.0, -1000.0, 460.0])).tolist() == [0x7E, 0xFE, 0x7E]
    # nearest: every value maps to a code whose value is closest
    rng = np.random.default_rng(0)
    v = rng.uniform(-448, 448, 20000) * rng.choice([1, 1e-2, 1e-4], 20000)
    c = P.fp8_encode(v)
    err = np.abs(P.fp8_decode(c) - v)
    alt = np.abs(P.fp8_table()[None, np.isfinite(P.fp8_table())] - v[:, None]).min(1)
    assert np.allclose(err, alt, rtol=0, atol=0)


def test_bf16_encode():
    x = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -1.0 - 2 ** -8, 3.140625], np.float32)
    assert P.bf16_encode(x).tolist() == [0x3F80, 0x3F80, 0x3F82, 0xBF80, 0x4049]
    ints = np.arange(0, 257, dtype=np.float32)
    assert np.array_equal(P.bf16_decode(P.bf16_encode(ints)), ints)
    rng = np.random.default_rng(1)
    v = rng.standard_normal(5000).astype(np.float32)
    d = P.bf16_decode(P.bf16_encode(v))
    assert (np.abs(d - v) <= np.abs(v) * 2.0 ** -8).all()


def test_fp8_scale_and_dequantize():
    x = np.array([[0.0, -3.5, 1.0], [0.0, 2.0, -4.0]], np.float32)
    c, s = P.fp8_quantize(x)
    assert s.tolist() == [1.0, np.float32(3.5) / np.float32(448), np.float32(4.0) / np.float32(448)]
    assert c[0, 1] == 0xFE and c[1, 2] == 0xFE  # column maxima map to +-448
    deq = P.fp8_dequantize(c, s)
    assert np.allclose(deq, x, rtol=2 ** -4, atol=0)


def test_precision_search_reduces_to_plain_search_when_lossless(c1_graph):
    base, q, g, entry, _, _ = c1_graph
    grid = np.rint(base * 4).astype(np.float32)  # values k/4 with |k| < 256: bf16-exact
    deq = P.bf16_decode(P.bf16_encode(grid))
    assert np.array_equal(deq, grid)
    a = core.search(grid, g, entry, q, 10, 40)
    b = P.search_precision(grid, deq, g, entry, q, 10, 40, rerank=40)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])


def test_rerank_only_reorders_the_searched_entries(c1_graph):
    base, q, g, entry, _, _ = c1_graph
    c, s = P.fp8_quantize(base)
    deq = P.fp8_dequantize(c, s)
    ids0, _ = P.search_precision(base, deq, g, entry, q, 10, 50, rerank=-1)
    ids1, d1 = P.search_precision(base, deq, g, entry, q, 10, 50, rerank=10)
    for a, b in zip(ids0, ids1):
        assert set(a.tolist()) == set(b.tolist())
    assert (np.diff(d1, axis=1) >= 0).all()
    assert np.allclose(d1, core.pair_keys(base, q, ids1), rtol=0, atol=0)
