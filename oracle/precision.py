"""Oracle for the precision form of the search (test infrastructure only).

The paper computes exact distances on full-precision vectors (Sec. 6.1); the
precision form stores vectors in BF16 or OCP FP8 E4M3 (per-dimension scale),
runs Alg. 1 on the dequantized values and re-scores the first ``rerank``
pool entries against the FP32 vectors. This module restates both number
formats from their definitions and runs that procedure with the FP64 oracle.

Encoders here pick the nearest representable value by comparing candidates
(ties to the even code); they do not use bit-rounding tricks, so they check
the library's bit-level encoders independently.
"""

from __future__ import annotations

import numpy as np

from . import core

FP8_MAX = 448.0


# ------------------------------------------------------------------ bfloat16
def bf16_decode(codes: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> float32 (exact: the upper half of a binary32)."""
    return (codes.astype(np.uint32) << 16).view(np.float32)


def bf16_encode(x: np.ndarray) -> np.ndarray:
    """Nearest bfloat16 to each finite float32, ties to an even last bit."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    u = x.view(np.uint32)
    lo = (u >> 16).astype(np.uint32)                     # truncation toward zero
    hi = lo + 1                                          # next value away from zero
    vx = x.astype(np.float64)
    dl = np.abs(bf16_decode(lo.astype(np.uint16)).astype(np.float64) - vx)
    dh = np.abs(bf16_decode(hi.astype(np.uint16)).astype(np.float64) - vx)
    pick_hi = (dh < dl) | ((dh == dl) & ((lo & 1) == 1))
    return np.where(pick_hi, hi, lo).astype(np.uint16)


# ------------------------------------------------------------------ FP8 E4M3
def fp8_table() -> np.ndarray:
    """Values of all 256 OCP E4M3 codes: sign | 4-bit exponent (bias 7) |
    3-bit mantissa; exponent 0 is subnormal (m * 2^-9); S.1111.111 is NaN;
    there are no infinities."""
    v = np.empty(256, np.float64)
    for c in range(256):
        s = -1.0 if c & 0x80 else 1.0
        e = (c >> 3) & 0xF
        m = c & 0x7
        if e == 0xF and m == 0x7:
            v[c] = np.nan
        elif e == 0:
            v[c] = s * m * 2.0 ** -9
        else:
            v[c] = s * (1.0 + m / 8.0) * 2.0 ** (e - 7)
    return v


_TAB = fp8_table()
_POS_CODES = np.arange(0x7F)          # 0 .. 0x7E: the finite non-negative codes
_POS_VALS = _TAB[_POS_CODES]          # ascending


def fp8_decode(codes: np.ndarray) -> np.ndarray:
    return _TAB[codes.astype(np.int64)]


def fp8_encode(v: np.ndarray) -> np.ndarray:
    """Nearest E4M3 code to each value, ties to the even code, magnitudes
    beyond 448 saturate to +-448."""
    v = np.asarray(v, np.float64)
    a = np.minimum(np.abs(v), FP8_MAX)
    j = np.clip(np.searchsorted(_POS_VALS, a), 1, len(_POS_VALS) - 1)
    lo, hi = j - 1, j
    dl = a - _POS_VALS[lo]
    dh = _POS_VALS[hi] - a
    pick_hi = (dh < dl) | ((dh == dl) & ((_POS_CODES[lo] & 1) == 1))
    code = np.where(pick_hi, _POS_CODES[hi], _POS_CODES[lo]).astype(np.uint8)
    code = np.where(a == 0, 0, code).astype(np.uint8)
    neg = np.signbit(v)
    return np.where(neg, code | 0x80, code).astype(np.uint8)


def fp8_scale(x: np.ndarray) -> np.ndarray:
    """Per-dimension scale s_j = max_i |x_ij| / 448 in float32 (1 if zero)."""
    m = np.abs(np.asarray(x, np.float32)).max(axis=0).astype(np.float32)
    s = np.where(m > 0, m / np.float32(FP8_MAX), np.float32(1.0))
    return s.astype(np.float32)


def fp8_quantize(x: np.ndarray):
    """Codes of x_ij / s_j (the quotient rounded to float32 first)."""
    x = np.asarray(x, np.float32)
    s = fp8_scale(x)
    q = (x / s[None, :]).astype(np.float32)
    return fp8_encode(q), s


def fp8_dequantize(codes: np.ndarray, s: np.ndarray) -> np.ndarray:
    """decode(code) * s_j rounded to float32 (the product is exact in FP64)."""
    return (fp8_decode(codes) * s.astype(np.float64)[None, :]).astype(np.float32)


# ------------------------------------------------------------------ search
def search_precision(base_f32, deq, graph, entry_ids, Q, K: int, L: int, metric: str = "l2",
                     rerank: int = 0):
    """Alg. 1 on the dequantized vectors ``deq`` (FP64 keys), then the first
    min(max(rerank, K), |S|) pool entries re-scored with exact FP64 keys
    against the FP32 vectors and re-sorted by (dist, id); the first K are
    returned, so every returned entry has been re-scored. rerank = 0 means K;
    without rerank (rerank < 0) the pool order is kept."""
    if rerank < 0:
        return core.search(deq, graph, entry_ids, Q, K, L, metric)[:2]
    rr = min(max(rerank, K), L)
    Kp = max(K, rr)
    ids, _, _, _ = core.search(deq, graph, entry_ids, Q, Kp, L, metric)
    keys = core.pair_keys(base_f32, Q, ids[:, :rr], metric)
    out_i = np.full((len(Q), K), core.SENT, np.uint32)
    out_d = np.full((len(Q), K), np.inf)
    for r in range(len(Q)):
        valid = ids[r, :rr] != core.SENT
        ii, kk = ids[r, :rr][valid], keys[r][valid]
        order = np.lexsort((ii, kk))[:K]
        out_i[r, :len(order)] = ii[order]
        out_d[r, :len(order)] = kk[order]
    return out_i, out_d
