"""Row comparison of GPU results against the oracle (shared by GPU tests).

A row whose id list equals the oracle's is exact. A differing row is
explained when the FP64 keys of both lists agree element by element within
the tolerance (near-equal keys ordered differently by FP32 and FP64 sums).
Otherwise the two runs took different trajectories; given both expansion
records (the order in which Alg. 1 took nodes), the row is tie-diverged when
the first expansion where they part chose two nodes whose FP64 keys agree
within the tolerance: Alg. 1 defines one trajectory, and a near-tie decided
differently by FP32 and FP64 arithmetic is the only admissible reason for
leaving it. Any other differing row is genuine, and fails every bar."""

import dataclasses

import numpy as np

from oracle import core

SENT = core.SENT


@dataclasses.dataclass
class Rows:
    exact: np.ndarray
    explained: np.ndarray
    tie_diverged: np.ndarray
    genuine: np.ndarray

    def summary(self) -> str:
        return (f"exact {self.exact.mean():.5f} explained {self.explained.mean():.5f} "
                f"tie-diverged {self.tie_diverged.mean():.5f} genuine {int(self.genuine.sum())}")


def _close(a, b, tol):
    """Element-wise |a - b| <= tol * max(|a|, |b|) over finite pairs; +inf
    pairs agree; an inf against a finite value does not."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    fa, fb = np.isfinite(a), np.isfinite(b)
    both = fa & fb
    a0, b0 = np.where(both, a, 0.0), np.where(both, b, 0.0)
    scale = np.maximum(np.maximum(np.abs(a0), np.abs(b0)), 1e-30)
    return (fa == fb) & (~both | (np.abs(a0 - b0) <= tol * scale))


def _rows_of(trace, rows):
    """Trace rows as uint32 (GPU -1 padding = 0xFFFFFFFF): ``trace`` is an
    array over all rows or a function rows -> array for those rows."""
    t = trace(rows) if callable(trace) else np.asarray(trace)[rows]
    return np.asarray(t).astype(np.uint32)


def tie_diverged(search_base, q, rows, g_trace, o_trace, metric="l2", tol=1e-5):
    """For each of ``rows``: True when the two expansion records first part
    at two nodes whose FP64 keys (against ``search_base``, the vectors the
    search ran on) agree within tol. False when they never part within the
    records, or one run stopped where the other expanded."""
    rows = np.asarray(rows, np.int64)
    out = np.zeros(len(rows), bool)
    if len(rows) == 0:
        return out
    gt = _rows_of(g_trace, rows)
    ot = _rows_of(o_trace, rows)
    T = min(gt.shape[1], ot.shape[1])
    for i, r in enumerate(rows):
        diff = np.nonzero(gt[i, :T] != ot[i, :T])[0]
        if len(diff) == 0:
            continue
        a, b = gt[i, diff[0]], ot[i, diff[0]]
        if a == SENT or b == SENT:
            continue
        k = core.pair_keys(search_base, q[r:r + 1], np.array([[a, b]], np.uint32), metric)[0]
        out[i] = bool(_close(k[:1], k[1:], tol)[0])
    return out


def classify(base, q, gi, oi, metric="l2", tol=1e-5, g_trace=None, o_trace=None, search_base=None):
    """Classify every row of the GPU ids ``gi`` against the oracle's ``oi``.

    base         vectors the returned distances refer to (FP32)
    g_trace      GPU expansion records [nq, T] (int32, -1 padding), or a
                 function rows -> records of those rows
    o_trace      oracle expansion records, the same way (a function re-runs
                 the oracle on just the rows that need it)
    search_base  vectors the search ran on (the dequantized copy for a
                 reduced-precision search; default ``base``)
    """
    gi = np.asarray(gi).astype(np.uint32)
    oi = np.asarray(oi).astype(np.uint32)
    exact = (gi == oi).all(1)
    explained = np.zeros_like(exact)
    tie = np.zeros_like(exact)
    bad = np.nonzero(~exact)[0]
    if len(bad):
        kg = core.pair_keys(base, q[bad], gi[bad], metric)
        ko = core.pair_keys(base, q[bad], oi[bad], metric)
        explained[bad[_close(kg, ko, tol).all(1)]] = True
    rest = np.nonzero(~exact & ~explained)[0]
    if len(rest) and g_trace is not None and o_trace is not None:
        sb = base if search_base is None else search_base
        tie[rest] = tie_diverged(sb, q, rest, g_trace, o_trace, metric, tol)
    return Rows(exact, explained, tie, ~exact & ~explained & ~tie)


def assert_parity(rows: Rows, min_exact: float = 0.999, what: str = ""):
    """The bar: no genuine row, and at least ``min_exact`` of the rows exact
    (at least one non-exact row is always allowed, so a small test is not
    stricter than the fraction says)."""
    assert not rows.genuine.any(), f"{what}: genuine mismatches in rows " \
        f"{np.nonzero(rows.genuine)[0][:20].tolist()} ({rows.summary()})"
    n = len(rows.exact)
    allowed = max(1, int(np.floor((1.0 - min_exact) * n + 1e-9)))
    assert (~rows.exact).sum() <= allowed, f"{what}: {rows.summary()}"


def assert_hops_explained(search_base, q, exact, g_hops, o_hops, g_trace, o_trace, metric="l2",
                          tol=1e-5, what=""):
    """On rows with the oracle's ids, the expansion count equals the
    oracle's unless the trajectories part at a key tie (a near-tie deep in
    the pool can reorder expansions without changing the returned ids)."""
    rows = np.nonzero(exact & (np.asarray(g_hops) != np.asarray(o_hops)))[0]
    ok = tie_diverged(search_base, q, rows, g_trace, o_trace, metric, tol)
    assert ok.all(), f"{what}: hop counts differ without a tie in rows {rows[~ok][:20].tolist()}"
    return len(rows)
