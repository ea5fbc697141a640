"""GPU parity of every compiled search shape against the oracle.

The search kernels are instantiated per vector type, per dimension (d = 32,
96, 100, 128, 300 and 960 have shapes of their own; any other d runs the
runtime-dimension kernel, here d = 64 and 200) and, for d = 128, per gather
variant (lanes per candidate x candidates in flight). Each shape runs in the
plain and the persistent batched form.

Data: the SIFT-shaped integer mixture (values 0..255) at each dimension, so
FP32 sums are exact and BF16 storage is lossless: ids, distances, expansion
counts and expansion records must equal the oracle's (Alg. 1 in FP64). FP8
storage is lossy: the oracle searches the dequantized vectors and every row
must be the oracle's, differ only by near-equal keys, or part from the
oracle's trajectory at a near-tie (no genuine difference).
"""

import numpy as np
import pytest

import synth
from oracle import core, precision as P

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
SENT = core.SENT

_INDEX = {}


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


def _index(d):
    """A 3,000-point NSSG index of the integer mixture at dimension d."""
    if d not in _INDEX:
        cfg = dict(kind="gmm_int", n=3_000, d=d, comps=8, rank=16, nq_unindexed=160,
                   nq_indexed=0, knn_k=40, l=60, R=32, alpha=60.0, s=10, metric="l2",
                   seed=7000 + d)
        base = synth.base_vectors(cfg)
        q = synth.queries(cfg, base)
        entry = synth.entry_choice(cfg)
        knn, _ = core.knn_graph(base, cfg["knn_k"])
        g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
        _INDEX[d] = (base, q, g, entry)
    return _INDEX[d]


def _codes(base, fmt):
    tb = _dev(base)
    if fmt == "f32":
        return tb, None, base
    from paper_1907_06146_amd import quantize
    codes, scale = quantize(tb, fmt)
    torch.cuda.synchronize()
    if fmt == "bf16":
        deq = P.bf16_decode(codes.view(torch.int16).cpu().numpy().view(np.uint16))
        assert np.array_equal(deq, base)  # integers up to 255 are exact in BF16
    else:
        deq = P.fp8_dequantize(codes.cpu().numpy(), scale.cpu().numpy())
    return codes, scale, deq


def _check(fmt, base, deq, q, gi, gd, ghops, gtr, oi, od, ohops, otr, what):
    if fmt == "fp8":
        from parity_util import assert_parity, classify
        rows = classify(deq, q, gi, oi, "l2", 1e-5, gtr, otr)
        assert_parity(rows, 0.99, what)
        return
    assert np.array_equal(gi, oi), what
    assert np.array_equal(gd.astype(np.float64), od), what
    assert np.array_equal(ghops, ohops), what
    assert np.array_equal(gtr, otr), what


SHAPES = ([("f32", d, 0) for d in (32, 64, 96, 100, 200, 300, 960)]
          + [("f32", 128, v) for v in range(7)]
          + [("bf16", d, 0) for d in (64, 96, 200, 960)]
          + [("bf16", 96, 4)] + [("bf16", 128, v) for v in (0, 2, 3, 4, 7, 8)]
          + [("fp8", d, 0) for d in (64, 96, 960)]
          + [("fp8", 128, v) for v in (0, 1, 2, 3)])


@pytest.mark.parametrize("fmt,d,variant", SHAPES)
def test_shape_plain_and_batched(fmt, d, variant):
    from paper_1907_06146_amd import search
    from paper_1907_06146_amd.batched import BatchedSearch
    base, q, g, entry = _index(d)
    codes, scale, deq = _codes(base, fmt)
    tg, te, tq = _dev(g), _dev(entry), _dev(q)
    for L, K in ((40, 10), (130, 100)):
        T = L + 64
        oi, od, _, ohops, otr = core.search(deq, g, entry, q, K, L, trace=T)
        out = search(codes, tg, te, tq, K, L, dim_scale=scale, stats=True, trace=T,
                     gather_variant=variant)
        torch.cuda.synchronize()
        gi, gd, _, ghops, gtr = [t.cpu().numpy() for t in out]
        _check(fmt, base, deq, q, gi.view(np.uint32), gd, ghops, gtr.view(np.uint32),
               oi, od, ohops, otr, f"{fmt} d={d} variant={variant} L={L} K={K}")
    # the persistent batched form: mixed L over all four pool capacities
    rng = np.random.default_rng(d + variant)
    Lq = rng.choice(np.arange(16, 513, 16), size=len(q)).astype(np.int32)
    Kq = rng.choice([1, 10, 100], size=len(q)).astype(np.int32)
    T = 512 + 64
    shapes = {cap: {"gather_variant": variant} for cap in (64, 128, 256, 512)}
    bs = BatchedSearch(codes, tg, te, tq, Lq, Kq, "l2", dim_scale=scale, shapes=shapes,
                       stats=True, trace=T, use_graph=False)
    ids, dd = bs.run()
    torch.cuda.synchronize()
    oi, od, _, ohops, otr = core.search(deq, g, entry, q, 100, 512, L_arr=Lq, K_arr=Kq, trace=T)
    gi = ids.cpu().numpy().view(np.uint32)
    gd = dd.cpu().numpy()
    _check(fmt, base, deq, q, gi, gd, bs.hops.cpu().numpy(), bs.trace.cpu().numpy().view(np.uint32),
           oi, od, ohops, otr, f"{fmt} d={d} variant={variant} batched")
    for r in range(len(q)):  # padding past each K_i
        assert (gi[r, Kq[r]:] == SENT).all() and np.isinf(gd[r, Kq[r]:]).all()
