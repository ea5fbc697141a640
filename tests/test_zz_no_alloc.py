"""ssg_search_batched_noalloc (work-queue counters in the library's own
per-device array) against ssg_search_batched (caller workspace), through
the C ABI: identical outputs on two calls in a row, the second with fewer
queries and fewer buckets, and the bucket-count limit rejected on the host."""

import ctypes

import numpy as np
import pytest

import synth
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


@pytest.fixture(scope="module")
def index():
    cfg = synth.CONFIGS["c4s"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)[:1500]
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    g = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)["graph"]
    return base, q, g, entry


def _pair(index, nq, L_choices, seed, dtype="f32", persistent=False):
    """Two BatchedSearch objects over the same queries: the workspace form
    and the no-allocation form (each with its own output buffers); with
    persistent=True every bucket runs as a persistent grid taking queries
    from its work-queue counter (the counters the no-allocation form keeps in
    its own array)."""
    from paper_1907_06146_amd import quantize
    from paper_1907_06146_amd.batched import BatchedSearch
    base, q, g, entry = index
    rng = np.random.default_rng(seed)
    Lq = rng.choice(L_choices, size=nq).astype(np.int32)
    Kq = rng.choice([1, 10, 100], size=nq).astype(np.int32)
    tb = _dev(base)
    kw = {}
    bse = tb
    if dtype == "bf16":
        bse, _ = quantize(tb, "bf16")
        kw = dict(base_f32=tb, rerank=-1)
    args = (bse, _dev(g), _dev(entry), _dev(q[:nq]), Lq, Kq, "ip")
    if persistent:
        kw["shapes"] = {cap: {"blocks": 96} for cap in (64, 128, 256, 512)}
    ref = BatchedSearch(*args, use_graph=False, stats=True, **kw)
    new = BatchedSearch(*args, use_graph=False, stats=True, no_alloc=True, **kw)
    return ref, new


@pytest.mark.parametrize("dtype,persistent", [("f32", True), ("bf16", True), ("f32", False)])
def test_no_alloc_equals_workspace_form(index, dtype, persistent):
    big = _pair(index, 1500, np.arange(16, 513, 16), 1, dtype, persistent)   # all four buckets
    small = _pair(index, 300, np.arange(16, 129, 16), 2, dtype, persistent)  # two buckets, fewer queries
    assert len(big[1].plan) == 4 and len(small[1].plan) == 2
    for ref, new in (big, small):  # two calls in a row, the second smaller
        ref.run()
        new.run()
        torch.cuda.synchronize()
        assert torch.equal(ref.out_ids, new.out_ids)
        assert torch.equal(ref.out_d, new.out_d)
        assert torch.equal(ref.hops, new.hops)
    # the first call's outputs are not disturbed by the second
    again = _pair(index, 1500, np.arange(16, 513, 16), 1, dtype, persistent)[1]
    again.run()
    torch.cuda.synchronize()
    assert torch.equal(again.out_ids, big[0].out_ids)


def test_no_alloc_rejects_too_many_buckets(index):
    from paper_1907_06146_amd import _lib
    ref, new = _pair(index, 64, np.arange(16, 65, 16), 3)
    arr = (_lib.Bucket * 65)()
    for i in range(65):
        arr[i] = new.buckets[0]
    st = torch.cuda.current_stream()
    rc = _lib.lib().ssg_search_batched_noalloc(ctypes.byref(new.desc), arr, 65,
                                               ctypes.c_void_p(st.cuda_stream))
    assert rc == _lib.SSG_EINVAL and "64" in _lib.last_error()
    rc = _lib.lib().ssg_search_batched_noalloc(ctypes.byref(new.desc), arr, 0,
                                               ctypes.c_void_p(st.cuda_stream))
    assert rc == _lib.SSG_EINVAL
