"""GPU parity at the boundary's maximum sizes: rows of 64 neighbour ids
(every slot used), 4,096 navigating nodes, a pool of 512, and a batched call
of 64 L buckets (the most one call takes), through the workspace and the
no-allocation entry points. Integer data, so every FP32 sum is exact and ids,
distances and expansion counts must equal the oracle's."""

import numpy as np
import pytest

from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
SENT = core.SENT


def _dev(a):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint32:
        a = a.view(np.int32)
    return torch.from_numpy(a).cuda()


@pytest.fixture(scope="module")
def full_rows():
    """6,000 integer points in 32-d, every row holding 64 distinct random
    neighbours (a dense random graph: long searches, full rows)."""
    rng = np.random.default_rng(77)
    n = 6000
    base = rng.integers(0, 64, size=(n, 32)).astype(np.float32)
    g = np.empty((n, 64), np.uint32)
    for i in range(n):
        g[i] = rng.choice(np.delete(np.arange(n), i), size=64, replace=False)
    q = rng.integers(0, 64, size=(96, 32)).astype(np.float32)
    return base, g, q


def test_full_rows_many_entries_largest_pool(full_rows):
    from paper_1907_06146_amd import search
    base, g, q = full_rows
    entry = np.random.default_rng(5).choice(len(base), 4096, replace=False).astype(np.uint32)
    for K, L in ((10, 512), (600, 512), (64, 64)):
        oi, od, ondc, ohops = core.search(base, g, entry, q, K, L)
        ids, dd, ndc, hops = search(_dev(base), _dev(g), _dev(entry), _dev(q), K, L, stats=True)
        torch.cuda.synchronize()
        assert np.array_equal(ids.cpu().numpy().view(np.uint32), oi), (K, L)
        assert np.array_equal(dd.cpu().numpy().astype(np.float64), od), (K, L)
        assert np.array_equal(hops.cpu().numpy(), ohops) and (ndc.cpu().numpy() >= ondc).all()


def test_sixty_four_buckets(full_rows):
    """Pool sizes 1..512 split into 64 buckets of capacity 8, 16, ..., 512:
    the same rows as the default four buckets and as the oracle."""
    from paper_1907_06146_amd.batched import BatchedSearch
    base, g, q = full_rows
    rng = np.random.default_rng(6)
    q = np.concatenate([q] * 4)  # 384 queries
    # every bucket of width 8 holds 6 queries
    Lq = np.array([8 * (i % 64 + 1) - (i // 64) % 8 for i in range(len(q))], np.int32)
    rng.shuffle(Lq)
    Kq = rng.choice([1, 10, 100], size=len(q)).astype(np.int32)
    entry = rng.choice(len(base), 10, replace=False).astype(np.uint32)
    args = (_dev(base), _dev(g), _dev(entry), _dev(q), Lq, Kq, "l2")
    bounds = tuple(range(8, 513, 8))
    assert len(bounds) == 64
    outs = []
    for kw in (dict(), dict(bounds=bounds), dict(bounds=bounds, no_alloc=True)):
        bs = BatchedSearch(*args, use_graph=False, stats=True, **kw)
        ids, dd = bs.run()
        torch.cuda.synchronize()
        outs.append((ids.cpu().numpy().view(np.uint32).copy(), dd.cpu().numpy().copy(),
                     bs.hops.cpu().numpy().copy()))
        bs.close()
    assert len(BatchedSearch(*args, use_graph=False, bounds=bounds).plan) == 64
    for o in outs[1:]:
        assert all(np.array_equal(x, y) for x, y in zip(o, outs[0]))
    oi, od, _, ohops = core.search(base, g, entry, q, 100, 512, L_arr=Lq, K_arr=Kq)
    assert np.array_equal(outs[0][0], oi)
    assert np.array_equal(outs[0][2], ohops)
