"""Host-side bucket planning of the batched search (no GPU)."""

import numpy as np
import pytest

torch = pytest.importorskip("torch")
from paper_1907_06146_amd.batched import plan_buckets  # noqa: E402


def test_buckets_partition_and_order():
    rng = np.random.default_rng(0)
    L = rng.choice(np.arange(16, 513, 16), size=1000)
    plan = plan_buckets(L)
    seen = np.concatenate([q for _, q in plan])
    assert sorted(seen.tolist()) == list(range(1000))
    lo = 0
    for (mL, q), hi in zip(plan, [b for b in (64, 128, 256, 512) if ((L > 0) & (L <= b)).any()]):
        assert (L[q] <= mL).all() and mL <= hi
        assert (np.diff(L[q]) <= 0).all()  # longest searches first
        ties = L[q][1:] == L[q][:-1]
        assert (np.diff(q)[ties] > 0).all()  # equal L: ascending index


def test_bad_pool_sizes_rejected():
    with pytest.raises(ValueError):
        plan_buckets(np.array([10, 600]))
    with pytest.raises(ValueError):
        plan_buckets(np.array([0, 10]))


def test_autotuner_candidates():
    """The shapes the autotuner times: every compiled gather variant of the
    storage type at d = 128 (and the query-in-LDS variant of 96-d BF16), both
    visited-cache sizes, one or two wavefronts per workgroup, and two queries
    per wavefront only where a grouped kernel exists (d = 96 or 128, pool
    capacity at most 256)."""
    torch = pytest.importorskip("torch")
    from paper_1907_06146_amd.autotune import candidate_shapes

    def variants(dt, d, cap=512):
        return sorted({s["gather_variant"] for s in candidate_shapes(dt, d, cap)})

    assert variants(torch.float32, 128) == [0, 1, 2, 3]
    assert variants(torch.bfloat16, 128) == [0, 2, 7, 8]
    assert variants(torch.uint8, 128) == [0, 3]
    assert variants(torch.bfloat16, 96) == [0, 4]
    assert variants(torch.float32, 960) == [0]
    for dt in (torch.float32, torch.bfloat16, torch.uint8):
        for d in (96, 128, 960):
            for cap in (64, 256, 512):
                shapes = candidate_shapes(dt, d, cap)
                grouped = [s for s in shapes if s["queries_per_wave"] == 2]
                assert bool(grouped) == (d in (96, 128) and cap <= 256)
                assert {s["hash_log2"] for s in shapes if s["queries_per_wave"] == 1} == {0, 11}
                assert {s["waves_per_block"] for s in shapes} == {1, 2}
