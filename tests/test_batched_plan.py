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
