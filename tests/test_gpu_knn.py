"""GPU exact kNN graph (the kNN graph Alg. 3 starts from) against the oracle:
the same neighbour ids in the same (squared L2, id) order and the same FP64
distances, on integer data (exact matrix-core path) and on float data (split
path with certificate and FP64 rescan)."""

import numpy as np
import pytest

import synth
from oracle import core

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _run(base, K):
    from paper_1907_06146_amd import knn_graph
    ids, dd, st = knn_graph(torch.from_numpy(np.ascontiguousarray(base, np.float32)).cuda(), K)
    torch.cuda.synchronize()
    return ids.cpu().numpy().view(np.uint32), dd.cpu().numpy(), st


def _check(base, K, expect_exact):
    gi, gd, st = _run(base, K)
    oi, od = core.knn_graph(base, K)
    print(f"n={len(base)} d={base.shape[1]} K={K}: {st}", flush=True)
    assert st["exact_path"] == expect_exact
    assert np.array_equal(gi, oi), f"{(gi != oi).any(1).sum()} rows differ"
    assert np.array_equal(gd, od.astype(np.float32))
    return st


def test_integer_data_exact_path():
    """SIFT-like integer vectors in [0, 255], d = 128: the matrix-core keys
    are exact, so the result equals the oracle with no rescan."""
    base = synth.base_vectors("c2s")
    st = _check(base, 100, True)
    assert st["rescanned_rows"] == 0 and st["candidates"] == 100


def test_float_data_split_path():
    base = synth.base_vectors("c1")
    _check(base, 40, False)


def test_ragged_shapes_and_unaligned_rows():
    """n not a multiple of the 128-row tile, d = 50 (rows not 16-byte
    aligned, dimensions padded to 64)."""
    rng = np.random.default_rng(7)
    base = rng.standard_normal((3001, 50)).astype(np.float32)
    _check(base, 17, False)
    ib = rng.integers(0, 256, (1000, 20)).astype(np.float32)
    _check(ib, 9, True)


def test_duplicate_points_tie_by_id():
    """Many exact duplicates: distance-0 ties ordered by id, on both paths
    (the float path's certificate cannot separate ties and rescans)."""
    rng = np.random.default_rng(3)
    proto = rng.integers(0, 256, (40, 64)).astype(np.float32)
    base = proto[rng.integers(0, 40, 2500)]
    _check(base, 30, True)
    fb = (proto / 7.0 + 0.01)[rng.integers(0, 40, 2500)].astype(np.float32)
    st = _check(fb, 30, False)
    assert st["rescanned_rows"] > 0


@pytest.mark.parametrize("n,K", [(2, 1), (30, 29), (129, 100)])
def test_every_point_a_candidate(n, K):
    rng = np.random.default_rng(n)
    _check(rng.standard_normal((n, 16)).astype(np.float32), K, False)


@pytest.mark.parametrize("name,K", [("c2", 100), ("c4", 100)])
def test_full_size_sampled_rows(name, K):
    """1M-point sets (integer 128-d, unit-norm float 96-d): sampled rows
    against the oracle's full FP64 scan."""
    import time
    base = synth.base_vectors(name)
    t = time.time()
    gi, gd, st = _run(base, K)
    print(f"{name}: kNN graph {time.time() - t:.2f}s {st}", flush=True)
    rows = np.random.default_rng(11).choice(len(base), 48, replace=False)
    oi, od = core.bruteforce(base, base[rows], K, "l2", skip=rows)
    assert np.array_equal(gi[rows], oi)
    assert np.array_equal(gd[rows], od.astype(np.float32))
    assert st["exact_path"] == (name == "c2")
