import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long CPU test")


@pytest.fixture(scope="session")
def oracle_lib():
    from oracle import core
    return core.lib()


@pytest.fixture(scope="session")
def c1_graph():
    """The tiny workload (10,000 x 32) with its NSSG built by the oracle:
    (base, queries, graph, entry_ids, gt_ids, gt_dists)."""
    import synth
    from oracle import core
    cfg = synth.CONFIGS["c1"]
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)
    entry = synth.entry_choice(cfg)
    knn, _ = core.knn_graph(base, cfg["knn_k"])
    res = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry)
    gt_i, gt_d = core.ground_truth(base, q, 10)
    return base, q, res["graph"], entry, gt_i, gt_d
