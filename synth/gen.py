"""Seeded generators for the synthetic stand-ins of the paper's datasets.

The paper evaluates on SIFT1M (128-d, LID 12.9), GIST1M (960-d, LID 29.1) and
Deep (96-d, LID 10.2) among others (Table 2). Those files are not available, so
every workload here is drawn from a seeded mixture with the same shape:

* ``c1``   10,000 x 32 Gaussian mixture, 50 components, sigma 0.3, plus 20
           base points reused as indexed queries.
* ``c2``   1,000,000 x 128 integers 0..255 (SIFT-like), 1,000 overlapping
           rank-16 Gaussian clusters, clipped and rounded (LID about 13).
* ``c3``   1,000,000 x 960 values in [0, 1] (GIST-like), 500 overlapping
           rank-20 clusters around a Dirichlet-shaped mean profile (LID about 28).
* ``c4``   1,000,000 x 96 unit-norm points of one shared rank-12 latent space
           with overlapping clusters (Deep-like), inner product, queries with
           per-query pool size L and result count K.
* ``c5``   5,000,000 x 96, the c4 distribution, for the serving loop.
* ``*s``   small variants of the same distributions for parity tests.

Determinism across machines: only random draws, element-wise IEEE arithmetic
(+, -, *, /, sqrt) and clipping/rounding are used to build the vectors. No
BLAS call and no vectorised transcendental function touches the data, so the
same numpy version produces bit-identical arrays on any x86-64 host.
``checksum`` gives a short digest that cache files record and loaders verify.
"""

from __future__ import annotations

import hashlib

import numpy as np

_CHUNK = 65536  # fixed row chunk: keeps the random stream order independent of memory

# Search sweep for the SIFT-shaped workload: L = 10..100 step 10, then 120..300 step 20.
_C2_SWEEP = list(range(10, 101, 10)) + list(range(120, 301, 20))

CONFIGS: dict[str, dict] = {
    "c1": dict(kind="gmm_iso", n=10_000, d=32, comps=50, sigma=0.3,
               nq_unindexed=100, nq_indexed=20, knn_k=40, l=100, R=24,
               alpha=60.0, s=10, L=50, K=10, metric="l2", seed=1000),
    "c2": dict(kind="gmm_int", n=1_000_000, d=128, comps=1000, rank=16,
               nq_unindexed=10_000, nq_indexed=0, knn_k=100, l=100, R=50,
               alpha=60.0, s=10, L=100, K=100, L_sweep=_C2_SWEEP,
               metric="l2", seed=2000, nq_steady=100_000),
    "c2s": dict(kind="gmm_int", n=20_000, d=128, comps=40, rank=16,
                nq_unindexed=500, nq_indexed=12, knn_k=100, l=100, R=50,
                alpha=60.0, s=10, L=64, K=100, metric="l2", seed=2100),
    # the exact-SSG study (10,000 points, like the paper's SIFT10K experiment):
    # a low-intrinsic-dimension set (rank-4 clusters), on which the 30-degree
    # SSG keeps a few hundred edges per node, and the SIFT-shaped mixture
    "ssg10k": dict(kind="gmm_int", n=10_000, d=128, comps=10, rank=4,
                   nq_unindexed=1_000, nq_indexed=0, s=10, metric="l2", seed=2300),
    "ssg10k_r16": dict(kind="gmm_int", n=10_000, d=128, comps=10, rank=16,
                       nq_unindexed=1_000, nq_indexed=0, s=10, metric="l2", seed=2400),
    "c3": dict(kind="dirichlet", n=1_000_000, d=960, comps=500, rank=20, eps=0.003,
               nq_unindexed=1_000, nq_indexed=0, knn_k=100, l=500, R=50,
               alpha=60.0, s=10, L=200, K=10, L_sweep=list(range(100, 501, 50)),
               metric="l2", seed=3000, nq_steady=16_000,
               knn="ivf", nlist=1000, nprobe=16, refine_J=32, refine_rounds=3),
    "c3s": dict(kind="dirichlet", n=8_000, d=960, comps=20, rank=20, eps=0.003,
                nq_unindexed=100, nq_indexed=4, knn_k=60, l=120, R=50,
                alpha=60.0, s=10, L=100, K=10, metric="l2", seed=3100),
    "c4": dict(kind="unit_lowrank", n=1_000_000, d=96, comps=1000, rank=12,
               nq_unindexed=100_000, nq_indexed=0, knn_k=100, l=100, R=50,
               alpha=60.0, s=10, L=128, K=10, metric="ip", seed=4000,
               L_choices=list(range(16, 513, 16)), K_choices=[1, 10, 100]),
    "c4s": dict(kind="unit_lowrank", n=20_000, d=96, comps=40, rank=12,
                nq_unindexed=2_000, nq_indexed=0, knn_k=60, l=100, R=50,
                alpha=60.0, s=10, L=128, K=10, metric="ip", seed=4100,
                L_choices=list(range(16, 513, 16)), K_choices=[1, 10, 100]),
    "c5": dict(kind="unit_lowrank", n=5_000_000, d=96, comps=5000, rank=12,
               nq_unindexed=95_000, nq_indexed=5_000, knn_k=64, l=100, R=32,
               alpha=60.0, s=10, L=96, K=10, metric="ip", seed=5000,
               L_choices=list(range(32, 257, 16)), K_choices=[10],
               knn="ivf", nlist=5000, nprobe=24, refine_J=32, refine_rounds=3),
}


def _cfg(name_or_cfg) -> dict:
    return CONFIGS[name_or_cfg] if isinstance(name_or_cfg, str) else name_or_cfg


# ---------------------------------------------------------------- mixtures
def _params(cfg: dict):
    """Mixture parameters, drawn first from the base stream."""
    rng = np.random.default_rng(cfg["seed"])
    d, k = cfg["d"], cfg["comps"]
    kind = cfg["kind"]
    if kind == "gmm_iso":
        return rng, dict(mu=rng.standard_normal((k, d)))
    if kind == "gmm_int":
        # overlapping clusters (centre spread 12 vs in-cluster spread ~24 per
        # dimension): one connected point cloud whose measured LID (MLE, k=20)
        # is about 13, like SIFT1M's 12.9
        mu = rng.normal(40.0, 12.0, (k, d))
        U = rng.normal(0.0, 6.0, (k, d, cfg["rank"]))
        return rng, dict(mu=mu, U=U)
    if kind == "dirichlet":
        # one skewed Dirichlet-shaped mean profile shared by all clusters, small
        # per-cluster offsets and low-rank in-cluster spread: overlapping
        # clusters in [0, 1] with a high intrinsic dimension, like GIST1M
        m = cfg.get("floor", 0.05) + rng.dirichlet(np.full(d, 0.5)) * (d * 0.1)
        mu = m[None, :] + rng.normal(0.0, cfg.get("c_off", 0.02), (k, d))
        V = rng.normal(0.0, cfg.get("u_std", 0.03), (k, d, cfg["rank"]))
        return rng, dict(mu=mu, U=V)
    if kind == "unit_lowrank":
        # one shared rank-r latent space (projection A) holding overlapping
        # Gaussian clusters; points are A u + noise, normalised to unit length,
        # so the data is one connected low-dimensional piece of the sphere
        r = cfg["rank"]
        A = rng.standard_normal((d, r))
        mu = rng.normal(0.0, cfg.get("c_spread", 1.0), (k, r))
        return rng, dict(A=A, mu=mu)
    raise ValueError(kind)


def _chunk_values(cfg: dict, p: dict, lab: np.ndarray, z: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Rows of one chunk from its labels and its two blocks of draws (z, then
    e). Element-wise IEEE operations only, so the result does not depend on
    which thread computes it."""
    kind = cfg["kind"]
    c = len(lab)
    if kind == "gmm_iso":
        x = p["mu"][lab] + cfg["sigma"] * e
    elif kind == "unit_lowrank":
        u = p["mu"][lab] + cfg.get("u_spread", 0.8) * z
        x = np.zeros((c, cfg["d"]))
        for t in range(cfg["rank"]):  # element-wise projection (no BLAS)
            x += u[:, t:t + 1] * p["At"][t][None, :]
        x += e
        s = np.zeros(c)
        for j in range(cfg["d"]):  # fixed-order squared norm
            s += x[:, j] * x[:, j]
        x = x / np.sqrt(s)[:, None]
    else:
        x = p["mu"][lab]  # fancy indexing returns a copy
        for t in range(cfg["rank"]):  # explicit element-wise low-rank product (no BLAS)
            x += p["Ut"][t][lab] * z[:, t:t + 1]
        x += e
        if kind == "gmm_int":
            x = np.rint(np.clip(x, 0.0, 255.0))
        else:  # dirichlet
            x = np.clip(x, 0.0, 1.0)
    return x.astype(np.float32)


def _draw(cfg: dict, p: dict, rng: np.random.Generator, m: int) -> np.ndarray:
    """Draw m points of the mixture from ``rng``; returns float32 (m, d).

    The random stream is consumed in one fixed order (labels, then per chunk
    of rows the latent draws and the noise); the arithmetic of each chunk runs
    on a small thread pool (numpy releases the interpreter lock there)."""
    import concurrent.futures as cf
    import os
    d, k, kind = cfg["d"], cfg["comps"], cfg["kind"]
    p = dict(p)
    if "U" in p:
        p["Ut"] = [np.ascontiguousarray(p["U"][:, :, t]) for t in range(cfg["rank"])]
    if "A" in p:
        p["At"] = [np.ascontiguousarray(p["A"][:, t]) for t in range(cfg["rank"])]
    out = np.empty((m, d), dtype=np.float32)
    labels = rng.integers(0, k, m)
    workers = max(1, min(8, os.cpu_count() or 1))
    pending = []

    def put(lo, hi, fut):
        out[lo:hi] = fut.result()

    with cf.ThreadPoolExecutor(workers) as ex:
        for lo in range(0, m, _CHUNK):
            hi = min(m, lo + _CHUNK)
            c = hi - lo
            if kind == "gmm_iso":
                z, e = None, rng.standard_normal((c, d))
            elif kind == "unit_lowrank":
                z = rng.standard_normal((c, cfg["rank"]))
                e = rng.normal(0.0, cfg.get("eps", 0.3), (c, d))
            else:
                z = rng.standard_normal((c, cfg["rank"]))
                e = rng.normal(0.0, 1.0 if kind == "gmm_int" else cfg.get("eps", 0.01), (c, d))
            pending.append((lo, hi, ex.submit(_chunk_values, cfg, p, labels[lo:hi], z, e)))
            while len(pending) > workers:  # bound the chunks held in memory
                put(*pending.pop(0))
        for item in pending:
            put(*item)
    return out


def base_vectors(cfg) -> np.ndarray:
    """The n x d float32 base set S of a workload."""
    cfg = _cfg(cfg)
    rng, p = _params(cfg)
    return _draw(cfg, p, rng, cfg["n"])


def indexed_query_ids(cfg) -> np.ndarray:
    """Ids of base points that are reused verbatim as indexed queries."""
    cfg = _cfg(cfg)
    m = cfg.get("nq_indexed", 0)
    rng = np.random.default_rng(cfg["seed"] + 11)
    return np.sort(rng.choice(cfg["n"], size=m, replace=False)).astype(np.uint32)


def queries(cfg, base: np.ndarray | None = None) -> np.ndarray:
    """Unindexed queries from the same mixture, then the indexed ones."""
    cfg = _cfg(cfg)
    _, p = _params(cfg)
    rng = np.random.default_rng(cfg["seed"] + 1)
    q = _draw(cfg, p, rng, cfg["nq_unindexed"])
    ids = indexed_query_ids(cfg)
    if len(ids):
        if base is None:
            base = base_vectors(cfg)
        q = np.concatenate([q, base[ids]], axis=0)
    return np.ascontiguousarray(q, dtype=np.float32)


def steady_queries(cfg) -> np.ndarray:
    """A second, larger set of unindexed queries from the same mixture (its
    own stream, seed + 5), all distinct from each other and from the main
    set, for throughput measured with the device full of searches."""
    cfg = _cfg(cfg)
    _, p = _params(cfg)
    rng = np.random.default_rng(cfg["seed"] + 5)
    return np.ascontiguousarray(_draw(cfg, p, rng, cfg["nq_steady"]), dtype=np.float32)


def query_params(cfg) -> tuple[np.ndarray, np.ndarray]:
    """Per-query pool size L_i and result count K_i for the mixed workloads."""
    cfg = _cfg(cfg)
    nq = cfg["nq_unindexed"] + cfg.get("nq_indexed", 0)
    rng = np.random.default_rng(cfg["seed"] + 3)
    if "L_choices" not in cfg:
        return (np.full(nq, cfg["L"], np.int32), np.full(nq, cfg["K"], np.int32))
    L = rng.choice(np.asarray(cfg["L_choices"], np.int32), size=nq)
    K = rng.choice(np.asarray(cfg["K_choices"], np.int32), size=nq)
    return L.astype(np.int32), K.astype(np.int32)


def entry_choice(cfg) -> np.ndarray:
    """s navigating nodes drawn without replacement (the random choice the
    indexing algorithm makes before DFS spanning)."""
    cfg = _cfg(cfg)
    rng = np.random.default_rng(cfg["seed"] + 2)
    return rng.choice(cfg["n"], size=cfg["s"], replace=False).astype(np.uint32)


def checksum(a: np.ndarray) -> str:
    """Short content digest of an array (dtype, shape and bytes)."""
    h = hashlib.sha1()
    h.update(str(a.dtype).encode())
    h.update(str(a.shape).encode())
    h.update(np.ascontiguousarray(a).view(np.uint8).reshape(-1).data)
    return h.hexdigest()[:16]
