"""Build the graph cache of a workload with the CPU oracle only.

    python -m oracle.build_cache c1 c2s c2 [--sweep] [--expand literal]

Steps (all FP64 oracle code, no GPU):
  1. regenerate base, queries and navigating nodes from the seed (synth);
  2. exact kNN graph (step 1 of Alg. 3, brute force);
  3. NSSG indexing (Alg. 3): expansion, SSG pruning, reverse-neighbour
     checking, DFS spanning from the navigating nodes;
  4. exact ground truth of the queries (Eq. 1's G);
  5. Alg. 1 from the nearest navigating node at the workload's pool sizes,
     recording ids, keys, NDC and hops as the stored expected values;
  6. for workloads with a steady-state query set (``nq_steady``): its exact
     top 10 and Alg. 1's first 10 ids, NDC and hops at the operating pool
     size;
  7. at the operating pool size, each query's sum of out-degrees over the
     nodes Alg. 1 expanded (from its expansion record): the neighbour-row
     bytes the search must read are 4 times that sum.
The kNN graph is kept under data/_cpu/ (not needed by GPU runs).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import synth  # noqa: E402
from oracle import cache, core  # noqa: E402


def log(*a):
    print(time.strftime("%H:%M:%S"), *a, flush=True)


def build(name: str, sweep: bool, expand: str, sweep_only: bool = False):
    cfg = synth.CONFIGS[name]
    core.lib()  # load the C oracle now: a rebuild during a long run cannot mix versions
    t0 = time.time()
    base = synth.base_vectors(cfg)
    q = synth.queries(cfg, base)
    entry = synth.entry_choice(cfg)
    Lq, Kq = synth.query_params(cfg)
    log(name, "data", base.shape, q.shape, f"{time.time() - t0:.1f}s")
    meta = dict(name=name, n=cfg["n"], d=cfg["d"], R=cfg["R"], s=cfg["s"], l=cfg["l"],
                alpha=cfg["alpha"], knn_k=cfg["knn_k"], metric=cfg["metric"], seed=cfg["seed"],
                expand=expand, base_sha=synth.checksum(base), queries_sha=synth.checksum(q),
                nq=int(q.shape[0]),
                readings=dict(visited_when_added=True, order="(dist,id)", seed="nearest_entry",
                              reverse="two_phase_reselect", zero_dist="dropped", dfs="lowest_id_first"))
    if not sweep_only:
        kpath = os.path.join(cache.data_root(), "_cpu", f"{name}_knn.npy")
        if os.path.exists(kpath):
            knn = np.load(kpath)
            log("knn loaded", knn.shape)
        else:
            t = time.time()
            if cfg.get("knn", "exact") == "ivf":
                knn, _ = core.knn_graph_ivf(base, cfg["knn_k"], cfg["nlist"], cfg["nprobe"],
                                            cfg["seed"] + 7, verbose=True)
                log("ivf knn", f"{time.time() - t:.1f}s", "accuracy", core.knn_accuracy(base, knn))
                knn = core.knn_refine(base, knn, cfg["refine_J"], cfg["refine_rounds"])
            else:
                knn, _ = core.knn_graph(base, cfg["knn_k"], verbose=cfg["n"] > 100_000)
            os.makedirs(os.path.dirname(kpath), exist_ok=True)
            np.save(kpath, knn)
            log("knn built", f"{time.time() - t:.1f}s")
        acc = core.knn_accuracy(base, knn, sample=300)
        meta.update(knn_method=cfg.get("knn", "exact"), knn_acc_1nn=acc[0], knn_acc_k=acc[1])
        log("knn accuracy (1-NN, K-NN)", acc)
        t = time.time()
        res = core.nssg_build(base, knn, cfg["l"], cfg["R"], cfg["alpha"], entry, expand)
        g = res["graph"]
        deg = (g != core.SENT).sum(1)
        log("nssg built", f"{time.time() - t:.1f}s", "AOD", deg.mean(), "MOD", deg.max(),
            "dfs edges", len(res["dfs_edges"]))
        meta.update(aod=float(deg.mean()), mod=int(deg.max()), n_dfs_edges=int(len(res["dfs_edges"])),
                    graph_sha=synth.checksum(g), build_s=time.time() - t)
        t = time.time()
        Kg = max(100, cfg["K"])
        gt_i, gt_d = core.ground_truth(base, q, Kg, cfg["metric"])
        log("ground truth", f"{time.time() - t:.1f}s")
        cache.save(name, dict(graph=g, entry_ids=entry, dfs_edges=res["dfs_edges"], gt_ids=gt_i,
                              gt_d=gt_d), meta)
    g = cache.load(name, "graph")
    gt_i = cache.load(name, "gt_ids")
    Ls = sorted(set(cfg.get("L_sweep", [])) | {cfg["L"]}) if sweep else [cfg["L"]]
    rows = []
    for L in Ls:
        t = time.time()
        ids, dd, ndc, hops = core.search(base, g, entry, q, cfg["K"], L, cfg["metric"])
        el = time.time() - t
        r10 = core.recall_at(ids, gt_i, 10) if cfg["K"] >= 10 else None
        row = dict(L=L, recall10=r10, ndc=float(ndc.mean()), hops=float(hops.mean()),
                   cpu_s=el, cpu_threads=os.cpu_count(), qps=q.shape[0] / el)
        rows.append(row)
        log(row)
        cache.save(name, {f"oracle_L{L}_ids": ids, f"oracle_L{L}_d": dd,
                          f"oracle_L{L}_ndc": ndc, f"oracle_L{L}_hops": hops}, {})
    if "L_choices" in cfg:  # mixed per-query L and K
        t = time.time()
        Kmax = int(Kq.max())
        ids, dd, ndc, hops = core.search(base, g, entry, q, Kmax, int(Lq.max()), cfg["metric"],
                                         L_arr=Lq, K_arr=Kq)
        log("mixed L/K oracle", f"{time.time() - t:.1f}s")
        cache.save(name, {"oracle_mixed_ids": ids, "oracle_mixed_d": dd, "oracle_mixed_ndc": ndc,
                          "oracle_mixed_hops": hops}, {})
    op = [r["L"] for r in rows if r["recall10"] is not None and r["recall10"] >= 0.95]
    L_op = op[0] if op else cfg["L"]
    if sweep:
        with open(os.path.join(cache.path(name), "sweep.json"), "w") as f:
            json.dump(dict(rows=rows, L_op=op[0] if op else None), f, indent=1)
    if cfg.get("nq_steady"):
        steady(name, cfg, base, g, entry, L_op)
    degsums(name, cfg, base, g, entry, L_op)
    log(name, "done", f"{time.time() - t0:.1f}s", "L_op", L_op)


def degsum_of(base, g, entry, q, K, L, metric):
    """Per query: the sum of the out-degrees of the nodes Alg. 1 expanded."""
    deg = (g != core.SENT).sum(1).astype(np.int64)
    out = np.empty(len(q), np.int64)
    for lo in range(0, len(q), 10_000):
        qq = q[lo:lo + 10_000]
        _, _, _, hops, tr = core.search(base, g, entry, qq, K, L, metric, trace=1)
        cap = int(hops.max())
        _, _, _, hops, tr = core.search(base, g, entry, qq, K, L, metric, trace=cap)
        valid = tr != core.SENT
        out[lo:lo + len(qq)] = np.where(valid, deg[np.where(valid, tr, 0).astype(np.int64)], 0).sum(1)
    return out


def degsums(name, cfg, base, g, entry, L):
    t = time.time()
    q = synth.queries(cfg, base)
    arrays = {f"oracle_L{L}_degsum": degsum_of(base, g, entry, q, cfg["K"], L, cfg["metric"])}
    if cfg.get("nq_steady"):
        arrays[f"steady_L{L}_degsum"] = degsum_of(base, g, entry, synth.steady_queries(cfg), cfg["K"], L,
                                                  cfg["metric"])
    cache.save(name, arrays, {})
    log("expanded-row degree sums", f"L={L}", f"{time.time() - t:.1f}s",
        {k: float(v.mean()) for k, v in arrays.items()})


def steady(name, cfg, base, g, entry, L):
    """Steady-state query set: exact top 10 and the oracle at pool size L."""
    t = time.time()
    qs = synth.steady_queries(cfg)
    gi, _ = core.ground_truth(base, qs, 10, cfg["metric"], verbose=True)
    log("steady ground truth", qs.shape, f"{time.time() - t:.1f}s")
    t = time.time()
    ids, _, ndc, hops = core.search(base, g, entry, qs, cfg["K"], L, cfg["metric"])
    r10 = core.recall_at(ids, gi, 10)
    log("steady oracle", f"L={L}", f"{time.time() - t:.1f}s", "recall@10", r10)
    cache.save(name, {"steady_gt_ids": gi, f"steady_L{L}_ids10": np.ascontiguousarray(ids[:, :10]),
                      f"steady_L{L}_ndc": ndc.astype(np.int32), f"steady_L{L}_hops": hops.astype(np.int32)},
               {"steady": dict(nq=int(len(qs)), L=int(L), recall10=r10, queries_sha=synth.checksum(qs),
                               ndc=float(ndc.mean()), hops=float(hops.mean()))})


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--sweep", action="store_true")
    ap.add_argument("--sweep-only", action="store_true")
    ap.add_argument("--expand", default="literal", choices=["literal", "hop1first"])
    ap.add_argument("--degsum-only", action="store_true",
                    help="only step 7, at the stored operating pool size")
    a = ap.parse_args()
    for nm in a.names:
        if a.degsum_only:
            core.lib()
            cfg = synth.CONFIGS[nm]
            sw = os.path.join(cache.path(nm), "sweep.json")
            L = (json.load(open(sw))["L_op"] if os.path.exists(sw) else None) or cfg["L"]
            degsums(nm, cfg, synth.base_vectors(cfg), cache.load(nm, "graph"), cache.load(nm, "entry_ids"), L)
            continue
        build(nm, a.sweep, a.expand, a.sweep_only)


if __name__ == "__main__":
    main()
