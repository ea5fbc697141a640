"""Exact-SSG study (Alg. 2, Table 1 and Theorem 3), computed by the oracle.

    python -m oracle.exact_ssg_study [--out summary.json] [--sets ssg10k,...]

For each 10,000 x 128 set and minimum angle: the exact SSG over all pairs
(Alg. 2), its average and largest out-degree, and greedy search paths
(Alg. 1 with L = 1 from a random start, FP64) on the whole graph and on the
graph truncated to each node's T nearest out-edges (the truncated SSG of
Table 1): the mean number of moves for 1,000 indexed queries (base points;
success = the point itself) and 1,000 unindexed queries (success = the
exact nearest neighbour).

Theorem 3 (Sec. 3.2, proof in the appendix): along the greedy path to an
unindexed query q, take each move p -> s made while every out-edge of p in
the exact SSG is shorter than delta(p, q) (the theorem's condition). The
move is monotonic towards q by construction of the greedy step; the
statistic is the fraction of such moves that also bring the search closer
to r, q's exact nearest neighbour (ties by the smaller id). The theorem
gives 0.5 + eps (0 < eps <= 0.5) for alpha <= 60 degrees and 1 for
alpha <= 30 degrees, for data distributed at random.
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
from oracle import core  # noqa: E402

SENT = core.SENT
TRUNC = {60.0: 40, 45.0: 80, 30.0: 120}  # out-edges kept in the truncated graphs


def greedy_paths(base, graph, Q, starts, trace_cap):
    """Alg. 1 with L = 1 from starts[i] for query i: (found id, moves, trace)."""
    found = np.empty(len(Q), np.uint32)
    moves = np.empty(len(Q), np.int64)
    tr = np.full((len(Q), trace_cap), SENT, np.uint32)
    for i, (q, s) in enumerate(zip(Q, starts)):
        ids, _, _, hops, t = core.search(base, graph, np.array([s], np.uint32), q[None], 1, 1,
                                         trace=trace_cap)
        found[i], moves[i], tr[i] = ids[0, 0], hops[0] - 1, t[0]
    return found, moves, tr


def theorem3(base, adj, deg, Q, nn, trace):
    """Moves p -> s along greedy paths to unindexed queries, and the fraction
    of them that also come closer to r = NN(q). Three sets of moves: those
    meeting the theorem's condition (every out-edge of p shorter than
    delta(p, q)); those whose chosen edge is shorter than delta(p, q) (the
    triangle the proof argues about); all moves."""
    b64 = base.astype(np.float64)
    maxedge = np.array([((b64[adj[i, :deg[i]]] - b64[i]) ** 2).sum(1).max() if deg[i] else 0.0
                        for i in range(len(base))])
    cnt = {"strict": [0, 0], "chosen_edge": [0, 0], "all": [0, 0]}
    for q, r, t in zip(Q.astype(np.float64), nn, trace):
        path = t[t != SENT].astype(np.int64)
        for p, s in zip(path[:-1], path[1:]):
            dpq = ((b64[p] - q) ** 2).sum()
            mono = ((b64[s] - b64[r]) ** 2).sum() < ((b64[p] - b64[r]) ** 2).sum()
            for key, ok in (("strict", maxedge[p] < dpq),
                            ("chosen_edge", ((b64[s] - b64[p]) ** 2).sum() < dpq), ("all", True)):
                if ok:
                    cnt[key][0] += 1
                    cnt[key][1] += int(mono)
    return {k: {"moves": c[0], "monotonic_to_nn": (c[1] / c[0] if c[0] else None)} for k, c in cnt.items()}


def study(name: str, alphas, seed: int = 2024):
    cfg = synth.CONFIGS[name]
    base = synth.base_vectors(cfg)
    n = len(base)
    Q = synth.queries(cfg, base)
    rng = np.random.default_rng(seed)
    idx_q = rng.choice(n, 1000, replace=False).astype(np.uint32)
    nn, _ = core.bruteforce(base, Q, 1)
    nn = nn[:, 0]
    s_idx = rng.integers(0, n, 1000).astype(np.uint32)
    s_un = rng.integers(0, n, len(Q)).astype(np.uint32)
    rows = []
    for alpha in alphas:
        t0 = time.time()
        adj, deg = core.ssg_exact(base, alpha)
        build = time.time() - t0
        mod = int(deg.max())
        full = np.ascontiguousarray(adj[:, :max(mod, 1)])
        T = TRUNC[alpha]
        tr_graph = np.ascontiguousarray(full[:, :T]) if mod > T else full
        for label, g in (("full", full), (f"truncated at {T}", tr_graph)):
            cap = 4 * int(np.sqrt(n)) + 64
            fi, mi, _ = greedy_paths(base, g, base[idx_q], s_idx, cap)
            fu, mu, tu = greedy_paths(base, g, Q, s_un, cap)
            gd = (g != SENT).sum(1)
            row = dict(set=name, alpha=alpha, graph=label, aod=float(gd.mean()), mod=int(gd.max()),
                       path_indexed=float(mi.mean()), found_indexed=float((fi == idx_q).mean()),
                       path_unindexed=float(mu.mean()), found_unindexed=float((fu == nn).mean()))
            if label == "full":
                row["exact_ssg_build_s"] = build
                row["theorem3"] = theorem3(base, adj, deg, Q, nn, tu)
            rows.append(row)
            print(json.dumps(row), flush=True)
    return rows


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--sets", default="ssg10k,ssg10k_r16")
    a = ap.parse_args()
    plan = {"ssg10k": (60.0, 45.0, 30.0), "ssg10k_r16": (60.0, 45.0)}
    rows = []
    for nm in a.sets.split(","):
        rows += study(nm, plan.get(nm, (60.0, 30.0)))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(rows, f, indent=1)


if __name__ == "__main__":
    main()
