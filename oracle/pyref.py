"""Independent pure-Python versions of Alg. 1 and of the SSG pruning rule.

TEST INFRASTRUCTURE ONLY, for tiny inputs. Written separately from the C
oracle (lists, Python floats = IEEE FP64, sequential sums) so the two can be
compared id for id: a mistake has to be made twice, the same way, to pass.
"""

from __future__ import annotations

import math

SENT = 0xFFFFFFFF


def _key(q, x, metric):
    if metric == "l2":
        s = 0.0
        for a, b in zip(q, x):
            t = float(a) - float(b)
            s += t * t
        return s
    s = 0.0
    for a, b in zip(q, x):
        s += float(a) * float(b)
    return -s


def search(base, graph, entry_ids, q, K, L, metric="l2", trace=False):
    """Alg. 1 from the navigating node nearest q. Returns (ids, keys, ndc,
    hops), and with trace=True also the ids of the expanded nodes in the
    order they were expanded."""
    base = [list(map(float, r)) for r in base]
    q = list(map(float, q))
    ndc = 0
    best = None
    for e in entry_ids:
        k = _key(q, base[e], metric)
        ndc += 1
        if best is None or (k, e) < best:
            best = (k, int(e))
    pool = [[best[0], best[1], False]]  # [key, id, checked]
    visited = {best[1]}
    hops = 0
    order = []
    while True:
        cur = next((c for c in pool if not c[2]), None)
        if cur is None:
            break
        cur[2] = True
        order.append(cur[1])
        for v in graph[cur[1]]:
            v = int(v)
            if v == SENT:
                break
            if v in visited:
                continue
            visited.add(v)
            pool.append([_key(q, base[v], metric), v, False])
            ndc += 1
        pool.sort(key=lambda c: (c[0], c[1]))
        del pool[L:]
        hops += 1
    ids = [c[1] for c in pool[:K]] + [SENT] * max(0, K - len(pool))
    keys = [c[0] for c in pool[:K]] + [math.inf] * max(0, K - len(pool))
    if trace:
        return ids, keys, ndc, hops, order
    return ids, keys, ndc, hops


def ssg_prune(base, i, cand_ids, alpha_deg, R=None):
    """SSG edge selection around node i from candidate ids: sort by (squared
    distance, id), keep a candidate when the angle at i to every kept edge is
    at least alpha. Uses the law of cosines on explicit vectors."""
    xi = [float(v) for v in base[i]]
    c2 = 0.25 if alpha_deg == 60.0 else math.cos(math.radians(alpha_deg)) ** 2
    cands = []
    for j in set(int(c) for c in cand_ids):
        if j == i:
            continue
        vec = [float(a) - b for a, b in zip(base[j], xi)]
        n2 = 0.0
        for t in vec:
            n2 += t * t
        if n2 == 0.0:
            continue
        cands.append((n2, j, vec))
    cands.sort(key=lambda c: (c[0], c[1]))
    kept = []
    for n2, j, vec in cands:
        if R is not None and len(kept) >= R:
            break
        ok = True
        for m2, k, w in kept:
            dot = 0.0
            for a, b in zip(vec, w):
                dot += a * b
            if dot > 0.0 and dot * dot > c2 * n2 * m2:
                ok = False
                break
        if ok:
            kept.append((n2, j, vec))
    return [j for _, j, _ in kept]


def bruteforce(base, q, K, metric="l2", skip=None):
    keys = sorted((_key(q, x, metric), j) for j, x in enumerate(base) if j != skip)
    top = keys[:K]
    return [j for _, j in top], [k for k, _ in top]
