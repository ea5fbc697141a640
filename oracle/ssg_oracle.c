/*
 * ssg_oracle.c -- CPU reference implementation of the Satellite System Graph
 * method (Fu, Wang, Cai: "High Dimensional Similarity Search with Satellite
 * System Graph", arXiv 1907.06146).
 *
 * TEST INFRASTRUCTURE ONLY. This file is the slow, plain oracle that the GPU
 * search is checked against. Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark load it. It shares no code, header, table or
 * helper with the HIP library.
 *
 * Arithmetic: every distance and every angle test is evaluated in IEEE FP64,
 * summed sequentially over the dimensions in index order, with floating-point
 * contraction disabled at compile time (-ffp-contract=off). fp32 inputs are
 * widened exactly. The total order on candidates is (distance, id) ascending.
 *
 * Entry points (all return 0 on success, a negative value on a bad argument):
 *   orc_bruteforce   exact top-K by full scan (ground truth; kNN rows)
 *   orc_rerank       exact top-K among a given candidate list per row
 *   orc_nssg_prune   Alg. 3 candidate expansion + SSG pruning per node
 *   orc_nssg_reverse Alg. 3 reverse-neighbour checking
 *   orc_dfs_connect  Alg. 3 navigating nodes + DFS spanning
 *   orc_search       Alg. 1 from the nearest navigating node
 *   orc_ssg_exact    Alg. 2 (exact SSG over all pairs, tiny n only)
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SENT 0xFFFFFFFFu

typedef struct {
    double dist;
    uint32_t id;
    uint32_t checked;
} cand_t;

static int cand_cmp(const void *pa, const void *pb) {
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->dist < b->dist) return -1;
    if (a->dist > b->dist) return 1;
    return (a->id > b->id) - (a->id < b->id);
}

/* Distance key between two fp32 vectors.
 * metric 0: squared Euclidean distance (same order as the Euclidean delta of
 *           the paper's notation section); metric 1: negative inner product. */
static double key_dist(const float *a, const float *b, int d, int metric) {
    double s = 0.0;
    if (metric == 0) {
        for (int j = 0; j < d; ++j) {
            double t = (double)a[j] - (double)b[j];
            s += t * t;
        }
        return s;
    }
    for (int j = 0; j < d; ++j) s += (double)a[j] * (double)b[j];
    return -s;
}

/* <a - c, b - c> in FP64, sequential over dimensions. */
static double dot_rel(const float *a, const float *b, const float *c, int d) {
    double s = 0.0;
    for (int j = 0; j < d; ++j) s += ((double)a[j] - (double)c[j]) * ((double)b[j] - (double)c[j]);
    return s;
}

/* ------------------------------------------------------------ top-K helpers */

/* Insert (dist,id) into a sorted array of at most K entries. */
static void topk_push(cand_t *top, int *cnt, int K, double dist, uint32_t id) {
    int c = *cnt;
    if (c == K) {
        cand_t last = top[K - 1];
        if (dist > last.dist || (dist == last.dist && id > last.id)) return;
        c = K - 1;
    }
    int p = c;
    while (p > 0 && (top[p - 1].dist > dist || (top[p - 1].dist == dist && top[p - 1].id > id))) {
        top[p] = top[p - 1];
        --p;
    }
    top[p].dist = dist;
    top[p].id = id;
    top[p].checked = 0;
    *cnt = c + 1;
}

/* Exact top-K of each query row by a full scan of the base set.
 * skip[r] (optional) is an id that row r must not return (the point itself
 * when a kNN graph is built). Output rows are padded with SENT / +inf. */
int orc_bruteforce(const float *base, int64_t n, int d, const float *Q, int64_t nq,
                   const int64_t *skip, int K, int metric, uint32_t *out_ids, double *out_d) {
    if (!base || !Q || !out_ids || !out_d || n < 0 || d < 1 || nq < 0 || K < 1) return -1;
#pragma omp parallel
    {
        cand_t *top = (cand_t *)malloc(sizeof(cand_t) * (size_t)K);
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nq; ++r) {
            int cnt = 0;
            const float *q = Q + (size_t)r * d;
            int64_t sk = skip ? skip[r] : -1;
            for (int64_t j = 0; j < n; ++j) {
                if (j == sk) continue;
                topk_push(top, &cnt, K, key_dist(q, base + (size_t)j * d, d, metric), (uint32_t)j);
            }
            for (int t = 0; t < K; ++t) {
                out_ids[(size_t)r * K + t] = t < cnt ? top[t].id : SENT;
                out_d[(size_t)r * K + t] = t < cnt ? top[t].dist : INFINITY;
            }
        }
        free(top);
    }
    return 0;
}

/* Exact top-K among cand[r][0..C) for each row (ids < 0 are ignored, as are
 * skip[r] and repeated ids). Used after a coarse candidate pass. */
int orc_rerank(const float *base, int64_t n, int d, const float *Q, int64_t nq,
               const int64_t *skip, const int64_t *cand, int C, int K, int metric,
               uint32_t *out_ids, double *out_d) {
    if (!base || !Q || !cand || !out_ids || !out_d || d < 1 || C < 1 || K < 1) return -1;
    int bad = 0;
#pragma omp parallel
    {
        cand_t *top = (cand_t *)malloc(sizeof(cand_t) * (size_t)K);
#pragma omp for schedule(dynamic, 64) reduction(| : bad)
        for (int64_t r = 0; r < nq; ++r) {
            int cnt = 0;
            const float *q = Q + (size_t)r * d;
            int64_t sk = skip ? skip[r] : -1;
            for (int c = 0; c < C; ++c) {
                int64_t j = cand[(size_t)r * C + c];
                if (j < 0 || j == sk) continue;
                if (j >= n) { bad = 1; continue; }
                int dup = 0;
                for (int c2 = 0; c2 < c; ++c2)
                    if (cand[(size_t)r * C + c2] == j) { dup = 1; break; }
                if (dup) continue;
                topk_push(top, &cnt, K, key_dist(q, base + (size_t)j * d, d, metric), (uint32_t)j);
            }
            for (int t = 0; t < K; ++t) {
                out_ids[(size_t)r * K + t] = t < cnt ? top[t].id : SENT;
                out_d[(size_t)r * K + t] = t < cnt ? top[t].dist : INFINITY;
            }
        }
        free(top);
    }
    return bad ? -2 : 0;
}

/* One refinement pass of an approximate kNN graph: the candidates of node i
 * are its current list plus the lists of its first J neighbours; the K
 * nearest by exact FP64 key (ties by id, i itself excluded) form the new row.
 * knn and out are n x K (may not alias). */
int orc_knn_refine(const float *base, int64_t n, int d, const uint32_t *knn, int K, int J,
                   uint32_t *out) {
    if (!base || !knn || !out || n < 2 || d < 1 || K < 1 || J < 0 || J > K) return -1;
#pragma omp parallel
    {
        uint32_t *stamp = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        cand_t *top = (cand_t *)malloc(sizeof(cand_t) * (size_t)K);
#pragma omp for schedule(dynamic, 256)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t tag = (uint32_t)i + 1u;
            int cnt = 0;
            const float *xi = base + (size_t)i * d;
            stamp[i] = tag;
            const uint32_t *row = knn + (size_t)i * K;
            for (int a = -1; a < J; ++a) {
                const uint32_t *src = a < 0 ? row : (row[a] == SENT ? NULL : knn + (size_t)row[a] * K);
                if (!src) continue;
                for (int t = 0; t < K; ++t) {
                    uint32_t v = src[t];
                    if (v == SENT || v >= (uint64_t)n || stamp[v] == tag) continue;
                    stamp[v] = tag;
                    topk_push(top, &cnt, K, key_dist(xi, base + (size_t)v * d, d, 0), v);
                }
            }
            for (int t = 0; t < K; ++t) out[(size_t)i * K + t] = t < cnt ? top[t].id : SENT;
        }
        free(stamp);
        free(top);
    }
    return 0;
}

/* ------------------------------------------------------------ SSG pruning */

/* Greedy SSG edge selection around node i (the pruning rule of Alg. 2, as
 * Alg. 3 applies it to a candidate set). cands must be sorted by (dist, id)
 * where dist is the squared distance to i. A candidate is kept when its
 * angle at i to every kept edge is at least alpha; "conflict" is
 * cos(angle) > cos(alpha), evaluated without square roots as
 *     dot > 0  and  dot^2 > cos^2(alpha) * |a|^2 * |b|^2 .
 * Selection stops after R kept edges (R <= 0: no cap). Returns the count. */
static int ssg_select(const float *base, int d, uint32_t i, const cand_t *cands, int nc,
                      double cos2a, int R, uint32_t *out) {
    const float *xi = base + (size_t)i * d;
    int kept = 0;
    /* squared lengths of kept edges, parallel to out[] */
    double *klen = (double *)malloc(sizeof(double) * (size_t)(nc > 0 ? nc : 1));
    for (int c = 0; c < nc && (R <= 0 || kept < R); ++c) {
        const float *xc = base + (size_t)cands[c].id * d;
        int conflict = 0;
        for (int k = 0; k < kept; ++k) {
            double dot = dot_rel(xc, base + (size_t)out[k] * d, xi, d);
            if (dot > 0.0 && dot * dot > cos2a * cands[c].dist * klen[k]) { conflict = 1; break; }
        }
        if (!conflict) {
            out[kept] = cands[c].id;
            klen[kept] = cands[c].dist;
            ++kept;
        }
    }
    free(klen);
    return kept;
}

/* Alg. 3, first loop: for every node i build the candidate set P from the
 * kNN graph and select out-edges with the SSG rule.
 * expand == 0: literal order -- for each kNN neighbour nb of i (ascending),
 *              add nb, then add nb's kNN list; stop as soon as |P| >= l.
 * expand == 1: all of i's kNN first, then neighbours' lists, same stop rule.
 * Candidates at distance 0 from i are dropped (the angle is undefined).
 * out: n x R, rows padded with SENT. */
int orc_nssg_prune(const float *base, int64_t n, int d, const uint32_t *knn, int Kk, int l,
                   int R, double cos2a, int expand, uint32_t *out) {
    if (!base || !knn || !out || n < 1 || d < 1 || Kk < 1 || l < 1 || R < 1) return -1;
    int err = 0;
#pragma omp parallel
    {
        uint32_t *stamp = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        int cap = l + Kk + 2;
        uint32_t *P = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)cap);
        cand_t *C = (cand_t *)malloc(sizeof(cand_t) * (size_t)cap);
        uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)R);
#pragma omp for schedule(dynamic, 256) reduction(| : err)
        for (int64_t i = 0; i < n; ++i) {
            uint32_t tag = (uint32_t)i + 1u;
            int np = 0;
            stamp[i] = tag; /* never add i itself */
            const uint32_t *row = knn + (size_t)i * Kk;
#define ADD_ID(v)                                                   \
    do {                                                            \
        uint32_t _v = (v);                                          \
        if (_v != SENT && _v < (uint32_t)n && stamp[_v] != tag) {   \
            stamp[_v] = tag;                                        \
            P[np++] = _v;                                           \
        }                                                           \
    } while (0)
            if (expand == 0) {
                for (int t = 0; t < Kk && row[t] != SENT; ++t) {
                    ADD_ID(row[t]);
                    const uint32_t *r2 = knn + (size_t)row[t] * Kk;
                    for (int t2 = 0; t2 < Kk; ++t2) ADD_ID(r2[t2]);
                    if (np >= l) break;
                }
            } else {
                for (int t = 0; t < Kk; ++t) ADD_ID(row[t]);
                if (np < l) {
                    for (int t = 0; t < Kk && row[t] != SENT; ++t) {
                        const uint32_t *r2 = knn + (size_t)row[t] * Kk;
                        for (int t2 = 0; t2 < Kk; ++t2) ADD_ID(r2[t2]);
                        if (np >= l) break;
                    }
                }
            }
#undef ADD_ID
            if (np > cap) { err = 1; np = cap; }
            int nc = 0;
            const float *xi = base + (size_t)i * d;
            for (int c = 0; c < np; ++c) {
                double dist = key_dist(xi, base + (size_t)P[c] * d, d, 0);
                if (dist == 0.0) continue;
                C[nc].dist = dist;
                C[nc].id = P[c];
                C[nc].checked = 0;
                ++nc;
            }
            qsort(C, (size_t)nc, sizeof(cand_t), cand_cmp);
            int k = ssg_select(base, d, (uint32_t)i, C, nc, cos2a, R, sel);
            for (int t = 0; t < R; ++t) out[(size_t)i * R + t] = t < k ? sel[t] : SENT;
        }
        free(stamp);
        free(P);
        free(C);
        free(sel);
    }
    return err ? -3 : 0;
}

/* Alg. 3, second loop (reverse-neighbour checking), order-independent form:
 * for every node j the candidates are its own out-edges plus every i with an
 * edge i -> j; they are sorted by distance to j and the SSG rule re-selects at
 * most R of them. */
int orc_nssg_reverse(const float *base, int64_t n, int d, const uint32_t *G1, int R,
                     double cos2a, uint32_t *out) {
    if (!base || !G1 || !out || n < 1 || d < 1 || R < 1) return -1;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < R; ++t) {
            uint32_t j = G1[(size_t)i * R + t];
            if (j == SENT) break;
            cnt[j + 1]++;
        }
    for (int64_t j = 0; j < n; ++j) cnt[j + 1] += cnt[j];
    uint32_t *rev = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(cnt[n] > 0 ? cnt[n] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)n);
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < R; ++t) {
            uint32_t j = G1[(size_t)i * R + t];
            if (j == SENT) break;
            rev[fill[j]++] = (uint32_t)i;
        }
    free(fill);
#pragma omp parallel
    {
        uint32_t *stamp = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        int64_t capn = 0;
        cand_t *C = NULL;
        uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)R);
#pragma omp for schedule(dynamic, 256)
        for (int64_t j = 0; j < n; ++j) {
            int64_t need = R + (cnt[j + 1] - cnt[j]);
            if (need > capn) {
                capn = need * 2;
                C = (cand_t *)realloc(C, sizeof(cand_t) * (size_t)capn);
            }
            uint32_t tag = (uint32_t)j + 1u;
            stamp[j] = tag;
            int nc = 0;
            const float *xj = base + (size_t)j * d;
            for (int t = 0; t < R; ++t) {
                uint32_t v = G1[(size_t)j * R + t];
                if (v == SENT) break;
                if (stamp[v] == tag) continue;
                stamp[v] = tag;
                C[nc].dist = key_dist(xj, base + (size_t)v * d, d, 0);
                C[nc].id = v;
                C[nc].checked = 0;
                ++nc;
            }
            for (int64_t e = cnt[j]; e < cnt[j + 1]; ++e) {
                uint32_t v = rev[e];
                if (stamp[v] == tag) continue;
                stamp[v] = tag;
                double dist = key_dist(xj, base + (size_t)v * d, d, 0);
                if (dist == 0.0) continue;
                C[nc].dist = dist;
                C[nc].id = v;
                C[nc].checked = 0;
                ++nc;
            }
            qsort(C, (size_t)nc, sizeof(cand_t), cand_cmp);
            int k = ssg_select(base, d, (uint32_t)j, C, nc, cos2a, R, sel);
            for (int t = 0; t < R; ++t) out[(size_t)j * R + t] = t < k ? sel[t] : SENT;
        }
        free(stamp);
        free(C);
        free(sel);
    }
    free(rev);
    free(cnt);
    return 0;
}

/* ------------------------------------------------------------ Alg. 1 search */

/* One query of Alg. 1 (Search-on-Graph) started from the given seed nodes.
 * The pool S holds at most L candidates sorted by (dist, id). A node becomes
 * visited when its distance is first computed. Each iteration expands the
 * first unchecked node of S, appends its unvisited neighbours, sorts S and
 * truncates it to L; the loop ends when S holds no unchecked node.
 * forget != 0: a node counts as visited only while it is in S (the result is
 * the same; nodes dropped from S may be computed again).
 * vis: caller-provided n-entry stamp array, tag: this query's stamp.
 * trace (optional): the id of each expanded node in expansion order, the
 * first trace_cap of them, then SENT. */
static void search_one(const float *base, int64_t n, int d, const uint32_t *graph, int R,
                       const uint32_t *seeds, int nseeds, const float *q, int K, int L,
                       int metric, int forget, uint32_t *vis, uint32_t tag, cand_t *S,
                       uint32_t *out_ids, double *out_d, int64_t *ndc_out, int64_t *hops_out,
                       uint32_t *trace, int trace_cap) {
    int64_t ndc = 0, hops = 0;
    int sz = 0;
    for (int e = 0; e < nseeds; ++e) {
        uint32_t v = seeds[e];
        S[sz].dist = key_dist(q, base + (size_t)v * d, d, metric);
        S[sz].id = v;
        S[sz].checked = 0;
        ++sz;
        ++ndc;
        if (!forget) vis[v] = tag;
    }
    qsort(S, (size_t)sz, sizeof(cand_t), cand_cmp);
    if (sz > L) sz = L;
    for (;;) {
        int i = 0;
        while (i < sz && S[i].checked) ++i;
        if (i == sz) break;
        S[i].checked = 1;
        if (trace && hops < trace_cap) trace[hops] = S[i].id;
        const uint32_t *row = graph + (size_t)S[i].id * R;
        for (int t = 0; t < R; ++t) {
            uint32_t v = row[t];
            if (v == SENT) break;
            int seen;
            if (forget) {
                seen = 0;
                for (int k = 0; k < sz; ++k)
                    if (S[k].id == v) { seen = 1; break; }
            } else {
                seen = vis[v] == tag;
                vis[v] = tag;
            }
            if (seen) continue;
            S[sz].dist = key_dist(q, base + (size_t)v * d, d, metric);
            S[sz].id = v;
            S[sz].checked = 0;
            ++sz;
            ++ndc;
        }
        qsort(S, (size_t)sz, sizeof(cand_t), cand_cmp);
        if (sz > L) sz = L;
        ++hops;
    }
    for (int t = 0; t < K; ++t) {
        out_ids[t] = t < sz ? S[t].id : SENT;
        out_d[t] = t < sz ? S[t].dist : INFINITY;
    }
    if (trace)
        for (int64_t t = hops; t < trace_cap; ++t) trace[t] = SENT;
    if (ndc_out) *ndc_out = ndc;
    if (hops_out) *hops_out = hops;
}

/* Nearest navigating node to q under the (dist, id) order. */
static uint32_t nearest_entry(const float *base, int d, const uint32_t *entry, int s,
                              const float *q, int metric) {
    double best = INFINITY;
    uint32_t bid = SENT;
    for (int e = 0; e < s; ++e) {
        double k = key_dist(q, base + (size_t)entry[e] * d, d, metric);
        if (k < best || (k == best && entry[e] < bid)) {
            best = k;
            bid = entry[e];
        }
    }
    return bid;
}

/* Thread count of the parallel loops (n < 1: leave it unchanged); returns
 * the count that later parallel regions use. Timing only. */
int orc_threads(int n) {
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
}

/* Batched Alg. 1 over nq queries. Each query starts from its nearest
 * navigating node (flags bit 1: seed every navigating node instead).
 * flags bit 0: "forget" visited mode. Per-query L_arr/K_arr override L/K when
 * given (K_arr rows still use a stride of Kmax = K). NDC counts distance
 * evaluations, including the s entry distances; hops counts expansions.
 * out_trace (optional, nq x trace_cap): each query's expanded node ids in
 * expansion order, padded with SENT. */
int orc_search(const float *base, int64_t n, int d, const uint32_t *graph, int R,
               const uint32_t *entry, int s, const float *Q, int64_t nq, int K, int L,
               const int32_t *L_arr, const int32_t *K_arr, int metric, int flags,
               uint32_t *out_ids, double *out_d, int64_t *out_ndc, int64_t *out_hops,
               uint32_t *out_trace, int trace_cap) {
    if (!base || !graph || !entry || !Q || !out_ids || !out_d) return -1;
    if (out_trace && trace_cap < 1) return -1;
    if (n < 1 || d < 1 || R < 1 || s < 1 || K < 1 || L < 1 || nq < 0) return -1;
    for (int e = 0; e < s; ++e)
        if (entry[e] >= (uint32_t)n) return -1;
    int maxL = L;
    if (L_arr)
        for (int64_t r = 0; r < nq; ++r) {
            if (L_arr[r] < 1) return -1;
            if (L_arr[r] > maxL) maxL = L_arr[r];
        }
    if (K_arr)
        for (int64_t r = 0; r < nq; ++r)
            if (K_arr[r] < 1 || K_arr[r] > K) return -1;
    int forget = flags & 1, seed_all = (flags >> 1) & 1;
#pragma omp parallel
    {
        uint32_t *vis = forget ? NULL : (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        cand_t *S = (cand_t *)malloc(sizeof(cand_t) * (size_t)(maxL + R + s + 1));
#pragma omp for schedule(dynamic, 1)
        for (int64_t r = 0; r < nq; ++r) {
            const float *q = Q + (size_t)r * d;
            int Lr = L_arr ? L_arr[r] : L;
            int Kr = K_arr ? K_arr[r] : K;
            uint32_t seed1;
            const uint32_t *seeds = entry;
            int nseeds = s;
            int64_t extra = 0;
            if (!seed_all) {
                seed1 = nearest_entry(base, d, entry, s, q, metric);
                seeds = &seed1;
                nseeds = 1;
                extra = s - 1; /* the other entry distances were computed too */
            }
            search_one(base, n, d, graph, R, seeds, nseeds, q, Kr, Lr, metric, forget, vis,
                       (uint32_t)(r + 1), S, out_ids + (size_t)r * K, out_d + (size_t)r * K,
                       out_ndc ? out_ndc + r : NULL, out_hops ? out_hops + r : NULL,
                       out_trace ? out_trace + (size_t)r * trace_cap : NULL, trace_cap);
            for (int t = Kr; t < K; ++t) {
                out_ids[(size_t)r * K + t] = SENT;
                out_d[(size_t)r * K + t] = INFINITY;
            }
            if (out_ndc) out_ndc[r] += extra;
        }
        free(vis);
        free(S);
    }
    return 0;
}

/* ------------------------------------------------------------ connectivity */

/* Alg. 3, last loop: for each navigating node (root), make every node
 * reachable from it. Iterative DFS marks what the root reaches; while a node
 * is unreached, the lowest-id unreached node u is attached by an edge w -> u
 * from the reached node w nearest to u that still has fewer than R edges.
 * w is taken from an Alg. 1 search for u from the root with pool l, and from
 * a full scan of reached nodes when that pool has no such node. The DFS then
 * continues from u. Added edges are appended to rows of graph (in place) and
 * listed in added[2*k], added[2*k+1]. Returns the number of added edges, or a
 * negative value (-4: no reached node has a free slot; -5: added overflow). */
int64_t orc_dfs_connect(const float *base, int64_t n, int d, uint32_t *graph, int R,
                        const uint32_t *roots, int s, int l, uint32_t *added, int64_t added_cap) {
    if (!base || !graph || !roots || n < 1 || d < 1 || R < 1 || s < 1 || l < 1) return -1;
    uint8_t *reached = (uint8_t *)malloc((size_t)n);
    uint32_t *stack = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
    uint32_t *vis = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
    cand_t *S = (cand_t *)malloc(sizeof(cand_t) * (size_t)(l + R + 2));
    uint32_t *pool_ids = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)l);
    double *pool_d = (double *)malloc(sizeof(double) * (size_t)l);
    int *deg = (int *)malloc(sizeof(int) * (size_t)n);
    for (int64_t i = 0; i < n; ++i) {
        int k = 0;
        while (k < R && graph[(size_t)i * R + k] != SENT) ++k;
        deg[i] = k;
    }
    int64_t nadd = 0;
    uint32_t tag = 0;
    int64_t rc = 0;
    for (int e = 0; e < s && rc == 0; ++e) {
        memset(reached, 0, (size_t)n);
        uint32_t start = roots[e];
        int64_t scan = 0;
        for (;;) {
            /* DFS from start over the current graph */
            int64_t top = 0;
            if (!reached[start]) {
                reached[start] = 1;
                stack[top++] = start;
            }
            while (top > 0) {
                uint32_t v = stack[--top];
                for (int t = 0; t < deg[v]; ++t) {
                    uint32_t w = graph[(size_t)v * R + t];
                    if (!reached[w]) {
                        reached[w] = 1;
                        stack[top++] = w;
                    }
                }
            }
            while (scan < n && reached[scan]) ++scan;
            if (scan == n) break;
            uint32_t u = (uint32_t)scan;
            const float *xu = base + (size_t)u * d;
            /* candidates: Alg. 1 from the root towards u */
            ++tag;
            if (tag == 0) {
                memset(vis, 0, sizeof(uint32_t) * (size_t)n);
                tag = 1;
            }
            uint32_t root = roots[e];
            search_one(base, n, d, graph, R, &root, 1, xu, l, l, 0, 0, vis, tag, S, pool_ids,
                       pool_d, NULL, NULL, NULL, 0);
            uint32_t w = SENT;
            for (int t = 0; t < l; ++t) {
                uint32_t c = pool_ids[t];
                if (c == SENT) break;
                if (c != u && reached[c] && deg[c] < R) { w = c; break; }
            }
            if (w == SENT) { /* full scan of reached nodes */
                double best = INFINITY;
                for (int64_t c = 0; c < n; ++c) {
                    if (!reached[c] || deg[c] >= R || (uint32_t)c == u) continue;
                    double dc = key_dist(xu, base + (size_t)c * d, d, 0);
                    if (dc < best) { best = dc; w = (uint32_t)c; }
                }
            }
            if (w == SENT) { rc = -4; break; }
            if (nadd >= added_cap) { rc = -5; break; }
            graph[(size_t)w * R + deg[w]] = u;
            deg[w]++;
            added[2 * nadd] = w;
            added[2 * nadd + 1] = u;
            ++nadd;
            start = u;
        }
    }
    free(reached);
    free(stack);
    free(vis);
    free(S);
    free(pool_ids);
    free(pool_d);
    free(deg);
    return rc ? rc : nadd;
}

/* ------------------------------------------------------------ Alg. 2 */

/* Exact SSG over all pairs (Alg. 2): for every node, all other nodes sorted by
 * (dist, id), then the greedy angular selection without a degree cap.
 * Zero-distance duplicates are skipped. out: n x cap, padded with SENT;
 * deg[i] is the full out-degree (returns -2 if some degree exceeds cap). */
int orc_ssg_exact(const float *base, int64_t n, int d, double cos2a, int cap, uint32_t *out,
                  int32_t *deg) {
    if (!base || !out || !deg || n < 2 || d < 1 || cap < 1) return -1;
    int over = 0;
#pragma omp parallel
    {
        cand_t *C = (cand_t *)malloc(sizeof(cand_t) * (size_t)n);
        uint32_t *sel = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)n);
#pragma omp for schedule(dynamic, 4) reduction(| : over)
        for (int64_t i = 0; i < n; ++i) {
            int nc = 0;
            const float *xi = base + (size_t)i * d;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                double dist = key_dist(xi, base + (size_t)j * d, d, 0);
                if (dist == 0.0) continue;
                C[nc].dist = dist;
                C[nc].id = (uint32_t)j;
                C[nc].checked = 0;
                ++nc;
            }
            qsort(C, (size_t)nc, sizeof(cand_t), cand_cmp);
            int k = ssg_select(base, d, (uint32_t)i, C, nc, cos2a, 0, sel);
            deg[i] = k;
            if (k > cap) over = 1;
            for (int t = 0; t < cap; ++t) out[(size_t)i * cap + t] = t < k ? sel[t] : SENT;
        }
        free(C);
        free(sel);
    }
    return over ? -2 : 0;
}

/* Exact FP64 keys of explicit (query, id) pairs; used to explain ties. */
int orc_pair_keys(const float *base, int64_t n, int d, const float *Q, int64_t nq,
                  const uint32_t *ids, int K, int metric, double *out) {
    if (!base || !Q || !ids || !out || d < 1 || K < 1) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < nq; ++r)
        for (int t = 0; t < K; ++t) {
            uint32_t v = ids[(size_t)r * K + t];
            out[(size_t)r * K + t] =
                (v == SENT || v >= (uint64_t)n) ? INFINITY
                                                : key_dist(Q + (size_t)r * d, base + (size_t)v * d, d, metric);
        }
    return 0;
}
