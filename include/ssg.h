/*
 * ssg.h -- C ABI of libssg, batched graph search on AMD Instinct MI355X
 * (gfx950) for the Satellite System Graph method (Fu, Wang, Cai,
 * arXiv 1907.06146).
 *
 * The library runs the paper's search (Alg. 1, "Search-on-Graph") over a
 * fixed-width navigating-SSG graph, starting every query from the navigating
 * node nearest to it (Sec. 4.1, last paragraph), for many queries at once.
 * The problem statement is k-nearest-neighbour search over a base set S with
 * Euclidean distance (Sec. 2.1, 2.2); the index is the n x m neighbour matrix
 * the paper stores graphs in (Sec. 6.2).
 *
 * Conventions for every entry point:
 *  - Array pointers documented as DEVICE point to memory on the current HIP
 *    device, allocated and owned by the caller. The library never frees,
 *    reallocates or retains them after the call returns.
 *  - Calls are asynchronous: they validate the arguments on the host, enqueue
 *    kernels on `stream` (a hipStream_t; NULL = the default stream) and
 *    return. The caller synchronises (e.g. through torch).
 *  - Argument errors are reported synchronously with a negative status and no
 *    work enqueued. A launch failure returns SSG_EDEVICE. The message of the
 *    last failing call on the calling thread is returned by ssg_last_error().
 *  - No C++ exception crosses the ABI. The library keeps no mutable global
 *    state except the thread-local error string and, for
 *    ssg_search_batched_noalloc, one counter array per device (and its
 *    looked-up address); every other entry point is reentrant.
 *  - Distances are returned as squared Euclidean distance (same order as the
 *    Euclidean distance of the paper's notation) or, for SSG_IP, as the
 *    negative inner product. Results are sorted ascending by (dist, id).
 */
#ifndef SSG_H_
#define SSG_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSG_OK = 0,
    SSG_EINVAL = -1,       /* bad argument (null pointer, size out of range) */
    SSG_ENOMEM = -2,       /* workspace too small */
    SSG_EDEVICE = -3,      /* HIP launch / runtime error */
    SSG_EUNSUPPORTED = -4  /* valid but not supported (L > SSG_L_MAX, dims, dtype) */
} ssg_status;

typedef enum { SSG_L2 = 0, SSG_IP = 1 } ssg_metric;

typedef enum {
    SSG_F32 = 0,     /* IEEE binary32 vectors */
    SSG_BF16 = 1,    /* bfloat16 vectors, FP32 accumulation */
    SSG_FP8E4M3 = 2  /* OCP FP8 E4M3 codes times a per-dimension FP32 scale */
} ssg_dtype;

#define SSG_SENTINEL 0xFFFFFFFFu /* padding id in graph rows and in results */
#define SSG_L_MAX 512            /* largest supported pool size */
#define SSG_R_MAX 64             /* largest supported graph row width */
#define SSG_K_MAX 4096           /* largest supported result count */

/* Search options (ssg_search_ex). Zero-initialise, then set what you need. */
typedef struct {
    int32_t exact_visited;    /* 1: visited set is an exact n-bit LDS bitset
                                 (requires n <= SSG_EXACT_VISITED_MAX_N); the
                                 distance count then equals Alg. 1's exactly */
    int32_t hash_log2;        /* log2 of the LDS visited-set entry count; 0 = default */
    int32_t waves_per_block;  /* wavefronts (queries) per workgroup; 0 = default */
    int32_t* out_ndc;         /* DEVICE int32[nq] distance computations, or NULL */
    int32_t* out_hops;        /* DEVICE int32[nq] expansions, or NULL */
    int32_t gather_variant;   /* alternative gather shape (tuning); 0 = default */
    const float* base_f32;    /* DEVICE n x d FP32 vectors: when set, the first
                                 rerank_k pool entries are re-scored exactly in
                                 FP32 against them and re-sorted before the K
                                 results are written (precision form: search on
                                 BF16/FP8, rerank in FP32); NULL = no rerank */
    int32_t rerank_k;         /* pool entries to rerank: max(rerank_k, K) capped
                                 at L (0 = K), so every returned entry has been
                                 re-scored */
    int64_t entry_group_size; /* > 0: queries form consecutive groups of this
                                 many, and group g starts from the n_entry ids
                                 entry_ids[g * n_entry ...] (entry_ids then
                                 holds ceil(nq / size) sets); used to search
                                 several shards' graphs, stored as one
                                 block-diagonal graph, in one launch;
                                 0 = every query uses the same n_entry ids */
    int32_t visited_kind;     /* form of the visited set when exact_visited is 0:
                                 0 = default (the tag cache when a 16-bit tag
                                 holds the ids, else the hash); 1 = hash of full
                                 ids, cleared and refilled from the pool when
                                 half full; 2 = 4-way tag cache (SSG_EUNSUPPORTED
                                 when the ids do not fit). Either form may forget
                                 ids, which costs recomputed distances but never
                                 changes the results. */
    uint32_t* out_trace;      /* DEVICE uint32 nq x trace_cap, or NULL: the ids of
                                 the first trace_cap expanded nodes of each query
                                 in expansion order (Alg. 1 takes the first
                                 unchecked pool entry each step), then
                                 SSG_SENTINEL; a debugging record that locates
                                 where two runs' trajectories part */
    int32_t trace_cap;        /* entries per trace row (>= 1 with out_trace) */
    int32_t queries_per_wave; /* searches sharing one 64-lane wavefront: 1 (64
                                 lanes per query), 2 (32 lanes each; needs
                                 L <= 256, the tag-cache visited set and a
                                 compiled dimension: 96 or 128), or 0 = the
                                 library's choice. Results are the same. */
} ssg_search_opts;

#define SSG_EXACT_VISITED_MAX_N 262144

/*
 * ssg_search -- Alg. 1 for nq queries, each from its nearest navigating node.
 *
 *   base       DEVICE, n x d row-major vectors of `dtype` (16-byte aligned).
 *              SSG_F32: float; SSG_BF16: uint16 bfloat16 bits;
 *              SSG_FP8E4M3: uint8 codes, value = decode(code) * dim_scale[j].
 *   n          number of base vectors, 1 <= n < 2^31.
 *   d          dimension; d % 4 == 0 (F32), d % 8 == 0 (BF16), d % 16 == 0 (FP8).
 *   dim_scale  DEVICE float[d] for SSG_FP8E4M3, else NULL.
 *   graph      DEVICE uint32 n x R; row i lists the out-neighbours of node i,
 *              then SSG_SENTINEL padding. Ids < n, no duplicates in a row.
 *   R          row width, 1 <= R <= SSG_R_MAX.
 *   entry_ids  DEVICE uint32[n_entry] navigating nodes (ids < n), 1..4096.
 *   queries    DEVICE float nq x d row-major (FP32 whatever `dtype` is).
 *   K, L       results per query (1..SSG_K_MAX) and pool size (1..SSG_L_MAX).
 *              K > L is allowed: slots past the final pool are padded.
 *   out_ids    DEVICE uint32 nq x K; out_dists DEVICE float nq x K. Row q holds
 *              the first min(K, |S|) entries of the final pool S of query q,
 *              then SSG_SENTINEL / +inf.
 *              With nq == 0 nothing is enqueued and queries / outputs may be NULL.
 *   workspace  unused by this entry point (may be NULL / 0).
 *   stream     hipStream_t to enqueue on.
 * Returns SSG_OK or a negative ssg_status.
 */
int ssg_search(const void* base, int64_t n, int32_t d, int32_t dtype, const float* dim_scale,
               const uint32_t* graph, int32_t R, const uint32_t* entry_ids, int32_t n_entry,
               const float* queries, int64_t nq, int32_t K, int32_t L, int32_t metric,
               uint32_t* out_ids, float* out_dists, void* workspace, size_t workspace_bytes,
               void* stream);

/* ssg_search with options (statistics, exact visited set, launch shape). */
int ssg_search_ex(const void* base, int64_t n, int32_t d, int32_t dtype, const float* dim_scale,
                  const uint32_t* graph, int32_t R, const uint32_t* entry_ids, int32_t n_entry,
                  const float* queries, int64_t nq, int32_t K, int32_t L, int32_t metric,
                  uint32_t* out_ids, float* out_dists, const ssg_search_opts* opts,
                  void* stream);

/*
 * ssg_quantize -- build a reduced-precision copy of the base vectors for the
 * precision form of the search (storage format only; not from the paper,
 * which computes exact distances on full-precision vectors, Sec. 6.1).
 *   base_f32   DEVICE float n x d.
 *   dtype      SSG_BF16: out is uint16 n x d, round-to-nearest-even bfloat16.
 *              SSG_FP8E4M3: dim_scale (DEVICE float[d], written) receives
 *              s_j = max_i |x_ij| / 448 (1 for an all-zero column) and out is
 *              uint8 n x d holding OCP E4M3 codes of x_ij / s_j, rounded to
 *              nearest even and saturated at +-448.
 * Asynchronous on `stream`; returns SSG_OK or SSG_EINVAL / SSG_EDEVICE.
 */
int ssg_quantize(const float* base_f32, int64_t n, int32_t d, int32_t dtype, float* dim_scale,
                 void* out, void* stream);

/* ------------------------------------------------------------------ batched
 * Mixed-workload form: queries with their own pool size L_i and result count
 * K_i, split into buckets of similar L (each bucket sizes its on-chip pool for
 * its largest L). Each bucket runs as a persistent kernel whose wavefronts
 * take query slots from a device work queue until it is exhausted, so long
 * and short searches balance across the GPU. Not from the paper, whose
 * search is one query per CPU thread; every query computes exactly Alg. 1
 * with its own L_i and K_i.
 */
typedef struct {
    const void* base;          /* DEVICE n x d, as in ssg_search */
    int64_t n;
    int32_t d, dtype, metric;
    const float* dim_scale;    /* DEVICE float[d] for FP8, else NULL */
    const float* base_f32;     /* DEVICE FP32 vectors for the rerank, or NULL */
    int32_t rerank;            /* 0: none; -m (1 <= m <= 16): rerank the first
                                  m * K_i entries of each query; > 0:
                                  max(rerank, K_i) entries (capped at L_i);
                                  below -16: SSG_EINVAL */
    const uint32_t* graph;     /* DEVICE n x R */
    int32_t R;
    const uint32_t* entry_ids; /* DEVICE [n_entry] */
    int32_t n_entry;
    const float* queries;      /* DEVICE nq x d FP32 */
    int64_t nq;
    const int32_t* L;          /* DEVICE int32[nq], each 1..SSG_L_MAX */
    const int32_t* K;          /* DEVICE int32[nq], each 1..kstride */
    int32_t kstride;           /* output row stride (>= every K_i, <= SSG_K_MAX) */
    uint32_t* out_ids;         /* DEVICE nq x kstride; row i: K_i results, then
                                  SSG_SENTINEL padding */
    float* out_dists;          /* DEVICE nq x kstride (+inf padding) */
    int32_t* out_ndc;          /* DEVICE int32[nq] or NULL */
    int32_t* out_hops;         /* DEVICE int32[nq] or NULL */
    uint32_t* out_trace;       /* DEVICE nq x trace_cap expansion record, as in
                                  ssg_search_opts, or NULL */
    int32_t trace_cap;
} ssg_batch_desc;

typedef struct {
    const int32_t* qlist;      /* DEVICE int32[count]: query indices of this bucket
                                  (processed in this order: put long searches first) */
    int64_t count;
    int32_t max_L;             /* >= every L_i of the bucket; sizes the pool */
    int32_t gather_variant;    /* launch shape (see ssg_search_opts); 0 = default */
    int32_t hash_log2;         /* 0 = default */
    int32_t waves_per_block;   /* 0 = default */
    int32_t blocks;            /* 0: one wavefront per listed query (the
                                  hardware starts the next query as a
                                  search ends); > 0: a persistent grid of
                                  that many workgroups taking queries from
                                  the bucket's work-queue counter (two
                                  queries per wavefront always run
                                  persistent, filling the GPU once) */
    int32_t visited_kind;      /* visited-set form, as ssg_search_opts.visited_kind
                                  (0 default, 1 hash, 2 tag cache) */
    int32_t queries_per_wave;  /* as ssg_search_opts.queries_per_wave (bucket
                                  max_L <= 256 for 2) */
} ssg_bucket;

/* Workspace for nb buckets (one work-queue counter each). */
size_t ssg_batch_workspace_bytes(int32_t nb);

/* Enqueue every bucket on `stream`, one after another (counters are reset by
 * a kernel first). The caller must not free the descriptor's arrays before
 * the work completes; the descriptor structs themselves may be freed on
 * return. Returns SSG_OK or a negative status. */
int ssg_search_batched(const ssg_batch_desc* desc, const ssg_bucket* buckets, int32_t nb,
                       void* workspace, size_t workspace_bytes, void* stream);

/*
 * ssg_search_batched_noalloc -- ssg_search_batched for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * hosts that forbid allocation): the work-queue counters live in a fixed
 * array inside the library (SSG_NOALLOC_SCRATCH_BYTES, one 256-byte slot per
 * bucket), so no workspace is passed and nothing is allocated.
 *   desc, buckets, nb, stream  as in ssg_search_batched; nb <= 64, else
 *                              SSG_EINVAL
 * Every call on one device shares that device's array: calls that overlap
 * on one device (other streams, other threads) race and must be serialised
 * by the caller. The counters are reset by a kernel at the start of each
 * bucket, so nothing carries over from the previous call. The array's
 * address is looked up on each device's first call (hipGetSymbolAddress);
 * each device keeps its copy until the process ends.
 */
#define SSG_NOALLOC_SCRATCH_BYTES 16384
int ssg_search_batched_noalloc(const ssg_batch_desc* desc, const ssg_bucket* buckets, int32_t nb,
                               void* stream);

/* A captured HIP graph of the same work with the buckets on parallel graph
 * branches, replayed by ssg_batch_graph_launch as one launch. The device
 * arrays named by the descriptor are baked into the graph: keep them alive
 * and in place until ssg_batch_graph_destroy; their contents may change
 * between launches. */
typedef struct ssg_batch_graph ssg_batch_graph;
int ssg_batch_graph_create(ssg_batch_graph** out, const ssg_batch_desc* desc,
                           const ssg_bucket* buckets, int32_t nb, void* workspace,
                           size_t workspace_bytes);
int ssg_batch_graph_launch(ssg_batch_graph* g, void* stream);
int ssg_batch_graph_destroy(ssg_batch_graph* g);

/*
 * ssg_probe_gather -- measurement aid (not part of the method): reads the rows
 * base[ids[i]] (row_bytes each) in the search kernel's access shape and
 * writes one checksum word per wavefront, so the random-row gather rate of the
 * device can be measured on its own.
 *   base  DEVICE, n rows of row_bytes (a positive multiple of 16), 16-byte aligned
 *   ids   DEVICE uint32[m], each < n (not checked on the device)
 *   out   DEVICE uint32[ceil(m / rows_per_wave)]
 */
int ssg_probe_gather(const void* base, int64_t n, int32_t row_bytes, const uint32_t* ids,
                     int64_t m, int32_t rows_per_wave, uint32_t* out, void* stream);

/*
 * ssg_knn_graph -- exact K-nearest-neighbour graph by brute force: the kNN
 * graph the indexing algorithm starts from (Alg. 3; the paper builds it
 * approximately, this builds it exactly), on the device's matrix cores.
 *   base        DEVICE float32 n x d row-major (16-byte aligned rows give
 *               vector loads), finite values
 *   n, d        2 <= n <= 2^25, d >= 1
 *   K           1 <= K <= min(100, n - 1)
 *   out_ids     DEVICE uint32 n x K: row i lists the K points nearest to
 *               point i, itself excluded, in ascending (squared Euclidean
 *               distance, id) order; the distance is the FP64 sum of
 *               (x_ij - x_kj)^2 over the dimensions in order
 *   out_dists   DEVICE float32 n x K: those distances rounded to float32
 *   workspace   DEVICE, 256-byte aligned, ssg_knn_workspace_bytes(n, d, K)
 *               bytes, owned by the caller, contents on entry ignored
 *   stats       HOST int64[4] or NULL: [0] 1 if the exact integer path ran
 *               (all values integers in [0, 255] and d <= 128), [1] rows
 *               whose certificate failed and were rescanned in FP64,
 *               [2] candidates kept per row, [3] reserved
 *   stream      hipStream_t (NULL: the legacy default stream)
 * Synchronous: the call waits on its stream (it reads two flag words back).
 * Returns SSG_OK; SSG_EINVAL for bad arguments; SSG_EDEVICE on a launch or
 * device error; SSG_EUNSUPPORTED if more than 4096 points tie at or below
 * some row's K-th distance, or if more than 1024 rows fail the certificate
 * and their FP64 rescans would evaluate more than 2^36 pairs.
 */
size_t ssg_knn_workspace_bytes(int64_t n, int32_t d, int32_t K);
int ssg_knn_graph(const float* base, int64_t n, int32_t d, int32_t K, uint32_t* out_ids,
                  float* out_dists, void* workspace, size_t workspace_bytes, int64_t* stats,
                  void* stream);

/*
 * ssg_nssg_prune -- first loop of the indexing algorithm (Alg. 3): for every
 * node i, candidates from the kNN graph and the SSG angular rule over them.
 * Candidates: for each kNN neighbour u of i in ascending order, u and then
 * u's whole kNN list (i and repeats skipped), stopping once at least l are
 * held; candidates at distance 0 from i are dropped. They are taken in
 * ascending (squared distance, id) order and one is kept unless a kept edge k
 * has <c - i, k - i> > 0 and <c - i, k - i>^2 > cos2a |c - i|^2 |k - i|^2
 * (Sec. 3.2's angle test, FP64, every operation rounded on its own).
 *   base    DEVICE float32 n x d
 *   knn     DEVICE uint32 n x Kk, rows ascending, padding SSG_SENTINEL
 *   l, R    candidate target (l + Kk + 2 <= 1024) and out-degree (R <= 64)
 *   cos2a   cos^2 of the minimum angle (0.25 for 60 degrees)
 *   out     DEVICE uint32 n x R: kept ids in selection order, then padding
 * Asynchronous on stream. SSG_EINVAL / SSG_EUNSUPPORTED for bad arguments.
 */
int ssg_nssg_prune(const float* base, int64_t n, int32_t d, const uint32_t* knn, int32_t Kk,
                   int32_t l, int32_t R, double cos2a, uint32_t* out, void* stream);

/*
 * ssg_nssg_reverse -- second loop of Alg. 3 (reverse-neighbour checking),
 * order-independent: node j re-selects, by the rule of ssg_nssg_prune, from
 * its own out-edges (in order) plus every i with an edge i -> j that is not
 * already one of them and is not at distance 0.
 *   g1         DEVICE uint32 n x R from ssg_nssg_prune (ids, then padding)
 *   out        DEVICE uint32 n x R (distinct from g1)
 *   workspace  DEVICE, 256-byte aligned, ssg_nssg_reverse_workspace_bytes(n, R)
 * Asynchronous on stream.
 */
size_t ssg_nssg_reverse_workspace_bytes(int64_t n, int32_t R);
int ssg_nssg_reverse(const float* base, int64_t n, int32_t d, const uint32_t* g1, int32_t R,
                     double cos2a, uint32_t* out, void* workspace, size_t workspace_bytes,
                     void* stream);

/*
 * ssg_merge_shards -- aggregation step of the partitioned search (Sec. 6.5:
 * the data set split at random into S shards, one graph per shard, every
 * query searched in all of them): merges each query's S result lists into
 * the first K_out by (distance, global id).
 *   ids, dists  DEVICE [S][nq][K] per-shard results (shard-local ids,
 *               SSG_SENTINEL / +inf padding), e.g. S ssg_search outputs
 *               written into consecutive slices
 *   id_map      DEVICE uint32[map_len]: shard s's local id l is
 *               id_map[map_off[s] + l]; a local id whose index falls outside
 *               [0, map_len) is treated as padding
 *   map_off     DEVICE int64[S]
 *   out_ids, out_dists  DEVICE [nq][K_out]; padding where fewer than K_out
 *               real results exist
 * Requires S * K <= 4096 and K_out <= S * K. Asynchronous on stream.
 */
int ssg_merge_shards(const uint32_t* ids, const float* dists, int32_t S, int64_t nq, int32_t K,
                     const uint32_t* id_map, const int64_t* map_off, int64_t map_len,
                     int32_t K_out, uint32_t* out_ids, float* out_dists, void* stream);

/*
 * ssg_exact_ssg -- the exact satellite system graph (Alg. 2): for every node
 * i, all other points in ascending (squared distance, id) order (distance 0
 * dropped), each kept unless a kept edge makes an angle below alpha with it
 * (the rule of ssg_nssg_prune, FP64), with no degree bound.
 *   base       DEVICE float32 n x d, 2 <= n <= 2^20 (cost grows as n^2)
 *   cos2a      cos^2 of the minimum angle
 *   out        DEVICE uint32 n x cap: the first cap kept ids in selection
 *              order (the graph truncated at cap), then padding
 *   deg        DEVICE int32[n]: the untruncated out-degree
 *   workspace  DEVICE, 256-byte aligned, ssg_exact_ssg_workspace_bytes(n)
 * Asynchronous on stream.
 */
size_t ssg_exact_ssg_workspace_bytes(int64_t n);
int ssg_exact_ssg(const float* base, int64_t n, int32_t d, double cos2a, int32_t cap, uint32_t* out,
                  int32_t* deg, void* workspace, size_t workspace_bytes, void* stream);

/*
 * ssg_query_lds_bytes -- on-chip (LDS) bytes one search of pool size L holds
 * while it runs, in the default launch shape of the batched form (the pool
 * capacity of L's bucket, the visited set of hash_log2 (0 = default), the
 * merge stage and, with rerank != 0, room for the rerank keys). Host only, no
 * device work; returns 0 for arguments the search would reject. Serving uses
 * it to admit queries against the device's LDS budget.
 */
size_t ssg_query_lds_bytes(int32_t L, int32_t R, int32_t d, int32_t dtype, int64_t n, int32_t rerank,
                           int32_t hash_log2);

/* Workspace bytes ssg_search needs (0: it keeps all search state on chip). */
size_t ssg_search_workspace_bytes(int64_t n, int64_t nq, int32_t L, int32_t R, int32_t dtype);

/*
 * ssg_validate_graph -- host-side check of a graph's preconditions.
 *   graph_host  HOST uint32 n x R.
 * Checks: ids < n, each row is ids then SSG_SENTINEL only, no duplicate ids in
 * a row, no self loops. Returns SSG_OK, or SSG_EINVAL with the first offending
 * row named in ssg_last_error().
 */
int ssg_validate_graph(const uint32_t* graph_host, int64_t n, int32_t R);

/* Message of the last failing call on this thread ("" if none). The pointer
 * stays valid until the next call on the same thread. */
const char* ssg_last_error(void);

/* Library version string. */
const char* ssg_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SSG_H_ */
