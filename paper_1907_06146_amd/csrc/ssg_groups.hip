// ssg_groups.hip -- the batched search of Alg. 1 (from the navigating node
// nearest each query, Sec. 4.1) with several queries per wavefront.
//
// A group of S = 32 (or 16) lanes owns one query, so a wavefront runs
// Q = 64 / S searches side by side. Every step of ssg_search.hip's search
// happens per group: the pool of at most L keys lives in the group's lanes
// (entry i in lane i % S, register i / S), ballots and DPP reductions are
// read per group, and each group has its own LDS region (merge stage, the
// batch of new candidates, the visited cache). One wavefront instruction
// thus serves Q queries, which matters because a search step is a chain of
// short dependent steps over at most R = 64 neighbour ids: with one query
// per wavefront most lanes of the ballot, visited-set and merge steps idle.
//
// Control flow is uniform over the wavefront: a group that has finished its
// search keeps executing with empty batches (its lanes do no stores), and
// every loop runs while any group has work, so ballots and lane reads never
// run under divergent execution.
//
// Visited set: the 4-way tag cache of ssg_search.hip (16-bit tags of a
// bijective image of the id). Inserts use a 64-bit LDS compare-and-swap on
// the whole set, so lanes that insert into one set in the same step cannot
// overwrite each other; an id is only forgotten when a full set evicts a
// way. Forgetting a node outside the pool is harmless (its key exceeded the
// L-th key, which never grows again, so a recomputed copy is cut at once);
// forgetting a pool member could let it return with its pool key. So the
// per-key duplicate check against the pool runs only in groups whose cache
// has evicted a way at least once in the current search.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "ssg.h"
#include "ssg_internal.h"
#include "ssg_search_common.h"

namespace {

// Broadcast of a 64-bit value from lane gbase + j of each group (j uniform
// within the group) to the whole group.
template <int S>
__device__ __forceinline__ uint64_t gread64(uint64_t v, int j, int gbase) {
  if constexpr (S == 64) {
    return readlane64(v, __builtin_amdgcn_readfirstlane(j));
  } else if constexpr (S == 32) {
    const int j0 = __builtin_amdgcn_readlane(j, 0);
    const int j1 = __builtin_amdgcn_readlane(j, 32);
    const uint64_t v0 = readlane64(v, j0);
    const uint64_t v1 = readlane64(v, 32 + j1);
    return gbase ? v1 : v0;
  } else {
    const int src = (gbase + j) << 2;  // ds_bpermute addresses lanes in bytes
    const uint32_t lo = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_ds_bpermute(src, (int)(uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
  }
}
template <int S>
__device__ __forceinline__ uint32_t gread32(uint32_t v, int j, int gbase) {
  if constexpr (S == 64) {
    return __builtin_amdgcn_readlane(v, __builtin_amdgcn_readfirstlane(j));
  } else if constexpr (S == 32) {
    const int j0 = __builtin_amdgcn_readlane(j, 0);
    const int j1 = __builtin_amdgcn_readlane(j, 32);
    const uint32_t v0 = __builtin_amdgcn_readlane(v, j0);
    const uint32_t v1 = __builtin_amdgcn_readlane(v, 32 + j1);
    return gbase ? v1 : v0;
  } else {
    return __builtin_amdgcn_ds_bpermute((gbase + j) << 2, (int)v);
  }
}

// Minimum of a 64-bit value over each group, on every lane of the group:
// row DPP shifts reduce each row of 16 into its lane 15; for S >= 32 a row
// broadcast folds row pairs (lane 31 holds rows 0-1, lane 63 rows 2-3).
template <int S>
__device__ __forceinline__ uint64_t gmin64(uint64_t v, int gbase) {
  v = dpp_min64<0x111>(v);
  v = dpp_min64<0x112>(v);
  v = dpp_min64<0x114>(v);
  v = dpp_min64<0x118>(v);
  if constexpr (S >= 32) v = dpp_min64<0x142>(v);  // row_bcast:15
  if constexpr (S == 64) {
    v = dpp_min64<0x143>(v);  // row_bcast:31
    return readlane64(v, 63);
  } else {
    return gread64<S>(v, S - 1, gbase);
  }
}

// The bits of a wavefront ballot that belong to this lane's group, shifted
// down to bit 0.
template <int S>
__device__ __forceinline__ uint64_t gbits(uint64_t ballot, int gbase) {
  if constexpr (S == 64) return ballot;
  else return (ballot >> gbase) & ((1ull << S) - 1ull);
}

constexpr uint32_t kMul = 0x9E3779B1u;  // odd: multiplication mod 2^k is a bijection

// ------------------------------------------------------------------ kernel
// T, DC, G, NP as in ssg_search.hip (DC compiled, the query in registers);
// PREG: pool registers per lane (pool capacity S * PREG); S: lanes per query.
// a.lds_per_wave holds the bytes of ONE group's region here.
template <typename T, int DC, int G, int NP, int PREG, int S>
__device__ __forceinline__ void run_groups(const Args& a, unsigned char* wave_lds, const int lane,
                                           const int64_t qid, const int L, const int K) {
  static_assert(S == 16 || S == 32 || S == 64, "lanes per query");
  static_assert(DC > 0 && S % G == 0, "compiled chunk count, whole candidate groups");
  constexpr int EPC = T::kEpc;
  constexpr int CPP = S / G;                 // candidates per pass per group
  constexpr int NCH = (DC + G - 1) / G;      // chunks per lane
  constexpr int LCAP = S * PREG;
  constexpr int NRL = 64 / S;                // row slots per lane (rows hold <= 64 ids)
  constexpr bool kScaled = T::kScaled;
  constexpr bool kPipe = NP * NCH <= 8;      // the staged pass stays in registers
  const int gl = lane % S;
  const int gbase = lane - gl;
  const uint64_t gmask = S == 64 ? ~0ull : (((1ull << S) - 1ull) << gbase);
  const bool live = qid >= 0;

  unsigned char* my = wave_lds + (size_t)(lane / S) * a.lds_per_wave;
  uint64_t* stage = reinterpret_cast<uint64_t*>(my);
  uint64_t* bkeys = stage + LCAP;
  uint32_t* bids = reinterpret_cast<uint32_t*>(bkeys + 64);
  uint32_t* table = bids + 64;

  const int g = gl % G;
  const int sub = gl / G;
  const float* q = a.queries + (size_t)(live ? qid : 0) * a.d;
  const bool ip = a.metric == 1;
  const int R = a.R;

  // query (and fp8 scale) fragment: lane g holds chunks g, g+G, ...
  float qf[NCH * EPC];
  float sf[kScaled ? NCH * EPC : 1];
#pragma unroll
  for (int t = 0; t < NCH; ++t) {
    const int ch = g + G * t;
    const bool ok = DC % G == 0 || ch < DC;
#pragma unroll
    for (int e = 0; e < EPC; e += 4) {
      const float4 v = ok ? *reinterpret_cast<const float4*>(q + ch * EPC + e) : make_float4(0, 0, 0, 0);
      qf[t * EPC + e] = v.x;
      qf[t * EPC + e + 1] = v.y;
      qf[t * EPC + e + 2] = v.z;
      qf[t * EPC + e + 3] = v.w;
      if constexpr (kScaled) {
        const float4 w = ok ? *reinterpret_cast<const float4*>(a.dim_scale + ch * EPC + e)
                            : make_float4(0, 0, 0, 0);
        sf[t * EPC + e] = w.x;
        sf[t * EPC + e + 1] = w.y;
        sf[t * EPC + e + 2] = w.z;
        sf[t * EPC + e + 3] = w.w;
      }
    }
  }

  // visited cache: 4 ways of 16-bit tags per 64-bit set word
  const uint32_t hmask = (1u << a.hash_log2) - 1u;
  const int twords = (int)((hmask + 1u) >> 1);
  for (int i = gl; i < twords; i += S) table[i] = 0u;
  const int tshift = a.id_bits - (a.hash_log2 - 2);
  const uint32_t kmask = (uint32_t)((1ull << a.id_bits) - 1u);
  bool evicted = false;  // this group's cache has dropped a tag in this search
  wave_sync();

  // test-and-insert; returns true when the id was not yet visited
  auto visit = [&](uint32_t id, bool& ev) -> bool {
    const uint32_t h = (id * kMul) & kmask;
    const uint32_t set = h >> tshift;
    const uint64_t tag = (h & ((1u << tshift) - 1u)) + 1u;
    unsigned long long* word = reinterpret_cast<unsigned long long*>(table) + set;
    unsigned long long w = *word;
    for (;;) {
      const uint64_t t0 = w & 0xFFFFu, t1 = (w >> 16) & 0xFFFFu, t2 = (w >> 32) & 0xFFFFu, t3 = w >> 48;
      if (t0 == tag || t1 == tag || t2 == tag || t3 == tag) return false;
      const int way = t0 == 0u ? 0 : t1 == 0u ? 1 : t2 == 0u ? 2 : t3 == 0u ? 3 : (int)((tag ^ (tag >> 2)) & 3u);
      const uint64_t old_tag = (w >> (16 * way)) & 0xFFFFu;
      const unsigned long long nw = (w & ~(0xFFFFull << (16 * way))) | (tag << (16 * way));
      const unsigned long long seen = atomicCAS(word, w, nw);
      if (seen == w) {
        ev |= old_tag != 0u;
        return true;
      }
      w = seen;  // another lane changed the set: look again
    }
  };

  // one distance term; the fp8 value is code * scale rounded to fp32 first
  struct Pass {
    uint4 buf[NP][NCH];
    uint32_t idp[NP];
    bool vp[NP];
  };
  auto issue = [&](Pass& ps, int c0, int m) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int c = c0 + p * CPP + sub;
      ps.vp[p] = c < m;
      ps.idp[p] = ps.vp[p] ? bids[c] : 0u;
    }
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const uint4* vec = reinterpret_cast<const uint4*>(a.base + (size_t)ps.idp[p] * a.dc * 16);
#pragma unroll
      for (int t = 0; t < NCH; ++t) {
        const int ch = g + G * t;
        if (DC % G == 0 || ch < DC) ps.buf[p][t] = vec[ch];
        else ps.buf[p][t] = make_uint4(0, 0, 0, 0);
      }
    }
  };
  auto finish = [&](Pass& ps, int c0) {
    float acc[NP];
#pragma unroll
    for (int p = 0; p < NP; ++p) acc[p] = 0.f;
    auto accumulate = [&](auto ip_c) {
      constexpr bool IP = decltype(ip_c)::value;
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
          const int ch = g + G * t;
          if (DC % G == 0 || ch < DC) {
            float x[EPC];
            T::decode(ps.buf[p][t], x);
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
              const float xv = kScaled ? __fmul_rn(x[e], sf[t * EPC + e]) : x[e];
              if constexpr (IP) {
                acc[p] = fmaf(qf[t * EPC + e], xv, acc[p]);
              } else {
                const float df = qf[t * EPC + e] - xv;
                acc[p] = fmaf(df, df, acc[p]);
              }
            }
          }
        }
      }
    };
    if (ip) accumulate(std::true_type{});
    else accumulate(std::false_type{});
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      acc[p] = group_sum<G>(acc[p], lane);
      if (ps.vp[p] && g == 0) bkeys[c0 + p * CPP + sub] = make_key(ip ? -acc[p] : acc[p], ps.idp[p]);
    }
  };
  // keys of bids[first * CPP * NP .. m) of every group
  auto batch_keys = [&](int m, int first) {
    for (int c0 = first * CPP * NP; __any(c0 < m); c0 += CPP * NP) {
      Pass ps;
      issue(ps, c0, m);
      finish(ps, c0);
    }
    wave_sync();
  };

  uint64_t pool[PREG];
#pragma unroll
  for (int k = 0; k < PREG; ++k) pool[k] = kNoKey;
  int size = 0, ndc = 0, hops = 0;
  uint32_t* trace_row = a.out_trace && live ? a.out_trace + (size_t)qid * a.trace_cap : nullptr;

  // ---- entry: the nearest navigating node seeds the pool
  uint32_t p;
  {
    const uint32_t* ent = a.entry + (a.entry_group > 0 ? (live ? qid : 0) / a.entry_group * a.s : 0);
    uint64_t best = kNoKey;
    for (int e0 = 0; e0 < a.s; e0 += S) {
      const int m = min(S, a.s - e0);
      if (gl < m) bids[gl] = ent[e0 + gl];
      wave_sync();
      batch_keys(m, 0);
      if (gl < m) best = min(best, bkeys[gl]);
      wave_sync();
    }
    best = gmin64<S>(best, gbase);
    ndc = a.s;
    if (gl == 0) pool[0] = best | 1ull;
    size = 1;
    p = key_id(best);
    bool ev = false;
    if (gl == 0) visit(p, ev);
    if (trace_row && gl == 0) trace_row[0] = p;
    wave_sync();
  }

  // Staging an expansion (all lanes call it; nb = kSent stages nothing):
  // its row's ids go through the visited cache, the new ones are compacted
  // into bids and the first gather pass is issued.
  Pass pend;
  int pm = 0;
  auto stage_row = [&](const uint32_t (&nb)[NRL]) {
    bool ev = false;
    bool fresh[NRL];
#pragma unroll
    for (int t = 0; t < NRL; ++t) fresh[t] = nb[t] != kSent && visit(nb[t], ev);
    int cnt = 0;
#pragma unroll
    for (int t = 0; t < NRL; ++t) {
      const uint64_t fm = __ballot(fresh[t]) & gmask;
      if (fresh[t]) bids[cnt + lane_prefix(fm)] = nb[t];
      cnt += __popcll(fm);
    }
    pm = cnt;
    evicted |= gbits<S>(__ballot(ev), gbase) != 0ull;
    wave_sync();
    if (kPipe && __any(pm > 0)) issue(pend, 0, pm);
  };
  auto read_row = [&](uint32_t node, bool ok, uint32_t (&nb)[NRL]) {
#pragma unroll
    for (int t = 0; t < NRL; ++t) {
      const int c = gl + t * S;
      nb[t] = ok && c < R ? a.graph[(size_t)node * R + c] : kSent;
    }
  };
  bool active = live;
  {
    uint32_t nb[NRL];
    read_row(p, active, nb);
    stage_row(nb);
  }

  for (;;) {
    if (!__any(active)) break;
    hops += active ? 1 : 0;

    // speculation: the first unchecked pool entry is the next expansion
    // unless a new key beats it; read its row alongside this step's gathers
    uint64_t um = kNoKey;
#pragma unroll
    for (int k = 0; k < PREG; ++k) um = min(um, (pool[k] & 1ull) ? kNoKey : pool[k]);
    const uint64_t u_spec = gmin64<S>(um, gbase);
    uint32_t nb_spec[NRL];
    read_row(key_id(u_spec), active && u_spec != kNoKey, nb_spec);

    // keys of the staged expansion's new ids (up to 64 per group)
    const int m = pm;
    ndc += m;
    if (__any(m > 0)) {
      if constexpr (kPipe) finish(pend, 0);
      batch_keys(m, kPipe ? 1 : 0);
    }
    // the L-th pool key: a new key above it is cut at once (it stays visited)
    uint64_t worst = kNoKey;
    if (__any(size == L)) {
      const int wl = (L - 1) % S, wr = (L - 1) / S;
      uint64_t wv = kNoKey;
#pragma unroll
      for (int k = 0; k < PREG; ++k)
        if (k == wr) wv = pool[k];
      wv = gread64<S>(wv, wl, gbase);
      if (size == L) worst = wv;
    }
    constexpr int NB = 64 / S;  // new keys per lane (chunks of S)
    uint64_t b[NB];
    uint64_t bmin = kNoKey;
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const int c = gl + t * S;
      b[t] = c < m ? bkeys[c] : kNoKey;
      if (b[t] > worst) b[t] = kNoKey;
    }
    // a pool member the cache forgot comes back with its pool key (up to
    // the checked bit): drop it so the pool never holds an id twice
    if (__any(evicted && m > 0)) {
      uint32_t plo[PREG];
#pragma unroll
      for (int k = 0; k < PREG; ++k) plo[k] = (uint32_t)pool[k] | 1u;
#pragma unroll
      for (int t = 0; t < NB; ++t) {
        uint64_t mm = evicted ? gbits<S>(__ballot(b[t] != kNoKey), gbase) : 0ull;
        while (__any(mm != 0ull)) {
          const bool act = mm != 0ull;
          const int j = act ? __builtin_ctzll(mm) : 0;
          const uint32_t bj = gread32<S>((uint32_t)b[t] | 1u, j, gbase);
          uint64_t hit = 0;
#pragma unroll
          for (int k = 0; k < PREG; ++k) hit |= gbits<S>(__ballot(act && plo[k] == bj), gbase);
          if (act && hit && gl == j) b[t] = kNoKey;
          mm &= mm - 1ull;
        }
      }
    }
#pragma unroll
    for (int t = 0; t < NB; ++t) bmin = min(bmin, b[t]);

    // next expansion, decided before the merge: the smallest unchecked key u
    // of (pool + new keys) is kept iff fewer than L keys precede it
    uint64_t u = u_spec;
    bool more = active && u != kNoKey;
    const uint64_t nmin = gmin64<S>(bmin, gbase);
    if (__any(active && nmin < u)) {
      if (active && nmin < u) u = nmin;
      int rank_u = 0;
#pragma unroll
      for (int k = 0; k < PREG; ++k) rank_u += __popcll(gbits<S>(__ballot(pool[k] < u), gbase));
      more = active && u != kNoKey && rank_u < L;
    }
    {
      if (more && trace_row && gl == 0 && hops < a.trace_cap) trace_row[hops] = key_id(u);
      uint32_t nb[NRL];
      if (__any(more && u != u_spec)) {
        read_row(key_id(u), more, nb);
#pragma unroll
        for (int t = 0; t < NRL; ++t)
          if (u == u_spec) nb[t] = more ? nb_spec[t] : kSent;
      } else {
#pragma unroll
        for (int t = 0; t < NRL; ++t) nb[t] = more ? nb_spec[t] : kSent;
      }
      stage_row(nb);  // its gathers overlap the merge below
    }

    // rank-based merge of the surviving new keys, one chunk of S at a time
#pragma unroll
    for (int t = 0; t < NB; ++t) {
      const uint64_t bm = gbits<S>(__ballot(b[t] != kNoKey), gbase);
      if (!__any(bm != 0ull)) continue;
      int rank = 0, qcnt = 0;
      int shift[PREG];
#pragma unroll
      for (int k = 0; k < PREG; ++k) shift[k] = 0;
      for (uint64_t mm = bm; __any(mm != 0ull); mm &= mm - 1ull) {
        const bool act = mm != 0ull;
        const int j = act ? __builtin_ctzll(mm) : 0;
        uint64_t bj = gread64<S>(b[t], j, gbase);
        if (!act) bj = kNoKey;
        int r = 0;
#pragma unroll
        for (int k = 0; k < PREG; ++k) {
          r += __popcll(gbits<S>(__ballot(pool[k] < bj), gbase));
          shift[k] += bj < pool[k] ? 1 : 0;
        }
        if (act && gl == j) rank = r;
        qcnt += bj < b[t] ? 1 : 0;
      }
#pragma unroll
      for (int k = 0; k < PREG; ++k) {
        const int np = k * S + gl + shift[k];
        if (pool[k] != kNoKey && np < L) stage[np] = pool[k];
      }
      if (b[t] != kNoKey && rank + qcnt < L) stage[rank + qcnt] = b[t];
      wave_sync();
      size = min(L, size + (int)__popcll(bm));
#pragma unroll
      for (int k = 0; k < PREG; ++k) {
        const int i = k * S + gl;
        pool[k] = i < size ? stage[i] : kNoKey;
      }
      wave_sync();
    }
    if (!more) active = false;
#pragma unroll
    for (int k = 0; k < PREG; ++k)
      if (more && pool[k] == u) pool[k] |= 1ull;  // mark the next expansion checked
  }

  // ---- optional rerank: exact FP32 keys of the first max(rerank, K) pool
  // entries against the FP32 vectors, re-sorted by (dist, id). The visited
  // cache is dead here, so its LDS holds the new keys; `stage` the order.
  if (a.base_f32 != nullptr) {
    constexpr int RL = S < 16 ? S : 16;  // lanes per candidate
    const int rr = live ? min(a.rerank < 0 ? -a.rerank * K : max(a.rerank, K), size) : 0;
    uint64_t* rkeys = reinterpret_cast<uint64_t*>(table);
    const int d4 = a.d >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(q);
    for (int c0 = 0; __any(c0 < rr); c0 += S) {
      const int cm = max(0, min(S, rr - c0));
#pragma unroll
      for (int k = 0; k < PREG; ++k)
        if (k == c0 / S && gl < cm) bids[gl] = key_id(pool[k]);
      wave_sync();
      for (int j0 = 0; __any(j0 < cm); j0 += S / RL) {
        const int c = j0 + gl / RL;
        const int lr = gl % RL;
        float acc = 0.f;
        uint32_t id = 0;
        if (c < cm) {
          id = bids[c];
          const float4* x4 = reinterpret_cast<const float4*>(a.base_f32 + (size_t)id * a.d);
          for (int ch = lr; ch < d4; ch += RL) {
            const float4 x = x4[ch], qq = q4[ch];
            if (ip) {
              acc = fmaf(qq.x, x.x, acc);
              acc = fmaf(qq.y, x.y, acc);
              acc = fmaf(qq.z, x.z, acc);
              acc = fmaf(qq.w, x.w, acc);
            } else {
              float df = qq.x - x.x;
              acc = fmaf(df, df, acc);
              df = qq.y - x.y;
              acc = fmaf(df, df, acc);
              df = qq.z - x.z;
              acc = fmaf(df, df, acc);
              df = qq.w - x.w;
              acc = fmaf(df, df, acc);
            }
          }
        }
        acc = group_sum<RL>(acc, lane);
        if (c < cm && lr == 0) rkeys[c0 + c] = make_key(ip ? -acc : acc, id);
      }
      wave_sync();
    }
    for (int i0 = 0; __any(i0 < rr); i0 += S) {
      const int i = i0 + gl;
      if (i < rr) {
        const uint64_t ki = rkeys[i];
        int r = 0;
        for (int j = 0; j < rr; ++j) r += rkeys[j] < ki ? 1 : 0;
        stage[r] = ki;
      }
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < PREG; ++k) {
      const int i = k * S + gl;
      pool[k] = i < rr ? stage[i] : kNoKey;
    }
    wave_sync();
  }

  // ---- output: first K pool entries, padded to the row stride
  if (live) {
    uint32_t* oid = a.out_ids + (size_t)qid * a.kstride;
    float* od = a.out_d + (size_t)qid * a.kstride;
#pragma unroll
    for (int k = 0; k < PREG; ++k) {
      const int i = k * S + gl;
      if (i < a.kstride) {
        const uint64_t key = i < K ? pool[k] : kNoKey;
        oid[i] = key == kNoKey ? kSent : key_id(key);
        od[i] = key == kNoKey ? __uint_as_float(0x7F800000u) : unord_f32((uint32_t)(key >> 32));
      }
    }
    for (int i = LCAP + gl; i < a.kstride; i += S) {
      oid[i] = kSent;
      od[i] = __uint_as_float(0x7F800000u);
    }
    if (gl == 0) {
      if (a.out_ndc) a.out_ndc[qid] = ndc;
      if (a.out_hops) a.out_hops[qid] = hops;
    }
    if (trace_row)
      for (int i = hops + gl; i < a.trace_cap; i += S) trace_row[i] = kSent;
  }
  wave_sync();  // the LDS of this wavefront is reused by its next queries
}

// Q queries per wavefront: wavefront w takes queries w * Q .. w * Q + Q - 1.
template <typename T, int DC, int G, int NP, int PREG, int S>
__global__ __launch_bounds__(256) void group_kernel(Args a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int Q = 64 / S;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  unsigned char* my = smem + (size_t)wv * Q * a.lds_per_wave;
  const int64_t slot0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wv) * Q;
  if (slot0 >= a.nq) return;  // uniform per wavefront
  const int64_t slot = slot0 + lane / S;
  run_groups<T, DC, G, NP, PREG, S>(a, my, lane, slot < a.nq ? slot : -1, a.L, a.K);
}

// Persistent form: each wavefront takes Q consecutive slots of the work
// queue at a time until the queue is exhausted.
template <typename T, int DC, int G, int NP, int PREG, int S>
__global__ __launch_bounds__(256) void group_kernel_batched(Args a) {
  extern __shared__ __align__(16) unsigned char smem[];
  constexpr int Q = 64 / S;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  unsigned char* my = smem + (size_t)wv * Q * a.lds_per_wave;
  int64_t slot0 = ((int64_t)blockIdx.x * (blockDim.x >> 6) + wv) * Q;
  for (;;) {
    if (a.counter) {
      uint32_t s0 = 0u;
      if (lane == 0) s0 = atomicAdd(a.counter, (uint32_t)Q);
      slot0 = (int64_t)__builtin_amdgcn_readfirstlane(s0);
    }
    if (slot0 >= a.nlist) break;  // uniform per wavefront
    const int64_t slot = slot0 + lane / S;
    int64_t qid = slot < a.nlist ? (a.qlist ? (int64_t)a.qlist[slot] : slot) : -1;
    if (qid >= a.nq) qid = -1;  // a bad queue entry is skipped, never dereferenced
    const int L = min(max(qid >= 0 && a.L_arr ? a.L_arr[qid] : a.L, 1), S * PREG);
    const int K = min(max(qid >= 0 && a.K_arr ? a.K_arr[qid] : a.K, 1), a.kstride);
    run_groups<T, DC, G, NP, PREG, S>(a, my, lane, qid, L, K);
    if (!a.counter) break;
  }
}

template <typename T, int DC, int G, int NP, int S>
KernelFn pick_group_preg(int preg, bool batched) {
  if (batched) {
    switch (preg) {
      case 2: return group_kernel_batched<T, DC, G, NP, 2, S>;
      case 3: return group_kernel_batched<T, DC, G, NP, 3, S>;
      case 4: return group_kernel_batched<T, DC, G, NP, 4, S>;
      case 8: return group_kernel_batched<T, DC, G, NP, 8, S>;
      default: return nullptr;
    }
  }
  switch (preg) {
    case 2: return group_kernel<T, DC, G, NP, 2, S>;
    case 3: return group_kernel<T, DC, G, NP, 3, S>;
    case 4: return group_kernel<T, DC, G, NP, 4, S>;
    case 8: return group_kernel<T, DC, G, NP, 8, S>;
    default: return nullptr;
  }
}

}  // namespace

// Kernel for a grouped launch, or null when no compiled shape fits: dtype
// and chunk count (16-byte chunks per vector), pool registers per lane, lanes
// per query. Gather shapes: 8 lanes per candidate, 2 passes in flight.
KernelFn ssg_internal_group_kernel(int dtype, int dc, int preg, int lanes, bool batched) {
  if (lanes != 32) return nullptr;
  if (dtype == SSG_F32) {
    switch (dc) {
      case 24: return pick_group_preg<F32T, 24, 8, 2, 32>(preg, batched);  // d = 96
      case 32: return pick_group_preg<F32T, 32, 8, 2, 32>(preg, batched);  // d = 128
      default: return nullptr;
    }
  }
  if (dtype == SSG_BF16) {
    switch (dc) {
      case 12: return pick_group_preg<BF16T, 12, 4, 2, 32>(preg, batched);  // d = 96
      case 16: return pick_group_preg<BF16T, 16, 8, 2, 32>(preg, batched);  // d = 128
      default: return nullptr;
    }
  }
  if (dtype == SSG_FP8E4M3) {
    switch (dc) {
      case 6: return pick_group_preg<FP8HwT, 6, 8, 2, 32>(preg, batched);  // d = 96
      case 8: return pick_group_preg<FP8HwT, 8, 8, 2, 32>(preg, batched);  // d = 128
      default: return nullptr;
    }
  }
  return nullptr;
}
