// ssg_search.hip -- gfx950 kernels for batched greedy best-first search over
// a navigating satellite-system graph (the paper's Alg. 1, started from the
// navigating node nearest each query, Sec. 4.1).
//
// Work mapping: one 64-lane wavefront owns one query from start to finish.
// Nothing about a query is shared with another wavefront, so no cross-wave
// synchronisation exists on the search path.
//
// Per-query state (all on chip):
//   pool      the candidate pool S of at most L entries, kept sorted, held in
//             VGPRs: entry i lives in lane i % 64, register slot i / 64.
//             An entry is one 64-bit key  ord(dist) << 32 | id << 1 | checked,
//             so unsigned order is the (dist, id) order and the checked flag
//             never decides it (ids in the pool are distinct).
//   visited   which node ids already have a distance. Forgetting an id can
//             only cost a recomputation, never change the result: a node that
//             left the pool left because its key exceeded the L-th key, which
//             never grows afterwards, so a recomputed copy is cut again at
//             once; a node still in the pool comes back with the same key and
//             is dropped before the merge. Three forms, all in LDS:
//               cache  (default) 4-way set-associative, 16-bit entries. The
//                      id is mapped by a bijection of its low k bits
//                      (multiplication by an odd constant mod 2^k); the high
//                      bits pick the set and the rest is the stored tag, so a
//                      hit is never false. A full set overwrites one way.
//               hash   open addressing of full ids, cleared and refilled from
//                      the pool when half full (used when the tag would not
//                      fit 16 bits).
//               exact  an n-bit bitset.
//   stage     LDS scratch for the merge (L keys), batch ids and keys (64 each).
//
// One iteration (one expansion of Alg. 1):
//   1. ballot over the pool for the first unchecked entry; mark it checked;
//   2. lanes 0..R-1 read the neighbour row (one coalesced row read);
//   3. each lane tests-and-inserts its id in the visited hash (LDS atomics);
//   4. surviving ids are compacted (ballot + mbcnt) into the batch;
//   5. G lanes per candidate gather the candidate's vector in 16-byte chunks
//      and reduce the distance across the group with lane shuffles;
//   6. rank-based merge: for every new key the number of smaller pool keys
//      (ballot + popcount) and of smaller new keys gives its slot; every pool
//      entry moves right by the number of smaller new keys; entries landing
//      at positions >= L fall off (truncation). Positions go through LDS once.
// The loop ends when no pool entry is unchecked; the first K keys are written.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>
#include <type_traits>

#include "ssg.h"
#include "ssg_internal.h"
#include "ssg_search_common.h"

namespace {

// ------------------------------------------------------------------ kernel
// T: stored element type; DC: chunks per vector (0 = runtime, query in LDS);
// G: lanes cooperating on one candidate; NP: gather passes whose loads are
// all issued before the first is consumed (NP * 64 / G candidates in flight);
// PREG: pool registers per lane (pool capacity 64 * PREG).
template <typename T, int DC, int G, int NP, int PREG, bool QL>
__device__ __forceinline__ void run_query(const Args& a, unsigned char* my, const int lane,
                                          const int64_t qid, const int L, const int K) {
  constexpr int EPC = T::kEpc;
  constexpr int CPP = 64 / G;                           // candidates per pass
  constexpr int NCH = DC > 0 ? (DC + G - 1) / G : 1;    // chunks per lane
  constexpr int LCAP = 64 * PREG;
  constexpr bool kCompiled = DC > 0;              // chunk count known at compile time
  constexpr bool kQueryInRegs = kCompiled && !QL;  // else the query (and scale) sit in LDS
  constexpr bool kScaled = T::kScaled;

  uint64_t* stage = reinterpret_cast<uint64_t*>(my);
  uint64_t* bkeys = stage + LCAP;
  uint32_t* bids = reinterpret_cast<uint32_t*>(bkeys + 64);
  float* qlds = reinterpret_cast<float*>(bids + 64);  // runtime-DC query (and scale) copy
  const int qlds_floats = kQueryInRegs ? 0 : a.dc * EPC * (kScaled ? 2 : 1);
  uint32_t* table = reinterpret_cast<uint32_t*>(qlds + qlds_floats);

  const int g = lane % G;
  const int grp = lane / G;
  const float* q = a.queries + (size_t)qid * a.d;
  const bool ip = a.metric == 1;
  const int R = a.R;

  // query (and fp8 scale) fragment: lane g holds chunks g, g+G, ...
  float qf[kQueryInRegs ? NCH * EPC : 1];
  float sf[kQueryInRegs && kScaled ? NCH * EPC : 1];
  if constexpr (kQueryInRegs) {
#pragma unroll
    for (int t = 0; t < NCH; ++t) {
      const int ch = g + G * t;
      const bool ok = DC % G == 0 || ch < DC;
#pragma unroll
      for (int e = 0; e < EPC; e += 4) {
        float4 v = ok ? *reinterpret_cast<const float4*>(q + ch * EPC + e) : make_float4(0, 0, 0, 0);
        qf[t * EPC + e] = v.x;
        qf[t * EPC + e + 1] = v.y;
        qf[t * EPC + e + 2] = v.z;
        qf[t * EPC + e + 3] = v.w;
        if constexpr (kScaled) {
          float4 w = ok ? *reinterpret_cast<const float4*>(a.dim_scale + ch * EPC + e)
                        : make_float4(0, 0, 0, 0);
          sf[t * EPC + e] = w.x;
          sf[t * EPC + e + 1] = w.y;
          sf[t * EPC + e + 2] = w.z;
          sf[t * EPC + e + 3] = w.w;
        }
      }
    }
  } else {
    for (int j = lane; j < a.d; j += 64) {
      qlds[j] = q[j];
      if constexpr (kScaled) qlds[a.d + j] = a.dim_scale[j];
    }
  }

  // visited structure
  const uint32_t hmask = (1u << a.hash_log2) - 1u;
  const int twords = a.vmode == 0 ? (int)((a.n + 31) >> 5)
                     : a.vmode == 2 ? (int)((hmask + 1u) >> 1)
                                    : (int)(hmask + 1u);
  const uint32_t tfill = a.vmode == 1 ? kSent : 0u;
  for (int i = lane; i < twords; i += 64) table[i] = tfill;
  const int tshift = a.id_bits - (a.hash_log2 - 2);           // cache: tag bits
  const uint32_t kmask = (uint32_t)((1ull << a.id_bits) - 1u);
  wave_sync();
  int hcount = 0;                         // ids inserted since the last clear
  const int hlimit = (int)((hmask + 1u) >> 1);

  // one distance term; the fp8 value is code * scale rounded to fp32 first
  auto term = [&](float acc, float qv, float xv) -> float {
    if (ip) return fmaf(qv, xv, acc);
    const float df = qv - xv;
    return fmaf(df, df, acc);
  };

  // One gather pass covers candidates c0 + p * CPP + grp (p < NP) of
  // bids[0..m): `issue` reads their ids and, on the compiled path, starts
  // every load of the pass; `finish` turns the loaded rows into keys in
  // bkeys. Between the two the loads are in flight.
  struct Pass {
    uint4 buf[NP][kCompiled ? NCH : 1];
    uint32_t idp[NP];
    bool vp[NP];
  };
  auto issue = [&](Pass& ps, int c0, int m) {
#pragma unroll
    for (int p = 0; p < NP; ++p) {
      const int c = c0 + p * CPP + grp;
      ps.vp[p] = c < m;
      ps.idp[p] = ps.vp[p] ? bids[c] : 0u;
    }
    if constexpr (kCompiled) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        const uint4* vec = reinterpret_cast<const uint4*>(a.base + (size_t)ps.idp[p] * a.dc * 16);
#pragma unroll
        for (int t = 0; t < NCH; ++t) {
          // lanes past the batch read row 0 (idp = 0) and their sums are
          // discarded; loading unconditionally avoids zeroing the registers
          const int ch = g + G * t;
          if (DC % G == 0 || ch < DC) ps.buf[p][t] = vec[ch];
          else ps.buf[p][t] = make_uint4(0, 0, 0, 0);
        }
      }
    }
  };
  // Keys of the pass set at c0 (m = the batch size, so that a batch that
  // fits the first pass computes only that pass). The metric and the pass
  // count are uniform, so both are chosen by one branch.
  auto finish = [&](Pass& ps, int c0, int m) {
    auto run = [&](auto ip_c, auto np_c) {
      constexpr bool IP = decltype(ip_c)::value;
      constexpr int NPL = decltype(np_c)::value;
      float acc[NPL];
#pragma unroll
      for (int p = 0; p < NPL; ++p) acc[p] = 0.f;
    if constexpr (kCompiled) {
      // with the query in LDS, re-read it per pass instead of letting the
      // compiler keep a register copy (the point is to free those registers)
      if constexpr (!kQueryInRegs) __asm__ volatile("" ::: "memory");
#pragma unroll
        for (int p = 0; p < NPL; ++p) {
#pragma unroll
          for (int t = 0; t < NCH; ++t) {
            const int ch = g + G * t;
            if (DC % G == 0 || ch < DC) {
              float x[EPC];
              T::decode(ps.buf[p][t], x);
#pragma unroll
              for (int e = 0; e < EPC; ++e) {
                float sv, qv;
                if constexpr (kQueryInRegs) {
                  sv = kScaled ? sf[t * EPC + e] : 1.f;
                  qv = qf[t * EPC + e];
                } else {
                  sv = kScaled ? qlds[a.d + ch * EPC + e] : 1.f;
                  qv = qlds[ch * EPC + e];
                }
                const float xv = kScaled ? __fmul_rn(x[e], sv) : x[e];
                if constexpr (IP) {
                  acc[p] = fmaf(qv, xv, acc[p]);
                } else {
                  const float df = qv - xv;
                  acc[p] = fmaf(df, df, acc[p]);
                }
              }
            }
          }
        }
    } else {
#pragma unroll
      for (int p = 0; p < NPL; ++p) {
        if (ps.vp[p]) {
          const uint4* vec = reinterpret_cast<const uint4*>(a.base + (size_t)ps.idp[p] * a.dc * 16);
#pragma unroll 4
          for (int ch = g; ch < a.dc; ch += G) {
            float x[EPC];
            T::decode(vec[ch], x);
#pragma unroll
            for (int e = 0; e < EPC; ++e) {
              const float xv = kScaled ? __fmul_rn(x[e], qlds[a.d + ch * EPC + e]) : x[e];
              acc[p] = term(acc[p], qlds[ch * EPC + e], xv);
            }
          }
        }
      }
    }
#pragma unroll
      for (int p = 0; p < NPL; ++p) {
        acc[p] = group_sum<G>(acc[p], lane);
        if (ps.vp[p] && g == 0)
          bkeys[c0 + p * CPP + grp] = IP ? make_key(-acc[p], ps.idp[p]) : make_key_nonneg(acc[p], ps.idp[p]);
      }
    };
    using One = std::integral_constant<int, 1>;
    using All = std::integral_constant<int, NP>;
    if (NP == 1 || c0 + CPP >= m) {
      if (ip) run(std::true_type{}, One{});
      else run(std::false_type{}, One{});
    } else {
      if (ip) run(std::true_type{}, All{});
      else run(std::false_type{}, All{});
    }
  };
  // keys of bids[first * CPP * NP .. m) (the passes before `first` are done)
  auto batch_keys = [&](int m, int first = 0) {
    for (int c0 = first * CPP * NP; c0 < m; c0 += CPP * NP) {
      Pass ps;
      issue(ps, c0, m);
      finish(ps, c0, m);
    }
    wave_sync();
  };

  // test-and-insert id; returns true when the id was not yet visited
  auto visit = [&](uint32_t id) -> bool {
    if (a.vmode == 2) {
      // set = high bits of the k-bit image, tag = the rest + 1 (0 marks empty)
      const uint32_t h = (id * 0x9E3779B1u) & kmask;
      const uint32_t set = h >> tshift;
      const uint32_t tag = (h & ((1u << tshift) - 1u)) + 1u;
      const uint64_t w = reinterpret_cast<const uint64_t*>(table)[set];
      const uint32_t t0 = (uint32_t)w & 0xFFFFu, t1 = (uint32_t)(w >> 16) & 0xFFFFu;
      const uint32_t t2 = (uint32_t)(w >> 32) & 0xFFFFu, t3 = (uint32_t)(w >> 48);
      if (t0 == tag || t1 == tag || t2 == tag || t3 == tag) return false;
      // lanes that pick the same way in one step overwrite each other: a loss
      // is a forgotten id, which is allowed
      const uint32_t way = t0 == 0u ? 0u : t1 == 0u ? 1u : t2 == 0u ? 2u : t3 == 0u ? 3u
                                                                               : (tag ^ (tag >> 2)) & 3u;
      reinterpret_cast<uint16_t*>(table)[set * 4u + way] = (uint16_t)tag;
      return true;
    }
    if (a.vmode == 0) {
      const uint32_t bit = 1u << (id & 31u);
      const uint32_t old = atomicOr(&table[id >> 5], bit);
      return (old & bit) == 0u;
    }
    // one LDS compare-and-swap per probe: an empty slot takes the id, a slot
    // holding the id means visited, anything else moves to the next slot
    uint32_t h = hash_slot(id, hmask);
    for (;;) {
      const uint32_t old = atomicCAS(&table[h], kSent, id);
      if (old == kSent) return true;
      if (old == id) return false;
      h = (h + 1u) & hmask;
    }
  };

  uint64_t pool[PREG];
#pragma unroll
  for (int k = 0; k < PREG; ++k) pool[k] = kNoKey;
  int size = 0;
  int ndc = 0, hops = 0;

  // ---- entry: the nearest navigating node seeds the pool and is expanded first
  uint32_t p;
  {
    uint64_t best = kNoKey;
    for (int e0 = 0; e0 < a.s; e0 += 64) {
      const int m = min(64, a.s - e0);
      if (lane < m) bids[lane] = a.entry[(a.entry_group > 0 ? qid / a.entry_group * a.s : 0) + e0 + lane];
      wave_sync();
      batch_keys(m);
      if (lane < m) best = min(best, bkeys[lane]);
      wave_sync();
    }
    best = wave_min64_split(best);
    ndc = a.s;
    if (lane == 0) pool[0] = best | 1ull;
    size = 1;
    p = key_id(best);
    if (lane == 0) visit(p);
    if (a.out_trace && lane == 0) a.out_trace[(size_t)qid * a.trace_cap] = p;
    hcount = 1;
    wave_sync();
  }
  // Staging an expansion: its row's ids go through the visited set, the new
  // ones are compacted into bids and the first gather pass is issued. The
  // loop stages the next expansion before merging the current one, so that
  // merge runs while the next gathers are in flight
  // (only where the staged pass is at most 8 chunks per lane: its registers
  // stay live across the merge)
  constexpr bool kPipe = kCompiled && NP * NCH <= 8;
  Pass pend;
  int pm = 0;  // candidates of the staged expansion
  auto stage_row = [&](uint32_t nb) {
    // hash form: rebuild from the pool when half full (the keys of the batch
    // being merged may be forgotten; the duplicate check below covers them)
    if (a.vmode == 1 && hcount + R > hlimit) {
      for (int i = lane; i <= (int)hmask; i += 64) table[i] = kSent;
      wave_sync();
#pragma unroll
      for (int k = 0; k < PREG; ++k)
        if (pool[k] != kNoKey) visit(key_id(pool[k]));
      wave_sync();
      hcount = size;
    }
    const bool fresh = nb != kSent && visit(nb);
    const uint64_t fm = __ballot(fresh);
    pm = __popcll(fm);
    if (fresh) bids[lane_prefix(fm)] = nb;
    wave_sync();
    hcount += pm;
    if (kPipe && pm > 0) issue(pend, 0, pm);
  };
  stage_row(lane < R ? a.graph[(size_t)p * R + lane] : kSent);

  for (;;) {
    ++hops;
    if (hops > a.n + 1) break;  // cannot happen (each node is expanded at most once); bounds the loop

    // speculation: the first unchecked pool entry is the next expansion unless
    // a new key beats it; read its row now, alongside this hop's gathers
    uint64_t u = kNoKey;
#pragma unroll
    for (int k = 0; k < PREG; ++k) {
      const uint64_t um = __ballot((pool[k] & 1ull) == 0ull);
      if (u == kNoKey && um) u = readlane64(pool[k], __builtin_ctzll(um));
    }
    const uint64_t u_spec = u;
    const uint32_t nb_spec =
        u_spec != kNoKey && lane < R ? a.graph[(size_t)key_id(u_spec) * R + lane] : kSent;

    // keys of the staged expansion's new ids
    const int m = pm;
    ndc += m;
    uint64_t b = kNoKey;
    if (m > 0) {
      if constexpr (kPipe) finish(pend, 0, m);
      batch_keys(m, kPipe ? 1 : 0);
      b = lane < m ? bkeys[lane] : kNoKey;
      if (size == L) {
        // a new key above the L-th pool key would land at position >= L and be
        // cut at once; drop it before the merge (it stays visited)
        uint64_t worst = kNoKey;
#pragma unroll
        for (int k = 0; k < PREG; ++k)
          if (k == ((L - 1) >> 6)) worst = readlane64(pool[k], (L - 1) & 63);
        if (b > worst) b = kNoKey;
      }
      if (a.vmode != 0) {
        // a pool member the visited set forgot comes back with its pool key
        // (up to the checked bit); drop it so the pool never holds an id twice
        // (an id decides it: equal ids have equal keys; the low word of a key
        // is id << 1 | checked, and ids stay below 2^31 - 1)
        uint32_t plo[PREG];
#pragma unroll
        for (int k = 0; k < PREG; ++k) plo[k] = (uint32_t)pool[k] | 1u;
        for (uint64_t mm = __ballot(b != kNoKey); mm; mm &= mm - 1) {
          const int j = __builtin_ctzll(mm);
          const uint32_t bj = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, j) | 1u;
          uint64_t hit = 0;
#pragma unroll
          for (int k = 0; k < PREG; ++k) hit |= __ballot(plo[k] == bj);
          if (hit && lane == j) b = kNoKey;
        }
      }
    }
    const uint64_t bm = __ballot(b != kNoKey);  // new keys that can enter the pool

    // next expansion, decided before the merge: the smallest unchecked key u
    // of (pool + new keys) is kept iff fewer than L keys precede it;
    // otherwise every kept entry is checked. When no new key is below
    // u_spec, u_spec keeps its pool position (< L).
    bool more = u != kNoKey;
    if (__ballot(b < u)) {
      u = wave_min64_split(b);  // below u_spec, so the smallest unchecked key
      int rank_u = 0;     // (no new key is below u)
#pragma unroll
      for (int k = 0; k < PREG; ++k) rank_u += __popcll(__ballot(pool[k] < u));
      more = rank_u < L;
    }
    if (more) {
      // expansion number hops + 1 (0-based: hops) is u
      if (a.out_trace && lane == 0 && hops < a.trace_cap)
        a.out_trace[(size_t)qid * a.trace_cap + hops] = key_id(u);
      // stage it now: its gathers overlap the merge below
      const uint32_t nb_next =
          u == u_spec ? nb_spec : lane < R ? a.graph[(size_t)key_id(u) * R + lane] : kSent;
      stage_row(nb_next);
    }

    // rank-based merge of the surviving new keys into the pool, truncated to L
    if (bm) {
      int rank = 0, qcnt = 0;
      int shift[PREG];
#pragma unroll
      for (int k = 0; k < PREG; ++k) shift[k] = 0;
      for (uint64_t mm = bm; mm; mm &= mm - 1) {
        const int j = __builtin_ctzll(mm);
        const uint64_t bj = readlane64(b, j);
        int r = 0;
#pragma unroll
        for (int k = 0; k < PREG; ++k) {
          r += __popcll(__ballot(pool[k] < bj));
          shift[k] += bj < pool[k] ? 1 : 0;
        }
        if (lane == j) rank = r;
        qcnt += bj < b ? 1 : 0;
      }
#pragma unroll
      for (int k = 0; k < PREG; ++k) {
        const int np = k * 64 + lane + shift[k];
        if (pool[k] != kNoKey && np < L) stage[np] = pool[k];
      }
      if (b != kNoKey && rank + qcnt < L) stage[rank + qcnt] = b;
      wave_sync();
      size = min(L, size + (int)__popcll(bm));
#pragma unroll
      for (int k = 0; k < PREG; ++k) {
        const int i = k * 64 + lane;
        pool[k] = i < size ? stage[i] : kNoKey;
      }
      wave_sync();
    }
    if (!more) break;
#pragma unroll
    for (int k = 0; k < PREG; ++k)
      if (pool[k] == u) pool[k] |= 1ull;  // mark the next expansion checked
  }

  // ---- optional rerank: exact FP32 keys of the first `rerank` pool entries
  // against the FP32 vectors, re-sorted by (dist, id). The visited table is
  // dead here, so its LDS holds the new keys; `stage` holds the sorted order.
  // (never fewer than K entries: every returned entry is re-scored)
  if (a.base_f32 != nullptr) {
    const int rr = min(a.rerank < 0 ? -a.rerank * K : max(a.rerank, K), size);
    uint32_t* rids = bids;  // reused 64 at a time
    uint64_t* rkeys = reinterpret_cast<uint64_t*>(table);
    const int d4 = a.d >> 2;
    const float4* q4 = reinterpret_cast<const float4*>(q);
    const int l16 = lane & 15;
    // compiled dimension: the query's chunks stay in registers and each round
    // issues every load of U candidate groups (4 candidates each, 16 lanes per
    // candidate, NR float4 per lane) before the first is used: up to 8 float4
    // per lane in flight (16 candidates of 128 floats), so a pool of 80 takes
    // 5 rounds of load latency
    constexpr int D4 = kCompiled ? DC * EPC / 4 : 1;
    constexpr int NR = (D4 + 15) / 16;
    constexpr int U = NR >= 8 ? 1 : 8 / NR;
    float4 qr[NR];
    if constexpr (kCompiled) {
#pragma unroll
      for (int t = 0; t < NR; ++t) {
        const int ch = l16 + 16 * t;
        qr[t] = D4 % 16 == 0 || ch < D4 ? q4[ch] : make_float4(0, 0, 0, 0);
      }
    }
    for (int c0 = 0; c0 < rr; c0 += 64) {
      const int cm = min(64, rr - c0);
      // ids of pool entries c0 .. c0+cm-1 (entry i sits in lane i % 64, slot i / 64)
#pragma unroll
      for (int k = 0; k < PREG; ++k)
        if (k == (c0 >> 6) && lane < cm) rids[lane] = key_id(pool[k]);
      wave_sync();
      if constexpr (kCompiled) {
        for (int j0 = 0; j0 < cm; j0 += 4 * U) {
          uint32_t idr[U];
          float4 xr[U][NR];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int c = j0 + 4 * u + (lane >> 4);
            idr[u] = c < cm ? rids[c] : 0u;  // past the list: row 0, discarded
            const float4* x4 = reinterpret_cast<const float4*>(a.base_f32 + (size_t)idr[u] * a.d);
#pragma unroll
            for (int t = 0; t < NR; ++t) {
              const int ch = l16 + 16 * t;
              xr[u][t] = D4 % 16 == 0 || ch < D4 ? x4[ch] : make_float4(0, 0, 0, 0);
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int c = j0 + 4 * u + (lane >> 4);
            float acc = 0.f;
#pragma unroll
            for (int t = 0; t < NR; ++t) {
              if (D4 % 16 == 0 || l16 + 16 * t < D4) {
                acc = term(acc, qr[t].x, xr[u][t].x);
                acc = term(acc, qr[t].y, xr[u][t].y);
                acc = term(acc, qr[t].z, xr[u][t].z);
                acc = term(acc, qr[t].w, xr[u][t].w);
              }
            }
            acc = group_sum<16>(acc, lane);
            if (c < cm && l16 == 0) rkeys[c0 + c] = make_key(ip ? -acc : acc, idr[u]);
          }
        }
        wave_sync();
        continue;
      }
      for (int j0 = 0; j0 < cm; j0 += 4) {  // 16 lanes per candidate
        const int c = j0 + (lane >> 4);
        float acc = 0.f;
        uint32_t id = 0;
        if (c < cm) {
          id = rids[c];
          const float4* x4 = reinterpret_cast<const float4*>(a.base_f32 + (size_t)id * a.d);
          for (int ch = l16; ch < d4; ch += 16) {
            const float4 x = x4[ch], qq = q4[ch];
            acc = term(acc, qq.x, x.x);
            acc = term(acc, qq.y, x.y);
            acc = term(acc, qq.z, x.z);
            acc = term(acc, qq.w, x.w);
          }
        }
        acc = group_sum<16>(acc, lane);
        if (c < cm && l16 == 0) rkeys[c0 + c] = make_key(ip ? -acc : acc, id);
      }
      wave_sync();
    }
    // rank sort: each key's slot is the number of smaller keys
    for (int i = lane; i < rr; i += 64) {
      const uint64_t ki = rkeys[i];
      int r = 0;
      for (int j = 0; j < rr; ++j) r += rkeys[j] < ki ? 1 : 0;
      stage[r] = ki;
    }
    wave_sync();
#pragma unroll
    for (int k = 0; k < PREG; ++k) {
      const int i = k * 64 + lane;
      pool[k] = i < rr ? stage[i] : kNoKey;
    }
    wave_sync();
  }

  // ---- output: first K pool entries, padded to the row stride
  uint32_t* oid = a.out_ids + (size_t)qid * a.kstride;
  float* od = a.out_d + (size_t)qid * a.kstride;
#pragma unroll
  for (int k = 0; k < PREG; ++k) {
    const int i = k * 64 + lane;
    if (i < a.kstride) {
      const uint64_t key = i < K ? pool[k] : kNoKey;
      oid[i] = key == kNoKey ? kSent : key_id(key);
      od[i] = key == kNoKey ? __uint_as_float(0x7F800000u) : unord_f32((uint32_t)(key >> 32));
    }
  }
  for (int i = LCAP + lane; i < a.kstride; i += 64) {
    oid[i] = kSent;
    od[i] = __uint_as_float(0x7F800000u);
  }
  if (lane == 0) {
    if (a.out_ndc) a.out_ndc[qid] = ndc;
    if (a.out_hops) a.out_hops[qid] = hops;
  }
  if (a.out_trace)
    for (int i = hops + lane; i < a.trace_cap; i += 64) a.out_trace[(size_t)qid * a.trace_cap + i] = kSent;
  wave_sync();  // LDS of this wave is reused by its next query
}

// One query per wavefront: query `slot` with the launch's L and K, or, with
// a query list (one L bucket of the batched form), query qlist[slot] with its
// own L_i and K_i clamped to the launch's pool capacity and row stride.
template <typename T, int DC, int G, int NP, int PREG, bool QL>
__global__ __launch_bounds__(256) void search_kernel(Args a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  unsigned char* my = smem + (size_t)wv * a.lds_per_wave;
  const int64_t slot = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
  int64_t qid = slot;
  int L = a.L, K = a.K;
  if (a.qlist) {
    if (slot >= a.nlist) return;  // uniform per wavefront
    qid = (int64_t)__builtin_amdgcn_readfirstlane((int)a.qlist[slot]);
    if (qid < 0 || qid >= a.nq) return;  // a bad list entry is skipped, never dereferenced
    L = __builtin_amdgcn_readfirstlane(min(max(a.L_arr ? a.L_arr[qid] : a.L, 1), 64 * PREG));
    K = __builtin_amdgcn_readfirstlane(min(max(a.K_arr ? a.K_arr[qid] : a.K, 1), a.kstride));
  } else if (slot >= a.nq) {
    return;
  }
  run_query<T, DC, G, NP, PREG, QL>(a, my, lane, qid, L, K);
}

// Persistent: every wavefront takes the next slot of the bucket's work queue
// until the queue is exhausted (each wavefront exits once its fetched slot is
// past the end).
template <typename T, int DC, int G, int NP, int PREG, bool QL>
__global__ __launch_bounds__(256) void search_kernel_batched(Args a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  unsigned char* my = smem + (size_t)wv * a.lds_per_wave;
  int64_t slot = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
  for (;;) {
    if (a.counter) {
      uint32_t s0 = 0u;
      if (lane == 0) s0 = atomicAdd(a.counter, 1u);
      slot = (int64_t)__builtin_amdgcn_readfirstlane(s0);
    }
    if (slot >= a.nlist) break;  // uniform per wavefront
    const int64_t qid = a.qlist ? (int64_t)__builtin_amdgcn_readfirstlane((int)a.qlist[slot]) : slot;
    if (qid >= 0 && qid < a.nq) {  // a bad queue entry is skipped, never dereferenced
      // per-query sizes are clamped to this launch's pool capacity and row stride
      const int L = __builtin_amdgcn_readfirstlane(min(max(a.L_arr ? a.L_arr[qid] : a.L, 1), 64 * PREG));
      const int K = __builtin_amdgcn_readfirstlane(min(max(a.K_arr ? a.K_arr[qid] : a.K, 1), a.kstride));
      run_query<T, DC, G, NP, PREG, QL>(a, my, lane, qid, L, K);
    }
    if (!a.counter) break;
  }
}

// ------------------------------------------------------------------ quantizer
// Storage forms for the precision variant of the search. Index preparation,
// run once per base set, not part of a query.
//   BF16: round-to-nearest-even of the upper 16 bits of each fp32 value.
//   FP8 : OCP E4M3 (bias 7, max 448, no infinities) codes of x / s_j with the
//         per-dimension scale s_j = max_i |x_ij| / 448 (1 if the column is 0),
//         round-to-nearest-even, saturating at +-448.
__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void absmax_cols_kernel(const float* x, int64_t n, int d, uint32_t* colmax) {
  const int j = blockIdx.y * blockDim.x + threadIdx.x;
  if (j >= d) return;
  float m = 0.f;
  for (int64_t i = blockIdx.x; i < n; i += gridDim.x) m = fmaxf(m, fabsf(x[(size_t)i * d + j]));
  atomicMax(&colmax[j], __float_as_uint(m));  // non-negative floats order like their bits
}

__global__ void scale_cols_kernel(float* s, int d) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d) return;
  const float m = __uint_as_float(__float_as_uint(s[j]));
  s[j] = m > 0.f ? __fdiv_rn(m, 448.f) : 1.f;
}

__device__ __forceinline__ uint32_t fp8_e4m3_rne(float v) {
  const uint32_t sgn = (__float_as_uint(v) >> 24) & 0x80u;
  const float a = fabsf(v);
  if (!(a < 448.f)) return sgn | 0x7Eu;
  if (a < 0.015625f) {  // below the smallest normal 2^-6: multiples of 2^-9
    const uint32_t m = (uint32_t)__builtin_rintf(a * 512.f);  // 8 rounds up to 2^-6 = code 0x08
    return sgn | m;
  }
  const uint32_t ua = __float_as_uint(a);
  int e = (int)(ua >> 23) - 127;
  uint32_t keep = (ua >> 20) & 7u;
  const uint32_t rest = ua & 0xFFFFFu;
  if (rest > 0x80000u || (rest == 0x80000u && (keep & 1u))) ++keep;
  if (keep == 8u) {
    keep = 0u;
    ++e;
  }
  const uint32_t mag = ((uint32_t)(e + 7) << 3) | keep;
  return sgn | (mag > 0x7Eu ? 0x7Eu : mag);
}

__global__ void encode_kernel(const float* x, int64_t n, int d, int dtype, const float* scale,
                              void* out) {
  const int64_t total = n * (int64_t)d;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float v = x[i];
    if (dtype == SSG_BF16) {
      const uint32_t u = __float_as_uint(v);
      static_cast<uint16_t*>(out)[i] = (uint16_t)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
    } else {
      const int j = (int)(i % d);
      static_cast<uint8_t*>(out)[i] = (uint8_t)fp8_e4m3_rne(__fdiv_rn(v, scale[j]));
    }
  }
}

// ------------------------------------------------------------------ gather probe
// Measurement aid: the search's memory access shape without the search. Each
// wavefront reads rows ids[i] (row_bytes each, 16-byte chunks spread over G
// lanes per row, 64/G rows per pass) and folds every word into a checksum so
// no load can be dropped; one word per wavefront is written.
template <int G>
__global__ __launch_bounds__(256) void gather_probe_kernel(const uint4* base, int chunks,
                                                           const uint32_t* ids, int64_t m,
                                                           int64_t per_wave, uint32_t* out) {
  const int lane = threadIdx.x & 63;
  const int64_t w = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int64_t lo = w * per_wave;
  const int64_t hi = min(m, lo + per_wave);
  uint32_t acc = 0u;
  for (int64_t r0 = lo; r0 < hi; r0 += 64 / G) {
    const int64_t r = r0 + lane / G;
    if (r < hi) {
      const uint4* row = base + (size_t)ids[r] * chunks;
      for (int c = lane % G; c < chunks; c += G) {
        const uint4 v = row[c];
        acc ^= v.x ^ v.y ^ v.z ^ v.w;
      }
    }
  }
  for (int off = 32; off >= 1; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
  if (lane == 0 && lo < m) out[w] = acc;
}

// ------------------------------------------------------------------ host side
// The calling thread's last error message: a fixed buffer, so that no call
// (the error paths included) allocates host memory.
struct ErrorText {
  char text[512] = {0};
  void clear() { text[0] = 0; }
  const char* c_str() const { return text; }
};
thread_local ErrorText g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err.text, sizeof g_err.text, fmt, ap);
  va_end(ap);
  return code;
}

struct Launch {
  KernelFn fn = nullptr;
  int preg = 0;
  bool query_in_regs = false;
};

template <typename T, int DC, int G, int NP, bool QL = false>
KernelFn pick_preg(int preg, bool batched) {
  if (batched) {
    switch (preg) {
      case 1: return search_kernel_batched<T, DC, G, NP, 1, QL>;
      case 2: return search_kernel_batched<T, DC, G, NP, 2, QL>;
      case 4: return search_kernel_batched<T, DC, G, NP, 4, QL>;
      default: return search_kernel_batched<T, DC, G, NP, 8, QL>;
    }
  }
  switch (preg) {
    case 1: return search_kernel<T, DC, G, NP, 1, QL>;
    case 2: return search_kernel<T, DC, G, NP, 2, QL>;
    case 4: return search_kernel<T, DC, G, NP, 4, QL>;
    default: return search_kernel<T, DC, G, NP, 8, QL>;
  }
}

// Launch tables: compile-time chunk counts for the dimensions of the paper's
// datasets (Table 2: 96, 100, 128, 300, 960) and of the tiny workload (32).
// G and NP set how many candidates' loads are in flight per wavefront
// (NP * 64 / G) and how many query floats a lane keeps in registers
// (EPC * DC / G). `variant` selects alternative gather shapes for tuning;
// shapes not listed use the runtime-chunk kernel (query in LDS).
template <typename T>
struct Table;
template <>
struct Table<F32T> {
  static Launch pick(int dc, int preg, int variant, bool batched) {
    Launch l{nullptr, preg, true};
    switch (dc) {
      case 8: l.fn = pick_preg<F32T, 8, 2, 1>(preg, batched); return l;    // d = 32: 32 in flight
      case 24: l.fn = pick_preg<F32T, 24, 4, 1>(preg, batched); return l;  // d = 96: 16
      case 25: l.fn = pick_preg<F32T, 25, 4, 1>(preg, batched); return l;  // d = 100: 16
      case 32:                                                     // d = 128
        switch (variant) {
          case 1: l.fn = pick_preg<F32T, 32, 8, 1>(preg, batched); return l;  // 8 in flight
          case 2: l.fn = pick_preg<F32T, 32, 4, 1>(preg, batched); return l;  // 16
          case 3: l.fn = pick_preg<F32T, 32, 4, 2>(preg, batched); return l;  // 32
          case 4: l.query_in_regs = false; l.fn = pick_preg<F32T, 32, 4, 1, true>(preg, batched); return l;
          case 5: l.query_in_regs = false; l.fn = pick_preg<F32T, 32, 4, 2, true>(preg, batched); return l;
          case 6: l.query_in_regs = false; l.fn = pick_preg<F32T, 32, 8, 2, true>(preg, batched); return l;
          // 8 lanes per candidate, 2 passes (16 in flight): the staged pass
          // stays within 120 VGPRs (4 waves per SIMD) at L <= 256
          default: l.fn = pick_preg<F32T, 32, 8, 2>(preg, batched); return l;
        }
      case 75: l.fn = pick_preg<F32T, 75, 16, 2>(preg, batched); return l;  // d = 300: 8
      case 240: l.fn = pick_preg<F32T, 240, 32, 4>(preg, batched); return l;  // d = 960: 8
      default: break;
    }
    l.query_in_regs = false;
    l.fn = pick_preg<F32T, 0, 16, 2>(preg, batched);
    return l;
  }
};
template <>
struct Table<BF16T> {
  static Launch pick(int dc, int preg, int variant, bool batched) {
    Launch l{nullptr, preg, true};
    switch (dc) {
      case 12:                                                             // d = 96
        if (variant == 4) { l.query_in_regs = false; l.fn = pick_preg<BF16T, 12, 4, 1, true>(preg, batched); return l; }
        l.fn = pick_preg<BF16T, 12, 4, 1>(preg, batched); return l;
      case 16:                                                      // d = 128
        switch (variant) {
          case 2: l.fn = pick_preg<BF16T, 16, 4, 1>(preg, batched); return l;  // 16 in flight
          case 3: l.fn = pick_preg<BF16T, 16, 4, 2>(preg, batched); return l;
          case 4: l.query_in_regs = false; l.fn = pick_preg<BF16T, 16, 4, 1, true>(preg, batched); return l;
          // 16 lanes per candidate, 2 passes (8 in flight): 80 VGPRs, so 6
          // wavefronts per SIMD when the visited cache is 4 KB (hash_log2 11)
          case 7: l.fn = pick_preg<BF16T, 16, 16, 2>(preg, batched); return l;
          case 8: l.fn = pick_preg<BF16T, 16, 8, 1>(preg, batched); return l;  // 8 in flight, 82 VGPRs
          // 8 lanes per candidate, 2 passes (16 in flight): measured 1.10 ms
          // against 1.16 ms for the 4-lane shape on 10,000 queries of 1M x 128
          default: l.fn = pick_preg<BF16T, 16, 8, 2>(preg, batched); return l;
        }
      case 120: l.fn = pick_preg<BF16T, 120, 32, 4>(preg, batched); return l;  // d = 960: 8
      default: break;
    }
    l.query_in_regs = false;
    l.fn = pick_preg<BF16T, 0, 16, 2>(preg, batched);
    return l;
  }
};
template <typename F>
struct Fp8Table {
  static Launch pick(int dc, int preg, bool batched, int wide = 0) {
    Launch l{nullptr, preg, true};
    switch (dc) {
      case 6: l.fn = pick_preg<F, 6, 4, 1>(preg, batched); return l;  // d = 96
      case 8:                                                          // d = 128
        // 8 lanes per candidate in 2 passes (16 in flight): a lane holds 16
        // query values and 16 scales instead of 32 each, so the kernel fits
        // 4 waves per SIMD (measured 1.00 against 1.08 ms on 1M x 128)
        if (wide == 2) { l.fn = pick_preg<F, 8, 8, 1>(preg, batched); return l; }  // 8 in flight, 94 VGPRs
        if (wide) { l.fn = pick_preg<F, 8, 8, 2>(preg, batched); return l; }
        l.fn = pick_preg<F, 8, 4, 1>(preg, batched); return l;
      case 60: l.fn = pick_preg<F, 60, 32, 4>(preg, batched); return l;  // d = 960: 8
      default: break;
    }
    l.query_in_regs = false;
    l.fn = pick_preg<F, 0, 16, 2>(preg, batched);
    return l;
  }
};
// FP8: the conversion instruction by default (checked code by code against the
// format definition); variant 1 keeps the bit-placement decode, variant 2 the
// 4-lane, one-pass gather shape, variant 3 the 8-lane one-pass shape
template <>
struct Table<FP8T> {
  static Launch pick(int dc, int preg, int variant, bool batched) {
    return variant == 1 ? Fp8Table<FP8T>::pick(dc, preg, batched)
                        : Fp8Table<FP8HwT>::pick(dc, preg, batched, variant == 3 ? 2 : variant == 2 ? 0 : 1);
  }
};

int check_common(const void* base, int64_t n, int32_t d, int32_t dtype, const float* dim_scale,
                 const uint32_t* graph, int32_t R, const uint32_t* entry_ids, int32_t n_entry,
                 const float* queries, int64_t nq, int32_t K, int32_t L, int32_t metric,
                 uint32_t* out_ids, float* out_dists) {
  if (nq < 0) return fail(SSG_EINVAL, "nq must be >= 0 (got %lld)", (long long)nq);
  if (n < 1 || n >= (int64_t)0x7FFFFFFF) return fail(SSG_EINVAL, "n must be in [1, 2^31-1) (got %lld)", (long long)n);
  if (d < 1) return fail(SSG_EINVAL, "d must be >= 1 (got %d)", d);
  if (R < 1) return fail(SSG_EINVAL, "R must be >= 1 (got %d)", R);
  if (n_entry < 1 || n_entry > 4096) return fail(SSG_EINVAL, "n_entry must be in [1, 4096] (got %d)", n_entry);
  if (K < 1) return fail(SSG_EINVAL, "K must be >= 1 (got %d)", K);
  if (L < 1) return fail(SSG_EINVAL, "L must be >= 1 (got %d)", L);
  if (metric != SSG_L2 && metric != SSG_IP) return fail(SSG_EINVAL, "unknown metric %d", metric);
  if (dtype != SSG_F32 && dtype != SSG_BF16 && dtype != SSG_FP8E4M3)
    return fail(SSG_EINVAL, "unknown dtype %d", dtype);
  if (!base || !graph || !entry_ids || (nq > 0 && (!queries || !out_ids || !out_dists)))
    return fail(SSG_EINVAL, "required pointer is NULL");
  if (dtype == SSG_FP8E4M3 && !dim_scale) return fail(SSG_EINVAL, "FP8 vectors need dim_scale");
  if (reinterpret_cast<uintptr_t>(base) % 16 || reinterpret_cast<uintptr_t>(queries) % 16)
    return fail(SSG_EINVAL, "base and queries must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(graph) % 4 || reinterpret_cast<uintptr_t>(entry_ids) % 4)
    return fail(SSG_EINVAL, "graph and entry_ids must be 4-byte aligned");
  const int epc = dtype == SSG_F32 ? 4 : dtype == SSG_BF16 ? 8 : 16;
  if (d % epc) return fail(SSG_EUNSUPPORTED, "d=%d must be a multiple of %d for this dtype", d, epc);
  if (d % 4) return fail(SSG_EUNSUPPORTED, "d must be a multiple of 4");
  if (R > SSG_R_MAX) return fail(SSG_EUNSUPPORTED, "R=%d exceeds %d", R, SSG_R_MAX);
  if (L > SSG_L_MAX) return fail(SSG_EUNSUPPORTED, "L=%d exceeds %d", L, SSG_L_MAX);
  if (K > SSG_K_MAX) return fail(SSG_EUNSUPPORTED, "K=%d exceeds %d", K, SSG_K_MAX);
  return SSG_OK;
}

int preg_for(int L) { return L <= 64 ? 1 : L <= 128 ? 2 : L <= 256 ? 4 : 8; }

Launch pick_launch(int dtype, int dc, int preg, int variant, bool batched) {
  return dtype == SSG_F32    ? Table<F32T>::pick(dc, preg, variant, batched)
         : dtype == SSG_BF16 ? Table<BF16T>::pick(dc, preg, variant, batched)
                             : Table<FP8T>::pick(dc, preg, variant, batched);
}

// LDS bytes per wavefront and the visited form for a pool capacity of 64*preg.
// kind: 0 = the tag cache where a 16-bit tag holds the ids, else the hash;
// 1 = hash; 2 = cache (fails when the ids do not fit); 3 = exact bitset.
struct VisitedPlan {
  int vmode = 1, hash_log2 = 0, id_bits = 0;
  size_t per_wave = 0;
};
int lds_layout(int preg, int R, int d, bool query_in_regs, int dtype, int kind, int64_t n,
               bool rerank, int hash_log2_req, VisitedPlan* vp) {
  const int lcap = 64 * preg;
  size_t fixed = (size_t)lcap * 8 + 64 * 8 + 64 * 4 +
                 (query_in_regs ? 0 : (size_t)d * 4 * (dtype == SSG_FP8E4M3 ? 2 : 1));
  size_t table;
  if (kind < 0 || kind > 3) return fail(SSG_EINVAL, "visited_kind must be in [0, 3]");
  if (kind == 3) {
    if (n > SSG_EXACT_VISITED_MAX_N)
      return fail(SSG_EUNSUPPORTED, "exact visited set needs n <= %d", SSG_EXACT_VISITED_MAX_N);
    table = (size_t)((n + 31) / 32) * 4;
    vp->vmode = 0;
    vp->hash_log2 = 0;
  } else {
    // default size: 4096 entries (8 KB as a tag cache), fastest for FP32,
    // BF16 and FP8 vectors on the 1M x 128 workload
    int hl = hash_log2_req > 0 ? hash_log2_req : 12;
    if (hl < 4 || hl > 15) return fail(SSG_EINVAL, "hash_log2 must be in [4, 15]");
    int k = 0;
    while (k < 32 && ((uint64_t)1 << k) < (uint64_t)n) ++k;  // every id < 2^k
    k = std::max(k, hl - 2);
    const bool fits = k - (hl - 2) <= 15;
    if (kind == 2 && !fits)
      return fail(SSG_EUNSUPPORTED, "visited cache: ids of n = %lld need tags over 16 bits at hash_log2 %d",
                  (long long)n, hl);
    vp->vmode = kind == 1 || !fits ? 1 : 2;
    if (vp->vmode == 1) {
      // the hash must hold the pool plus one row at load <= 1/2; the cache has
      // no such need (a small one forgets more and recomputes more)
      while ((1 << hl) < 2 * (lcap + R) + 64) ++hl;
      if (hl > 15) return fail(SSG_EINVAL, "hash_log2 too large");
    }
    vp->hash_log2 = hl;
    vp->id_bits = vp->vmode == 2 ? k : 0;
    table = vp->vmode == 2 ? (size_t)2 << hl : (size_t)4 << hl;
  }
  if (rerank) table = std::max(table, (size_t)lcap * 8);  // the rerank reuses it for keys
  vp->per_wave = (fixed + table + 15) & ~(size_t)15;
  return SSG_OK;
}

// Launch with two queries per wavefront (32 lanes each, ssg_groups.hip).
// want: the caller's queries_per_wave (0 = the library's choice, 1, 2).
// On success gp->fn is the kernel, or null when the one-query form runs
// (want 1, or want 0 and the default or the shape says so); a shape that
// cannot run grouped is an error only when the caller asked for 2.
// vp->per_wave is the bytes of ONE query's LDS region.
struct GroupPlan {
  KernelFn fn = nullptr;
  int preg = 0;
  VisitedPlan vp;
};
int group_preg_for(int L) { return L <= 64 ? 2 : L <= 96 ? 3 : L <= 128 ? 4 : L <= 256 ? 8 : 0; }
int default_queries_per_wave(int dtype) {
  (void)dtype;
  return 1;
}
int plan_groups(int want, int dtype, int dc, int L, int kind, int64_t n, bool rerank, int hl_req,
                bool batched, GroupPlan* gp) {
  gp->fn = nullptr;
  if (want < 0 || want > 2) return fail(SSG_EINVAL, "queries_per_wave must be 0, 1 or 2");
  if (want == 1 || (want == 0 && default_queries_per_wave(dtype) == 1)) return SSG_OK;
  auto no = [&](const char* why) {
    return want == 2 ? fail(SSG_EUNSUPPORTED, "two queries per wavefront: %s", why) : SSG_OK;
  };
  if (kind == 1 || kind == 3) return no("needs the tag-cache visited set");
  const int preg = group_preg_for(L);
  if (preg == 0) return no("needs L <= 256");
  KernelFn fn = ssg_internal_group_kernel(dtype, dc, preg, 32, batched);
  if (!fn) return no("no compiled shape for this dtype and dimension");
  // default 2048 entries (4 KB): with two queries per wavefront LDS, not
  // registers, bounds how many searches a compute unit holds
  const int hl = hl_req > 0 ? hl_req : 11;
  if (hl < 4 || hl > 15) return fail(SSG_EINVAL, "hash_log2 must be in [4, 15]");
  int k = 0;
  while (k < 32 && ((uint64_t)1 << k) < (uint64_t)n) ++k;
  k = std::max(k, hl - 2);
  if (k - (hl - 2) > 15) return no("the ids need visited-cache tags over 16 bits");
  const int lcap = 32 * preg;
  size_t table = (size_t)2 << hl;
  if (rerank) table = std::max(table, (size_t)lcap * 8);
  gp->fn = fn;
  gp->preg = preg;
  gp->vp.vmode = 2;
  gp->vp.hash_log2 = hl;
  gp->vp.id_bits = k;
  gp->vp.per_wave = ((size_t)lcap * 8 + 64 * 8 + 64 * 4 + table + 15) & ~(size_t)15;
  return SSG_OK;
}


}  // namespace

int ssg_internal_fail(int code, const char* msg) { return fail(code, "%s", msg); }
void ssg_internal_clear_error() { g_err.clear(); }

extern "C" {

const char* ssg_last_error(void) { return g_err.c_str(); }

const char* ssg_version(void) { return "libssg 0.1 gfx950"; }

size_t ssg_search_workspace_bytes(int64_t, int64_t, int32_t, int32_t, int32_t) { return 0; }

size_t ssg_query_lds_bytes(int32_t L, int32_t R, int32_t d, int32_t dtype, int64_t n, int32_t rerank,
                           int32_t hash_log2) {
  if (L < 1 || L > SSG_L_MAX || R < 1 || R > SSG_R_MAX || d < 1 || n < 1) return 0;
  if (dtype != SSG_F32 && dtype != SSG_BF16 && dtype != SSG_FP8E4M3) return 0;
  const int epc = dtype == SSG_F32 ? 4 : dtype == SSG_BF16 ? 8 : 16;
  if (d % epc) return 0;
  const int preg = preg_for(L);
  const Launch lc = pick_launch(dtype, d / epc, preg, 0, true);
  VisitedPlan vp;
  const ErrorText keep = g_err;  // a size query leaves the error message alone
  const int rc = lds_layout(preg, R, d, lc.query_in_regs, dtype, 0, n, rerank != 0, hash_log2, &vp);
  g_err = keep;
  return rc ? 0 : vp.per_wave;
}

int ssg_validate_graph(const uint32_t* graph, int64_t n, int32_t R) {
  if (!graph || n < 1 || R < 1) return fail(SSG_EINVAL, "bad graph arguments");
  std::string seen;
  for (int64_t i = 0; i < n; ++i) {
    const uint32_t* row = graph + (size_t)i * R;
    bool tail = false;
    for (int t = 0; t < R; ++t) {
      const uint32_t v = row[t];
      if (v == kSent) { tail = true; continue; }
      if (tail) return fail(SSG_EINVAL, "row %lld: id after padding at slot %d", (long long)i, t);
      if (v >= (uint64_t)n) return fail(SSG_EINVAL, "row %lld: id %u >= n", (long long)i, v);
      if (v == (uint64_t)i) return fail(SSG_EINVAL, "row %lld: self loop", (long long)i);
      for (int u = 0; u < t; ++u)
        if (row[u] == v) return fail(SSG_EINVAL, "row %lld: duplicate id %u", (long long)i, v);
    }
  }
  g_err.clear();
  return SSG_OK;
}

int ssg_search_ex(const void* base, int64_t n, int32_t d, int32_t dtype, const float* dim_scale,
                  const uint32_t* graph, int32_t R, const uint32_t* entry_ids, int32_t n_entry,
                  const float* queries, int64_t nq, int32_t K, int32_t L, int32_t metric,
                  uint32_t* out_ids, float* out_dists, const ssg_search_opts* opts,
                  void* stream) {
  int rc = check_common(base, n, d, dtype, dim_scale, graph, R, entry_ids, n_entry, queries, nq, K,
                        L, metric, out_ids, out_dists);
  if (rc) return rc;
  ssg_search_opts o{};
  if (opts) o = *opts;
  if (nq == 0) { g_err.clear(); return SSG_OK; }
  const int preg = preg_for(L);
  const int epc = dtype == SSG_F32 ? 4 : dtype == SSG_BF16 ? 8 : 16;
  const int dc = d / epc;
  Launch lc = pick_launch(dtype, dc, preg, o.gather_variant, false);
  // one wavefront per workgroup measured fastest on the 1M x 128 workload
  // (finer-grained dispatch, no LDS fragmentation across waves)
  int wpb = o.waves_per_block > 0 ? o.waves_per_block : 1;
  if (wpb > 4) return fail(SSG_EINVAL, "waves_per_block must be in [1, 4]");
  Args a{};
  a.base = static_cast<const unsigned char*>(base);
  a.n = n;
  a.d = d;
  a.dc = dc;
  a.dim_scale = dtype == SSG_FP8E4M3 ? dim_scale : nullptr;
  a.graph = graph;
  a.R = R;
  a.entry = entry_ids;
  a.s = n_entry;
  a.queries = queries;
  a.nq = nq;
  a.K = K;
  a.L = L;
  a.metric = metric;
  a.out_ids = out_ids;
  a.out_d = out_dists;
  a.out_ndc = o.out_ndc;
  a.out_hops = o.out_hops;
  a.qlist = nullptr;
  a.nlist = nq;
  a.L_arr = nullptr;
  a.K_arr = nullptr;
  a.kstride = K;
  a.counter = nullptr;
  if (o.entry_group_size < 0) return fail(SSG_EINVAL, "entry_group_size must be >= 0");
  a.entry_group = o.entry_group_size;
  if (o.trace_cap < 0 || (o.out_trace && o.trace_cap < 1))
    return fail(SSG_EINVAL, "out_trace needs trace_cap >= 1");
  a.out_trace = o.trace_cap > 0 ? o.out_trace : nullptr;
  a.trace_cap = o.trace_cap;
  a.base_f32 = o.base_f32;
  a.rerank = 0;
  if (o.base_f32) {
    if (reinterpret_cast<uintptr_t>(o.base_f32) % 16)
      return fail(SSG_EINVAL, "base_f32 must be 16-byte aligned");
    if (o.rerank_k < 0) return fail(SSG_EINVAL, "rerank_k must be >= 0");
    a.rerank = std::min(std::max(o.rerank_k, K), L);
  }
  const int kind = o.exact_visited ? 3 : o.visited_kind;
  if (kind < 0 || kind > 3) return fail(SSG_EINVAL, "visited_kind must be in [0, 3]");
  GroupPlan gp;
  rc = plan_groups(o.queries_per_wave, dtype, dc, L, kind, n, o.base_f32 != nullptr, o.hash_log2,
                   false, &gp);
  if (rc) return rc;
  VisitedPlan vp = gp.vp;
  int qpw = 1;
  if (gp.fn) {
    lc.fn = gp.fn;
    qpw = 2;
  } else {
    rc = lds_layout(preg, R, d, lc.query_in_regs, dtype, kind, n, o.base_f32 != nullptr, o.hash_log2,
                    &vp);
    if (rc) return rc;
  }
  a.vmode = vp.vmode;
  a.hash_log2 = vp.hash_log2;
  a.id_bits = vp.id_bits;
  const size_t per_wave = vp.per_wave * qpw;  // a grouped launch: one region per query
  if (per_wave * wpb > 64 * 1024) {
    wpb = (int)((64 * 1024) / per_wave);
    if (wpb < 1) return fail(SSG_EUNSUPPORTED, "per-query LDS need %zu exceeds the CU", per_wave);
  }
  a.lds_per_wave = (int)vp.per_wave;
  const size_t lds = per_wave * wpb;
  hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t per_block = (int64_t)wpb * qpw;
  const int64_t blocks = (nq + per_block - 1) / per_block;
  if (blocks > 0x7FFFFFFF) return fail(SSG_EINVAL, "too many queries");
  hipLaunchKernelGGL(lc.fn, dim3((unsigned)blocks), dim3(64 * wpb), lds, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SSG_EDEVICE, "launch: %s", hipGetErrorString(e));
  g_err.clear();
  return SSG_OK;
}

int ssg_probe_gather(const void* base, int64_t n, int32_t row_bytes, const uint32_t* ids,
                     int64_t m, int32_t rows_per_wave, uint32_t* out, void* stream) {
  if (!base || !ids || !out || n < 1 || m < 0 || rows_per_wave < 1)
    return fail(SSG_EINVAL, "bad probe arguments");
  if (row_bytes < 16 || row_bytes % 16 || reinterpret_cast<uintptr_t>(base) % 16)
    return fail(SSG_EINVAL, "row_bytes must be a positive multiple of 16, base 16-byte aligned");
  if (m == 0) { g_err.clear(); return SSG_OK; }
  const int chunks = row_bytes / 16;
  const int64_t waves = (m + rows_per_wave - 1) / rows_per_wave;
  const int64_t blocks = (waves + 3) / 4;
  if (blocks > 0x7FFFFFFF) return fail(SSG_EINVAL, "too many rows");
  hipStream_t st = static_cast<hipStream_t>(stream);
  const uint4* b = static_cast<const uint4*>(base);
  if (chunks >= 32)
    hipLaunchKernelGGL(gather_probe_kernel<8>, dim3((unsigned)blocks), dim3(256), 0, st, b, chunks,
                       ids, m, (int64_t)rows_per_wave, out);
  else
    hipLaunchKernelGGL(gather_probe_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, st, b, chunks,
                       ids, m, (int64_t)rows_per_wave, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SSG_EDEVICE, "launch: %s", hipGetErrorString(e));
  g_err.clear();
  return SSG_OK;
}

int ssg_quantize(const float* base_f32, int64_t n, int32_t d, int32_t dtype, float* dim_scale,
                 void* out, void* stream) {
  if (!base_f32 || !out || n < 1 || d < 1) return fail(SSG_EINVAL, "bad quantize arguments");
  if (dtype != SSG_BF16 && dtype != SSG_FP8E4M3)
    return fail(SSG_EINVAL, "quantize supports SSG_BF16 and SSG_FP8E4M3");
  if (dtype == SSG_FP8E4M3 && !dim_scale) return fail(SSG_EINVAL, "FP8 needs dim_scale");
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (dtype == SSG_FP8E4M3) {
    uint32_t* cm = reinterpret_cast<uint32_t*>(dim_scale);
    hipLaunchKernelGGL(fill_u32_kernel, dim3((d + 255) / 256), dim3(256), 0, st, cm, 0u, (int64_t)d);
    const int rows = (int)std::min<int64_t>(n, 2048);
    hipLaunchKernelGGL(absmax_cols_kernel, dim3(rows, (d + 255) / 256), dim3(256), 0, st, base_f32,
                       n, d, cm);
    hipLaunchKernelGGL(scale_cols_kernel, dim3((d + 255) / 256), dim3(256), 0, st, dim_scale, d);
  }
  const int64_t total = n * (int64_t)d;
  const int blocks = (int)std::min<int64_t>((total + 255) / 256, 65536);
  hipLaunchKernelGGL(encode_kernel, dim3(blocks), dim3(256), 0, st, base_f32, n, d, dtype,
                     dim_scale, out);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SSG_EDEVICE, "launch: %s", hipGetErrorString(e));
  g_err.clear();
  return SSG_OK;
}

}  // extern "C"

namespace {

struct BucketLaunch {
  KernelFn fn;
  Args a;
  unsigned blocks;
  unsigned threads;
  size_t lds;
  uint32_t* counter;
};

constexpr int kMaxBuckets = 64;

// Checks a batched call and fills out[0..nb) (capacity kMaxBuckets).
int prepare_batched(const ssg_batch_desc* D, const ssg_bucket* B, int nb, void* ws, size_t wsb,
                    BucketLaunch* out) {
  if (!D || !B) return fail(SSG_EINVAL, "descriptor or buckets is NULL");
  if (nb < 1 || nb > kMaxBuckets) return fail(SSG_EINVAL, "nb must be in [1, %d] (got %d)", kMaxBuckets, nb);
  if (!ws || wsb < ssg_batch_workspace_bytes(nb) || reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(SSG_ENOMEM, "workspace must be 256-byte aligned and hold %zu bytes",
                ssg_batch_workspace_bytes(nb));
  int maxL = 1;
  for (int i = 0; i < nb; ++i) maxL = std::max(maxL, B[i].max_L);
  int rc = check_common(D->base, D->n, D->d, D->dtype, D->dim_scale, D->graph, D->R, D->entry_ids,
                        D->n_entry, D->queries, D->nq, D->kstride, maxL, D->metric, D->out_ids,
                        D->out_dists);
  if (rc) return rc;
  if (D->nq > 0 && (!D->L || !D->K)) return fail(SSG_EINVAL, "per-query L and K arrays are required");
  if (D->rerank < -16) return fail(SSG_EINVAL, "rerank must be in [-16, -1], 0 or positive");
  if (D->rerank != 0 && !D->base_f32) return fail(SSG_EINVAL, "rerank needs base_f32");
  if (D->base_f32 && reinterpret_cast<uintptr_t>(D->base_f32) % 16)
    return fail(SSG_EINVAL, "base_f32 must be 16-byte aligned");
  if (D->trace_cap < 0 || (D->out_trace && D->trace_cap < 1))
    return fail(SSG_EINVAL, "out_trace needs trace_cap >= 1");
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return fail(SSG_EDEVICE, "cannot query the device");
  const int epc = D->dtype == SSG_F32 ? 4 : D->dtype == SSG_BF16 ? 8 : 16;
  const int dc = D->d / epc;
  for (int i = 0; i < nb; ++i) {
    const ssg_bucket& b = B[i];
    if (b.count < 0 || (b.count > 0 && !b.qlist)) return fail(SSG_EINVAL, "bucket %d: bad query list", i);
    if (b.max_L < 1 || b.max_L > SSG_L_MAX) return fail(SSG_EUNSUPPORTED, "bucket %d: max_L %d", i, b.max_L);
    if (b.waves_per_block < 0 || b.waves_per_block > 4 || b.blocks < 0)
      return fail(SSG_EINVAL, "bucket %d: bad launch shape", i);
    const int preg = preg_for(b.max_L);
    // blocks == 0: one wavefront per listed query (the plain kernel reading
    // the list; the hardware starts the next query as a search ends); > 0: a
    // persistent grid of that many workgroups pulling from the work queue
    const bool per_query = b.blocks == 0;
    Launch lc = pick_launch(D->dtype, dc, preg, b.gather_variant, !per_query);
    BucketLaunch bl{};
    Args& a = bl.a;
    if (b.visited_kind < 0 || b.visited_kind > 2)
      return fail(SSG_EINVAL, "bucket %d: visited_kind must be 0, 1 or 2", i);
    GroupPlan gp;
    rc = plan_groups(b.queries_per_wave, D->dtype, dc, b.max_L, b.visited_kind, D->n,
                     D->base_f32 != nullptr, b.hash_log2, true, &gp);
    if (rc) return rc;
    VisitedPlan vp = gp.vp;
    int qpw = 1;
    if (gp.fn) {
      lc.fn = gp.fn;
      qpw = 2;
    } else {
      rc = lds_layout(preg, D->R, D->d, lc.query_in_regs, D->dtype, b.visited_kind, D->n,
                      D->base_f32 != nullptr, b.hash_log2, &vp);
      if (rc) return rc;
    }
    a.vmode = vp.vmode;
    a.hash_log2 = vp.hash_log2;
    a.id_bits = vp.id_bits;
    const size_t per_wave = vp.per_wave * qpw;
    int wpb = b.waves_per_block > 0 ? b.waves_per_block : 1;
    while (wpb > 1 && per_wave * wpb > 64 * 1024) --wpb;
    if (per_wave > 64 * 1024) return fail(SSG_EUNSUPPORTED, "bucket %d: LDS need too large", i);
    a.base = static_cast<const unsigned char*>(D->base);
    a.n = D->n;
    a.d = D->d;
    a.dc = dc;
    a.dim_scale = D->dtype == SSG_FP8E4M3 ? D->dim_scale : nullptr;
    a.graph = D->graph;
    a.R = D->R;
    a.entry = D->entry_ids;
    a.s = D->n_entry;
    a.queries = D->queries;
    a.nq = D->nq;
    a.K = D->kstride;
    a.L = b.max_L;
    a.metric = D->metric;
    a.out_ids = D->out_ids;
    a.out_d = D->out_dists;
    a.out_ndc = D->out_ndc;
    a.out_hops = D->out_hops;
    a.lds_per_wave = (int)vp.per_wave;
    a.base_f32 = D->rerank != 0 ? D->base_f32 : nullptr;
    a.rerank = D->rerank;
    a.qlist = b.qlist;
    a.nlist = b.count;
    a.L_arr = D->L;
    a.K_arr = D->K;
    a.kstride = D->kstride;
    a.out_trace = D->trace_cap > 0 ? D->out_trace : nullptr;
    a.trace_cap = D->trace_cap;
    bl.counter = reinterpret_cast<uint32_t*>(static_cast<unsigned char*>(ws) + (size_t)i * 256);
    a.counter = bl.counter;
    bl.fn = lc.fn;
    bl.threads = 64u * wpb;
    bl.lds = per_wave * wpb;
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(lc.fn),
                                                     (int)bl.threads, bl.lds) != hipSuccess ||
        per_cu < 1)
      per_cu = 1;
    const int64_t need = (b.count + (int64_t)wpb * qpw - 1) / ((int64_t)wpb * qpw);
    int64_t want = b.blocks > 0 ? b.blocks : (int64_t)per_cu * cus;
    if (per_query && qpw == 1) want = need;
    bl.blocks = (unsigned)std::max<int64_t>(1, std::min(want, std::max<int64_t>(need, 1)));
    out[i] = bl;
  }
  return SSG_OK;
}

void enqueue_bucket(const BucketLaunch& bl, hipStream_t st) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(1), dim3(64), 0, st, bl.counter, 0u, (int64_t)1);
  hipLaunchKernelGGL(bl.fn, dim3(bl.blocks), dim3(bl.threads), bl.lds, st, bl.a);
}

}  // namespace

// Work-queue counters of ssg_search_batched_noalloc: one 256-byte slot per
// bucket, at most kMaxBuckets buckets. Every device the library runs on holds
// its own copy until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returns on that device.
static __device__ __align__(256) unsigned char scratch[SSG_NOALLOC_SCRATCH_BYTES];
static_assert(SSG_NOALLOC_SCRATCH_BYTES == kMaxBuckets * 256, "one counter slot per bucket");

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(SSG_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(SSG_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SSG_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SSG_OK;
}

}  // namespace

struct ssg_batch_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

extern "C" {

size_t ssg_batch_workspace_bytes(int32_t nb) { return (size_t)std::max(nb, 0) * 256; }

int ssg_search_batched(const ssg_batch_desc* desc, const ssg_bucket* buckets, int32_t nb,
                       void* workspace, size_t workspace_bytes, void* stream) {
  BucketLaunch bl[kMaxBuckets];
  int rc = prepare_batched(desc, buckets, nb, workspace, workspace_bytes, bl);
  if (rc) return rc;
  if (desc->nq == 0) { g_err.clear(); return SSG_OK; }
  hipStream_t st = static_cast<hipStream_t>(stream);
  for (int i = 0; i < nb; ++i) enqueue_bucket(bl[i], st);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(SSG_EDEVICE, "launch: %s", hipGetErrorString(e));
  g_err.clear();
  return SSG_OK;
}

int ssg_search_batched_noalloc(const ssg_batch_desc* desc, const ssg_bucket* buckets, int32_t nb,
                               void* stream) {
  if (nb < 1 || nb > kMaxBuckets)
    return fail(SSG_EINVAL, "nb must be in [1, %d] (got %d): the counters live in a %d-byte array",
                kMaxBuckets, nb, SSG_NOALLOC_SCRATCH_BYTES);
  void* ws = nullptr;
  const int rc = scratch_address(&ws);
  if (rc) return rc;
  return ssg_search_batched(desc, buckets, nb, ws, ssg_batch_workspace_bytes(nb), stream);
}

int ssg_batch_graph_create(ssg_batch_graph** out, const ssg_batch_desc* desc,
                           const ssg_bucket* buckets, int32_t nb, void* workspace,
                           size_t workspace_bytes) {
  if (!out) return fail(SSG_EINVAL, "out is NULL");
  *out = nullptr;
  BucketLaunch bl[kMaxBuckets];
  int rc = prepare_batched(desc, buckets, nb, workspace, workspace_bytes, bl);
  if (rc) return rc;
  hipStream_t cap = nullptr;
  std::vector<hipStream_t> br(nb, nullptr);
  std::vector<hipEvent_t> join(nb, nullptr);
  hipEvent_t fork = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipStreamCreateWithFlags(&br[i], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&fork, hipEventDisableTiming);
  for (int i = 0; i < nb && e == hipSuccess; ++i) e = hipEventCreateWithFlags(&join[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    // record every step; the first failure is reported after the capture ends
    hipError_t ce = hipEventRecord(fork, cap);
    for (int i = 0; i < nb; ++i) {
      if (ce == hipSuccess) ce = hipStreamWaitEvent(br[i], fork, 0);
      if (ce == hipSuccess && desc->nq > 0) enqueue_bucket(bl[i], br[i]);
      if (ce == hipSuccess) ce = hipEventRecord(join[i], br[i]);
      if (ce == hipSuccess) ce = hipStreamWaitEvent(cap, join[i], 0);
    }
    const hipError_t le = hipGetLastError();
    e = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess && ce != hipSuccess) e = ce;
    if (e == hipSuccess && le != hipSuccess) e = le;
  }
  if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  for (int i = 0; i < nb; ++i) {
    if (join[i]) (void)hipEventDestroy(join[i]);
    if (br[i]) (void)hipStreamDestroy(br[i]);
  }
  if (fork) (void)hipEventDestroy(fork);
  if (cap) (void)hipStreamDestroy(cap);
  if (e != hipSuccess) {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    return fail(SSG_EDEVICE, "graph capture: %s", hipGetErrorString(e));
  }
  auto* g = new (std::nothrow) ssg_batch_graph;
  if (!g) {
    hipGraphExecDestroy(exec);
    hipGraphDestroy(graph);
    return fail(SSG_ENOMEM, "out of host memory");
  }
  g->graph = graph;
  g->exec = exec;
  *out = g;
  g_err.clear();
  return SSG_OK;
}

int ssg_batch_graph_launch(ssg_batch_graph* g, void* stream) {
  if (!g || !g->exec) return fail(SSG_EINVAL, "graph is NULL");
  hipError_t e = hipGraphLaunch(g->exec, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(SSG_EDEVICE, "hipGraphLaunch: %s", hipGetErrorString(e));
  g_err.clear();
  return SSG_OK;
}

int ssg_batch_graph_destroy(ssg_batch_graph* g) {
  if (!g) return SSG_OK;
  if (g->exec) hipGraphExecDestroy(g->exec);
  if (g->graph) hipGraphDestroy(g->graph);
  delete g;
  g_err.clear();
  return SSG_OK;
}

int ssg_search(const void* base, int64_t n, int32_t d, int32_t dtype, const float* dim_scale,
               const uint32_t* graph, int32_t R, const uint32_t* entry_ids, int32_t n_entry,
               const float* queries, int64_t nq, int32_t K, int32_t L, int32_t metric,
               uint32_t* out_ids, float* out_dists, void* workspace, size_t workspace_bytes,
               void* stream) {
  (void)workspace;
  (void)workspace_bytes;
  return ssg_search_ex(base, n, d, dtype, dim_scale, graph, R, entry_ids, n_entry, queries, nq, K,
                       L, metric, out_ids, out_dists, nullptr, stream);
}

}  // extern "C"
