// ssg_knn.hip -- exact K-nearest-neighbour graph on gfx950 matrix cores: the
// first step of the indexing algorithm (Alg. 3 starts from a kNN graph; this
// builds it exactly, by brute force, instead of approximately).
//
// Row i of the result lists the K points nearest to point i (itself
// excluded) in ascending (squared Euclidean distance, id) order, with the
// distance of each pair computed in FP64 by summing (x_ij - x_kj)^2 over the
// dimensions in order.
//
// Pipeline (all on the device; the call synchronises its stream twice):
//   1. prep     BF16 copies of the base (hi, and the rounding residual lo),
//               squared norms, and whether every value is an integer in
//               [0, 255] with d <= 128.
//   2. scan     one workgroup per block of 128 rows sweeps all columns in
//               tiles of 128. Dot products come from MFMA
//               (v_mfma_f32_16x16x32_bf16); s = |y|^2 - 2<x, y> orders the
//               columns of a row like the distance. Values at or below the
//               row's running threshold go to an LDS queue; when the queue
//               overflows it is bucketed by row and merged into each row's
//               sorted candidate list (K' entries, kept in HBM); the
//               threshold is the list's K'-th s.
//        exact  integer data in [0, 255], d <= 128: BF16 holds every value
//               exactly and every FP32 partial sum is an integer below 2^24,
//               so s is exact and K' = K.
//        split  otherwise: <x, y> ~ xh.yh + xh.yl + xl.yh (three MFMAs) with a
//               bounded error, and K' = K + 28.
//   3. rerank   one wavefront per row: FP64 distances of the K' candidates,
//               rank-sorted by (distance, id); the first K are written. In
//               split mode a row is certified when its exact K-th distance is
//               below the smallest distance any non-candidate can have (the
//               K'-th s minus the error bound); other rows are listed.
//   4. fallback each listed row is rescanned in FP64 against every point,
//               keeping those at or below its K-th (distance, id).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <type_traits>

#include "ssg.h"
#include "ssg_device.h"
#include "ssg_internal.h"

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

constexpr int BM = 128;       // rows per workgroup
constexpr int BN = 64;        // columns per tile
constexpr int NT = 256;       // threads per scan workgroup (4 wavefronts, 2 x 2 of 64 x 32)
constexpr int NW = NT / 64;
constexpr int QW = 1024;      // LDS queue entries per wavefront
constexpr int KP_MAX = 128;   // candidate list length
constexpr int MARGIN = 28;    // extra candidates kept in split mode
constexpr int FB_ROWS = 256;  // fallback rows per launch
constexpr int FB_CAP = 4096;  // fallback entries per row
constexpr int64_t N_MAX = (int64_t)1 << 25;  // column ids take 25 bits of a queue entry

// -------------------------------------------------------------- helpers
__device__ __forceinline__ uint32_t ord_f32(float f) {
  uint32_t b = __float_as_uint(f);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(b);
}
__device__ __forceinline__ uint16_t bf16_rne(float x) {  // inputs are finite
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
// Global-memory views of workspace pointers. The pointers reach the kernels
// inside argument structs, so the compiler cannot tell their address space
// and would emit flat accesses, which count against the LDS wait counter as
// well: every LDS wait would then also wait for the tile prefetch.
template <class T>
__device__ __forceinline__ const __attribute__((address_space(1))) T* gmem(const T* p) {
  return (const __attribute__((address_space(1))) T*)p;
}
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T* gmem(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Number of entries of the ascending array a[0..cnt) below key.
__device__ __forceinline__ uint32_t lower_bound(const uint64_t* a, uint32_t cnt, uint64_t key) {
  uint32_t lo = 0, hi = cnt;
  while (lo < hi) {
    uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo;
}

using ssgdev::exact_l2;

struct Ws {
  uint16_t* xh;        // [NP x DP] BF16 of the base, zero padded
  uint16_t* xl;        // [NP x DP] BF16 of the rounding residual
  float* ny;           // [NP] squared norms (FP32 of the FP64 sum)
  float* nrm;          // [NP] norms
  uint64_t* lists;     // [NP x KP] sorted candidate keys  ord(s) << 32 | id
  uint32_t* lcnt;      // [NP] candidates per row
  uint32_t* flags;     // [0] non-integer data seen, [1] max norm bits, [2] rows to rescan, [3] rescan overflow
  uint32_t* fail_rows; // [n]
  double* fail_thr;    // [n] exact K-th distance of a listed row
  uint32_t* fail_tid;  // [n] and its id
  double* fb_d;        // [FB_ROWS x FB_CAP]
  uint32_t* fb_id;     // [FB_ROWS x FB_CAP]
};

struct Layout {
  int64_t NP;
  int DP, KP;
  size_t off_xh, off_xl, off_ny, off_nrm, off_lists, off_lcnt, off_flags, off_fail, off_thr,
      off_tid, off_fbd, off_fbi, total;
};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

Layout layout(int64_t n, int d, int K) {
  Layout L{};
  L.NP = (n + BM - 1) / BM * BM;
  L.DP = (d + 63) / 64 * 64;
  L.KP = (int)std::min<int64_t>(n - 1, (int64_t)K + MARGIN);
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t r = o; o = align256(o + bytes); return r; };
  L.off_xh = take((size_t)L.NP * L.DP * 2);
  L.off_xl = take((size_t)L.NP * L.DP * 2);
  L.off_ny = take((size_t)L.NP * 4);
  L.off_nrm = take((size_t)L.NP * 4);
  L.off_lists = take((size_t)L.NP * KP_MAX * 8);
  L.off_lcnt = take((size_t)L.NP * 4);
  L.off_flags = take(64);
  L.off_fail = take((size_t)n * 4);
  L.off_thr = take((size_t)n * 8);
  L.off_tid = take((size_t)n * 4);
  L.off_fbd = take((size_t)FB_ROWS * FB_CAP * 8);
  L.off_fbi = take((size_t)FB_ROWS * FB_CAP * 4);
  L.total = o;
  return L;
}

Ws bind(void* ws, const Layout& L) {
  char* b = static_cast<char*>(ws);
  Ws w;
  w.xh = reinterpret_cast<uint16_t*>(b + L.off_xh);
  w.xl = reinterpret_cast<uint16_t*>(b + L.off_xl);
  w.ny = reinterpret_cast<float*>(b + L.off_ny);
  w.nrm = reinterpret_cast<float*>(b + L.off_nrm);
  w.lists = reinterpret_cast<uint64_t*>(b + L.off_lists);
  w.lcnt = reinterpret_cast<uint32_t*>(b + L.off_lcnt);
  w.flags = reinterpret_cast<uint32_t*>(b + L.off_flags);
  w.fail_rows = reinterpret_cast<uint32_t*>(b + L.off_fail);
  w.fail_thr = reinterpret_cast<double*>(b + L.off_thr);
  w.fail_tid = reinterpret_cast<uint32_t*>(b + L.off_tid);
  w.fb_d = reinterpret_cast<double*>(b + L.off_fbd);
  w.fb_id = reinterpret_cast<uint32_t*>(b + L.off_fbi);
  return w;
}

// ------------------------------------------------------------------ prep
__global__ void knn_clear_flags(uint32_t* flags) {
  if (threadIdx.x < 16) flags[threadIdx.x] = 0u;
}

// One wavefront per PREP_ROWS consecutive (padded) rows. The largest norm and
// the non-integer flag are reduced over a wavefront's rows before the one
// atomic update each (an atomic per row would serialise a million updates on
// one word).
constexpr int PREP_ROWS = 32;

__global__ __launch_bounds__(256) void knn_prep(const float* __restrict__ base, int64_t n, int d,
                                                int DP, int64_t NP, Ws w) {
  const int lane = threadIdx.x & 63;
  const int64_t row0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * PREP_ROWS;
  if (row0 >= NP) return;
  const auto src = gmem(base);
  const auto xh = gmem(w.xh), xl = gmem(w.xl);
  uint32_t maxbits = 0;
  bool nonint = false;
  const int64_t row1 = row0 + PREP_ROWS < NP ? row0 + PREP_ROWS : NP;
  for (int64_t row = row0; row < row1; ++row) {
    double ss = 0.0;
    for (int j = lane; j < DP; j += 64) {
      const bool in = row < n && j < d;
      const float x = in ? src[row * d + j] : 0.f;
      const uint16_t h = bf16_rne(x);
      const uint16_t l = bf16_rne(x - bf16_f32(h));  // x - h is exact
      xh[row * DP + j] = h;
      xl[row * DP + j] = l;
      ss += (double)x * (double)x;
      nonint |= in && !(x >= 0.f && x <= 255.f && rintf(x) == x);
    }
    for (int off = 32; off >= 1; off >>= 1) ss += __shfl_xor(ss, off, 64);
    if (lane == 0) {
      const float nr = (float)sqrt(ss);
      gmem(w.ny)[row] = (float)ss;
      gmem(w.nrm)[row] = nr;
      if (row < n) maxbits = max(maxbits, __float_as_uint(nr));  // non-negative floats order like their bits
    }
  }
  const uint64_t bad = __ballot(nonint);
  if (lane == 0) {
    atomicMax(&w.flags[1], maxbits);
    if (bad) atomicOr(&w.flags[0], 1u);
  }
}

// ------------------------------------------------------------------ scan
struct ScanArgs {
  Ws w;
  int64_t n;
  int DP, KP;
};

// Wavefront w of a scan workgroup computes rows 64 * (w >> 1) + [0, 64) and
// columns 32 * (w & 1) + [0, 32) of each 128 x 64 tile: 4 x 2 MFMA blocks
// of 16 x 16. Two workgroups share a CU, so the two wavefronts on a SIMD
// belong to different workgroups and their phases (matrix cores, threshold
// tests, barriers) overlap. Lane l holds, for block (bi, bj), rows 16 bi + 4 (l >> 4) + i
// (i < 4) of column 16 bj + (l & 15).
template <bool SPLIT, int NKS>
struct ScanSmem {
  static constexpr bool AREG = NKS > 0;              // A fragments held in registers
  static constexpr int KC = AREG ? 32 * NKS : 32;    // dimensions per staged chunk
  static constexpr int SS = KC + 8;                  // LDS row stride (bf16): conflict-free 16-byte reads
  static constexpr int NB = SPLIT ? 2 : 1;
  struct Stage {
    uint16_t sB[NB][BN * SS];
    uint16_t sA[AREG ? 1 : NB][AREG ? 8 : BM * SS];
  };
  struct Merge {                                     // used only between tiles
    uint64_t q2[NW * QW];                            // entries bucketed by row
    uint64_t mt[NW][2 * KP_MAX + 64];                // per wavefront: list, output, new keys
  };
  union {
    Stage st;
    Merge mg;
  };
  uint64_t q[NW * QW];                               // one queue segment per wavefront
  uint32_t rowcnt[BM], rowoff[BM], rowfill[BM], lcnt[BM];
  float tau[BM];
  uint32_t qn[NW];
  uint32_t flag;
};

// Merges every wavefront's queue segment into the per-row candidate lists;
// called by all threads. Leaves the segments empty.
template <class SM>
__device__ void merge_queue(SM& sm, uint64_t* lists, int KP, int64_t r0) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int t = tid; t < BM; t += NT) { sm.rowcnt[t] = 0; sm.rowfill[t] = 0; }
  __syncthreads();
  for (int e = tid; e < NW * QW; e += NT)
    if ((uint32_t)(e % QW) < sm.qn[e / QW]) atomicAdd(&sm.rowcnt[(sm.q[e] >> 25) & 127u], 1u);
  __syncthreads();
  if (wave == 0) {  // exclusive prefix over 128 row counts, two per lane
    const uint32_t v0 = sm.rowcnt[2 * lane], v1 = sm.rowcnt[2 * lane + 1];
    uint32_t inc = v0 + v1;
    for (int off = 1; off < 64; off <<= 1) {
      const uint32_t t = __shfl_up(inc, off, 64);
      if (lane >= off) inc += t;
    }
    const uint32_t ex = inc - v0 - v1;
    sm.rowoff[2 * lane] = ex;
    sm.rowoff[2 * lane + 1] = ex + v0;
  }
  __syncthreads();
  for (int e = tid; e < NW * QW; e += NT) {
    if ((uint32_t)(e % QW) >= sm.qn[e / QW]) continue;
    const uint64_t v = sm.q[e];
    const uint32_t r = (uint32_t)(v >> 25) & 127u;
    sm.mg.q2[sm.rowoff[r] + atomicAdd(&sm.rowfill[r], 1u)] = v;
  }
  __syncthreads();
  uint64_t* Lk = sm.mg.mt[wave];
  uint64_t* Ok = Lk + KP_MAX;
  uint64_t* Nk = Lk + 2 * KP_MAX;
  // the next row's list is loaded while the current row is merged
  uint64_t pre0 = 0, pre1 = 0;
  auto fetch = [&](int r) {
    if (r >= BM) return;
    const uint32_t lc = sm.lcnt[r];
    const auto gl = gmem(lists + (r0 + r) * KP_MAX);
    if ((uint32_t)lane < lc) pre0 = gl[lane];
    if ((uint32_t)lane + 64 < lc) pre1 = gl[lane + 64];
  };
  fetch(wave);
  for (int r = wave; r < BM; r += NW) {
    const uint32_t cnt = sm.rowcnt[r];
    uint32_t lc = sm.lcnt[r];
    if ((uint32_t)lane < lc) Lk[lane] = pre0;
    if ((uint32_t)lane + 64 < lc) Lk[lane + 64] = pre1;
    fetch(r + NW);
    if (cnt == 0) continue;
    const uint32_t off = sm.rowoff[r];
    const auto gl = gmem(lists + (r0 + r) * KP_MAX);
    wave_sync();
    for (uint32_t c0 = 0; c0 < cnt; c0 += 64) {
      const uint32_t m = min(64u, cnt - c0);
      uint64_t nk = ~0ull;
      if ((uint32_t)lane < m) {
        const uint64_t v = sm.mg.q2[off + c0 + lane];
        nk = (v & 0xFFFFFFFF00000000ull) | (v & 0x1FFFFFFull);
      }
      // rank among the new keys: the keys are broadcast from LDS (Ok is
      // free until the scatter below), several reads in flight at a time
      // (a readlane per key costs more: each result passes through SGPRs)
      if ((uint32_t)lane < m) Ok[lane] = nk;
      wave_sync();
      uint32_t r1 = 0;
#pragma unroll 4
      for (uint32_t j = 0; j < m; ++j) r1 += Ok[j] < nk;
      wave_sync();
      if ((uint32_t)lane < m) Nk[r1] = nk;
      wave_sync();
      if ((uint32_t)lane < m) {
        const uint32_t p = r1 + lower_bound(Lk, lc, nk);
        if (p < (uint32_t)KP) Ok[p] = nk;
      }
      for (uint32_t k = lane; k < lc; k += 64) {
        const uint64_t lk = Lk[k];
        const uint32_t p = k + lower_bound(Nk, m, lk);
        if (p < (uint32_t)KP) Ok[p] = lk;
      }
      wave_sync();
      lc = min((uint32_t)KP, lc + m);
      for (uint32_t k = lane; k < lc; k += 64) Lk[k] = Ok[k];
      wave_sync();
    }
    for (uint32_t k = lane; k < lc; k += 64) gl[k] = Lk[k];
    if (lane == 0) {
      sm.lcnt[r] = lc;
      sm.tau[r] = lc == (uint32_t)KP ? unord_f32((uint32_t)(Lk[KP - 1] >> 32)) : INFINITY;
    }
    wave_sync();
  }
  if (tid < NW) sm.qn[tid] = 0;
  __syncthreads();
}

template <bool SPLIT, int NKS>
__global__ __launch_bounds__(NT, 2) void knn_scan(ScanArgs a) {
  using SM = ScanSmem<SPLIT, NKS>;
  constexpr bool AREG = SM::AREG;
  constexpr int KC = SM::KC, SS = SM::SS, NB = SM::NB;
  constexpr int KS = KC / 32;                    // MFMA k-steps per chunk
  constexpr int CPT = BN * KC / 8 / NT;          // 16-byte pieces per thread per staged operand
  constexpr int BJ = 2;                          // 16-column MFMA blocks per wavefront
  __shared__ __align__(16) SM sm;

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wm = wave >> 1, wn = wave & 1;
  const int64_t n = a.n;
  const int DP = a.DP;
  const int64_t r0 = (int64_t)blockIdx.x * BM;
  const int nchunk = AREG ? 1 : DP / KC;
  const int64_t ntiles = (n + BN - 1) / BN;
  // the argument block's fields as plain values: a reference to the block
  // (lambdas, helper calls) would make the compiler keep a private copy of it
  const uint16_t* const xh = a.w.xh;
  const uint16_t* const xl = a.w.xl;
  const float* const nyp = a.w.ny;
  uint64_t* const lists = a.w.lists;
  uint32_t* const lcntp = a.w.lcnt;
  const int KP = a.KP;
  auto xs = [=](int h) { return h ? xl : xh; };
  uint64_t* qseg = sm.q + wave * QW;

  for (int t = tid; t < BM; t += NT) {
    sm.lcnt[t] = 0;
    sm.tau[t] = (r0 + t < n) ? INFINITY : -INFINITY;
  }
  if (tid < NW) sm.qn[tid] = 0;
  if (tid == 0) sm.flag = 0;

  // A fragments of this wavefront's 64 rows (exact mode, all dimensions)
  bf16x8 areg[AREG ? NB : 1][4][AREG ? NKS : 1];
  if constexpr (AREG) {
#pragma unroll
    for (int h = 0; h < NB; ++h)
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          const int64_t row = r0 + 64 * wm + 16 * bi + (lane & 15);
          areg[h][bi][ks] = *reinterpret_cast<const bf16x8*>(xs(h) + row * DP + 32 * ks + 8 * (lane >> 4));
        }
  }

  // staged-operand registers (the next chunk is loaded while this one is used)
  constexpr int CPA = AREG ? 1 : BM * KC / 8 / NT;  // A pieces per thread (staged path)
  constexpr int PPR = KC / 8;                        // 16-byte pieces per row of a chunk
  constexpr int RPC = NT / PPR;                      // rows between a thread's pieces
  static_assert(NT % PPR == 0, "pieces of a chunk row split evenly over the threads");
  // piece c of this thread: row tid / PPR + c * RPC, 16-byte column tid % PPR
  const uint32_t boff = (uint32_t)((tid / PPR) * DP + (tid % PPR) * 8) * 2u;  // bytes
  const uint32_t bstep = (uint32_t)RPC * (uint32_t)DP * 2u;
  const int soff = (tid / PPR) * SS + (tid % PPR) * 8;                       // LDS elements
  u32x4 pb[NB][CPT];
  u32x4 pa[AREG ? 1 : NB][CPA];
  float nyn[BJ];  // squared norms of the prefetched tile's columns
  auto load_chunk = [&](int64_t tile, int chunk) {
    const int kc = chunk * KC;
    if (chunk == 0) {
      const auto nyt = gmem(nyp + tile * BN + 32 * wn + (lane & 15));
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) nyn[bj] = nyt[16 * bj];
    }
#pragma unroll
    for (int h = 0; h < NB; ++h) {
      const char* tb = reinterpret_cast<const char*>(xs(h) + tile * BN * DP + kc);
#pragma unroll
      for (int c = 0; c < CPT; ++c) {  // uniform base per piece, one per-thread offset
        const char* tbc = tb + (size_t)c * bstep;
        pb[h][c] = *gmem(reinterpret_cast<const u32x4*>(tbc + boff));
      }
      if constexpr (!AREG) {
        const char* ta = reinterpret_cast<const char*>(xs(h) + r0 * DP + kc);
#pragma unroll
        for (int c = 0; c < CPA; ++c) {
          const char* tac = ta + (size_t)c * bstep;
          pa[h][c] = *gmem(reinterpret_cast<const u32x4*>(tac + boff));
        }
      }
    }
  };
  auto store_chunk = [&]() {
#pragma unroll
    for (int h = 0; h < NB; ++h) {
#pragma unroll
      for (int c = 0; c < CPT; ++c)
        *reinterpret_cast<u32x4*>(&sm.st.sB[h][soff + c * RPC * SS]) = pb[h][c];
      if constexpr (!AREG) {
#pragma unroll
        for (int c = 0; c < CPA; ++c)
          *reinterpret_cast<u32x4*>(&sm.st.sA[h][soff + c * RPC * SS]) = pa[h][c];
      }
    }
  };

  load_chunk(0, 0);
  __syncthreads();
  float tr[16];
#pragma unroll
  for (int bi = 0; bi < 4; ++bi)
#pragma unroll
    for (int i = 0; i < 4; ++i) tr[bi * 4 + i] = sm.tau[64 * wm + 16 * bi + 4 * (lane >> 4) + i];
  uint32_t qn = 0;  // entries in this wavefront's segment (uniform)

  for (int64_t tile = 0; tile < ntiles; ++tile) {
    f32x4 acc[4][BJ];
#pragma unroll
    for (int bi = 0; bi < 4; ++bi)
#pragma unroll
      for (int bj = 0; bj < BJ; ++bj) acc[bi][bj] = f32x4{0.f, 0.f, 0.f, 0.f};

    float nyc[BJ];
    for (int chunk = 0; chunk < nchunk; ++chunk) {
      __syncthreads();  // previous chunk's readers are done with the LDS tiles
      store_chunk();
      if (chunk == 0) {
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) nyc[bj] = nyn[bj];
      }
      __syncthreads();
      {  // prefetch the next chunk (or the next tile's first chunk)
        int nc = chunk + 1;
        int64_t nt = tile;
        if (nc == nchunk) { nc = 0; ++nt; }
        if (nt < ntiles) load_chunk(nt, nc);
      }
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) {
        bf16x8 bfr[NB][BJ];
        bf16x8 afr[NB][4];
#pragma unroll
        for (int h = 0; h < NB; ++h)
#pragma unroll
          for (int bj = 0; bj < BJ; ++bj)
            bfr[h][bj] = *reinterpret_cast<const bf16x8*>(
                &sm.st.sB[h][(32 * wn + 16 * bj + (lane & 15)) * SS + 32 * ks + 8 * (lane >> 4)]);
#pragma unroll
        for (int h = 0; h < NB; ++h)
#pragma unroll
          for (int bi = 0; bi < 4; ++bi) {
            if constexpr (AREG)
              afr[h][bi] = areg[h][bi][ks];
            else
              afr[h][bi] = *reinterpret_cast<const bf16x8*>(
                  &sm.st.sA[h][(64 * wm + 16 * bi + (lane & 15)) * SS + 32 * ks + 8 * (lane >> 4)]);
          }
#pragma unroll
        for (int bi = 0; bi < 4; ++bi)
#pragma unroll
          for (int bj = 0; bj < BJ; ++bj) {
            acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[0][bi], bfr[0][bj], acc[bi][bj], 0, 0, 0);
            if constexpr (SPLIT) {
              acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[0][bi], bfr[1][bj], acc[bi][bj], 0, 0, 0);
              acc[bi][bj] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(afr[1][bi], bfr[0][bj], acc[bi][bj], 0, 0, 0);
            }
          }
      }
    }

    // ---- epilogue: threshold test, append to this wavefront's segment
    const int64_t c0 = tile * BN;
    const bool special = (c0 < r0 + BM && c0 + BN > r0) || c0 + BN > n;  // self pairs, absent columns
    // Appends the selected elements that pass the threshold; returns those
    // that found the segment full. SPECIAL tiles also drop self pairs and
    // absent columns; SEL restricts the test to the elements set in sel.
    // Per-tile forms of the row and column codes, so that no per-element
    // constant is live across the tile loop: element (bi, bj, i) of this lane
    // is row rbase + 16 bi + i, column cbase + 16 bj; its queue code is
    // kb[bj] + ((16 bi + i) << 25) and it is a self pair iff
    // db[bj] == 16 bi + i.
    const uint32_t rbase = (uint32_t)(64 * wm + 4 * (lane >> 4));
    const uint32_t cbase = (uint32_t)(c0 + 32 * wn + (lane & 15));
    const uint32_t n32 = (uint32_t)n;
    uint32_t kb[BJ], db[BJ];
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      kb[bj] = (rbase << 25) | (cbase + 16 * bj);
      db[bj] = cbase + 16 * bj - (uint32_t)r0 - rbase;
    }
    auto push = [&](auto special_c, auto sel_c, uint64_t sel) -> uint64_t {
      constexpr bool SPECIAL = decltype(special_c)::value;
      constexpr bool SEL = decltype(sel_c)::value;
      // branch-free pass: which 16 x 16 blocks hold a passing element
      uint32_t blocks = 0;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) {
          uint64_t m = 0;
#pragma unroll
          for (int i = 0; i < 4; ++i) m |= __ballot(fmaf(-2.f, acc[bi][bj][i], nyc[bj]) <= tr[bi * 4 + i]);
          blocks |= (m != 0 ? 1u : 0u) << (bi * BJ + bj);
        }
      uint64_t left = 0;
      if (blocks == 0 && !SPECIAL) return left;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int bj = 0; bj < BJ; ++bj) {
          if (!SPECIAL && !((blocks >> (bi * BJ + bj)) & 1u)) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int e = (bi * BJ + bj) * 4 + i;
            const float s = fmaf(-2.f, acc[bi][bj][i], nyc[bj]);
            bool surv = s <= tr[bi * 4 + i];
            if constexpr (SEL) surv = surv && ((sel >> e) & 1ull);
            if constexpr (SPECIAL)
              surv = surv && cbase + 16 * bj < n32 && db[bj] != (uint32_t)(16 * bi + i);
            const uint64_t m = __ballot(surv);
            if (m) {
              const uint32_t pos = qn + mbcnt64(m);
              if (surv) {
                if (pos < (uint32_t)QW)
                  qseg[pos] = ((uint64_t)ord_f32(s) << 32) | (kb[bj] + ((uint32_t)(16 * bi + i) << 25));
                else
                  left |= 1ull << e;
              }
              qn = min(qn + (uint32_t)__popcll(m), (uint32_t)QW);
            }
          }
        }
      return left;
    };
    using T_ = std::true_type;
    using F_ = std::false_type;
    uint64_t pend = special ? push(T_{}, F_{}, 0ull) : push(F_{}, F_{}, 0ull);
    // merge when a segment overflowed or has less room than one more tile's worst case
    const bool need = __ballot(pend != 0) != 0 || qn > (uint32_t)(QW - 64);
    if (lane == 0) {
      sm.qn[wave] = qn;
      if (need) sm.flag = 1;
    }
    __syncthreads();
    while (sm.flag) {
      merge_queue(sm, lists, KP, r0);  // ends with a barrier; empties the segments
      qn = 0;
#pragma unroll
      for (int bi = 0; bi < 4; ++bi)
#pragma unroll
        for (int i = 0; i < 4; ++i) tr[bi * 4 + i] = sm.tau[64 * wm + 16 * bi + 4 * (lane >> 4) + i];
      if (tid == 0) sm.flag = 0;
      __syncthreads();
      pend = special ? push(T_{}, T_{}, pend) : push(F_{}, T_{}, pend);  // now above the threshold: dropped
      const bool again = __ballot(pend != 0) != 0;
      if (lane == 0) {
        sm.qn[wave] = qn;
        if (again) sm.flag = 1;
      }
      __syncthreads();
    }
  }
  bool any = false;  // segments were published before the last barrier
  for (int w = 0; w < NW; ++w) any |= sm.qn[w] > 0;
  if (any) merge_queue(sm, lists, KP, r0);
  __syncthreads();
  for (int t = tid; t < BM; t += NT) gmem(lcntp)[r0 + t] = sm.lcnt[t];
}

// ---------------------------------------------------------------- rerank
struct RerankArgs {
  const float* base;
  int64_t n;
  int d, DP, K, KP;
  int exact;
  double e_rel;   // error of s relative to |x| * max|y|
  double e_abs;   // error of s relative to max|y|^2 + 2 |x| max|y|
  Ws w;
  uint32_t* out_ids;
  float* out_d;
};

// One wavefront per row: exact distances of the candidates, rank sort,
// output, certificate.
__global__ __launch_bounds__(256) void knn_rerank(RerankArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= a.n) return;
  const uint32_t lc = a.w.lcnt[row];
  const float* q = a.base + row * a.d;
  double dv[2];
  uint32_t iv[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t k = lane + 64 * t;
    dv[t] = INFINITY;
    iv[t] = 0xFFFFFFFFu;
    if (k < lc) {
      iv[t] = (uint32_t)(a.w.lists[row * KP_MAX + k] & 0xFFFFFFFFull);
      dv[t] = exact_l2(q, a.base + (int64_t)iv[t] * a.d, a.d);
    }
  }
  uint32_t rk[2] = {0, 0};
  for (uint32_t j = 0; j < lc; ++j) {
    const int t = j >> 6, src = j & 63;
    const double dj = __shfl(t ? dv[1] : dv[0], src, 64);
    const uint32_t ij = __shfl(t ? iv[1] : iv[0], src, 64);
#pragma unroll
    for (int u = 0; u < 2; ++u) rk[u] += (dj < dv[u]) || (dj == dv[u] && ij < iv[u]);
  }
  double dK = 0.0;
  uint32_t iK = 0;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t k = lane + 64 * t;
    if (k < lc && rk[t] < (uint32_t)a.K) {
      a.out_ids[row * a.K + rk[t]] = iv[t];
      a.out_d[row * a.K + rk[t]] = (float)dv[t];
    }
    const uint64_t hit = __ballot(k < lc && rk[t] == (uint32_t)(a.K - 1));
    if (hit) {
      const int src = __builtin_ctzll(hit);
      dK = __shfl(dv[t], src, 64);
      iK = __shfl(iv[t], src, 64);
    }
  }
  if (a.exact || lc < (uint32_t)a.KP || (int64_t)a.KP >= a.n - 1) return;  // exact keys, or every point was a candidate
  if (lane == 0) {
    const float sK = unord_f32((uint32_t)(a.w.lists[row * KP_MAX + a.KP - 1] >> 32));
    const double xn = (double)a.w.nrm[row];
    const double M = (double)__uint_as_float(a.w.flags[1]);
    double nx = 0.0;
    for (int j = 0; j < a.d; ++j) nx += (double)q[j] * (double)q[j];
    const double err = a.e_rel * xn * M + a.e_abs * (M * M + 2.0 * xn * M) + 1e-30;
    const double lower = (double)sK + nx - err;
    if (!(dK < lower)) {
      const uint32_t slot = atomicAdd(&a.w.flags[2], 1u);
      a.w.fail_rows[slot] = (uint32_t)row;
      a.w.fail_thr[slot] = dK;
      a.w.fail_tid[slot] = iK;
    }
  }
}

// -------------------------------------------------------------- fallback
// One workgroup per listed row: every point at or below the row's K-th
// (distance, id) is collected, then rank-sorted.
__global__ __launch_bounds__(256) void knn_fallback(const float* __restrict__ base, int64_t n, int d,
                                                    int K, Ws w, uint32_t first, uint32_t* out_ids,
                                                    float* out_d) {
  __shared__ uint32_t cnt;
  const int tid = threadIdx.x;
  const uint32_t slot = first + blockIdx.x;
  const int64_t row = w.fail_rows[slot];
  const double T = w.fail_thr[slot];
  const uint32_t Tid = w.fail_tid[slot];
  double* fd = w.fb_d + (int64_t)blockIdx.x * FB_CAP;
  uint32_t* fi = w.fb_id + (int64_t)blockIdx.x * FB_CAP;
  if (tid == 0) cnt = 0;
  __syncthreads();
  const float* q = base + row * d;
  for (int64_t j = tid; j < n; j += 256) {
    if (j == row) continue;
    const double dj = exact_l2(q, base + j * d, d);
    if (dj < T || (dj == T && (uint32_t)j <= Tid)) {
      const uint32_t p = atomicAdd(&cnt, 1u);
      if (p < (uint32_t)FB_CAP) { fd[p] = dj; fi[p] = (uint32_t)j; }
    }
  }
  __syncthreads();
  const uint32_t c = cnt;
  if (c > (uint32_t)FB_CAP) {
    if (tid == 0) atomicOr(&w.flags[3], 1u);
    return;
  }
  __threadfence_block();
  for (uint32_t e = tid; e < c; e += 256) {
    const double de = fd[e];
    const uint32_t ie = fi[e];
    uint32_t r = 0;
    for (uint32_t f = 0; f < c; ++f) r += (fd[f] < de) || (fd[f] == de && fi[f] < ie);
    if (r < (uint32_t)K) {
      out_ids[row * K + r] = ie;
      out_d[row * K + r] = (float)de;
    }
  }
}

using ScanFn = void (*)(ScanArgs);

template <bool SPLIT, int NKS>
int launch_scan(const ScanArgs& a, int64_t blocks, hipStream_t s) {
  hipLaunchKernelGGL((knn_scan<SPLIT, NKS>), dim3((unsigned)blocks), dim3(NT), 0, s, a);
  return hipGetLastError() == hipSuccess ? SSG_OK : SSG_EDEVICE;
}

int fail_msg(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail_msg(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  return ssg_internal_fail(code, buf);
}

}  // namespace

extern "C" {

size_t ssg_knn_workspace_bytes(int64_t n, int32_t d, int32_t K) {
  if (n < 2 || d < 1 || K < 1) return 0;
  return layout(n, d, K).total;
}

int ssg_knn_graph(const float* base, int64_t n, int32_t d, int32_t K, uint32_t* out_ids,
                  float* out_dists, void* workspace, size_t workspace_bytes, int64_t* stats,
                  void* stream) {
  if (!base || !out_ids || !out_dists || !workspace)
    return fail_msg(SSG_EINVAL, "ssg_knn_graph: null pointer argument");
  if (n < 2 || n > N_MAX) return fail_msg(SSG_EINVAL, "ssg_knn_graph: n=%lld outside [2, 2^25]", (long long)n);
  if (d < 1) return fail_msg(SSG_EINVAL, "ssg_knn_graph: d=%d", d);
  if (K < 1 || K > KP_MAX - MARGIN || K > n - 1)
    return fail_msg(SSG_EINVAL, "ssg_knn_graph: K=%d outside [1, min(%d, n-1)]", K, KP_MAX - MARGIN);
  const Layout L = layout(n, d, K);
  if (workspace_bytes < L.total)
    return fail_msg(SSG_EINVAL, "ssg_knn_graph: workspace of %zu bytes, %zu needed", workspace_bytes, L.total);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail_msg(SSG_EINVAL, "ssg_knn_graph: workspace not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const Ws w = bind(workspace, L);

  hipLaunchKernelGGL(knn_clear_flags, dim3(1), dim3(64), 0, s, w.flags);
  const int64_t prep_waves = (L.NP + PREP_ROWS - 1) / PREP_ROWS;
  hipLaunchKernelGGL(knn_prep, dim3((unsigned)((prep_waves + 3) / 4)), dim3(256), 0, s, base, n, d, L.DP, L.NP,
                     w);
  uint32_t flags[4];
  if (hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_knn_graph: prep failed: %s", hipGetErrorString(hipGetLastError()));
  const bool exact = flags[0] == 0 && d <= 128;

  ScanArgs sa{w, n, L.DP, exact ? K : L.KP};
  const int64_t blocks = L.NP / BM;
  int rc;
  if (exact)
    rc = L.DP <= 64 ? launch_scan<false, 2>(sa, blocks, s) : launch_scan<false, 4>(sa, blocks, s);
  else
    rc = launch_scan<true, 0>(sa, blocks, s);
  if (rc) return fail_msg(rc, "ssg_knn_graph: scan launch failed: %s", hipGetErrorString(hipGetLastError()));

  RerankArgs ra{};
  ra.base = base; ra.n = n; ra.d = d; ra.DP = L.DP; ra.K = K; ra.KP = sa.KP; ra.exact = exact;
  const double u = std::ldexp(1.0, -24);
  // <x,y> error of the three-product split: dropped terms <= 3.1 * 2^-16 |x||y|, FP32
  // accumulation of 3*DP exact products <= (3*DP + 16) * u * 1.05 |x||y|; s doubles it.
  ra.e_rel = 1.25 * 2.0 * (3.1 * std::ldexp(1.0, -16) + (3.0 * L.DP + 16.0) * u * 1.05);
  // rounding of |y|^2 to FP32 and of the fused s = |y|^2 - 2<x,y>
  ra.e_abs = 1.25 * 3.0 * u;
  ra.w = w; ra.out_ids = out_ids; ra.out_d = out_dists;
  hipLaunchKernelGGL(knn_rerank, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, ra);
  if (hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_knn_graph: scan/rerank failed: %s", hipGetErrorString(hipGetLastError()));
  const uint32_t nfail = flags[2];
  if (nfail > 1024 && (double)nfail * (double)n > 68719476736.0)  // 2^36 rescanned pairs
    return fail_msg(SSG_EUNSUPPORTED,
                    "ssg_knn_graph: %u rows failed the certificate (error bound too wide for this data)", nfail);
  for (uint32_t f = 0; f < nfail; f += FB_ROWS) {
    const uint32_t m = std::min<uint32_t>(FB_ROWS, nfail - f);
    hipLaunchKernelGGL(knn_fallback, dim3(m), dim3(256), 0, s, base, n, d, K, w, f, out_ids, out_dists);
  }
  if (nfail) {
    if (hipMemcpyAsync(flags, w.flags, sizeof flags, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return fail_msg(SSG_EDEVICE, "ssg_knn_graph: rescan failed: %s", hipGetErrorString(hipGetLastError()));
    if (flags[3])
      return fail_msg(SSG_EUNSUPPORTED, "ssg_knn_graph: more than %d points tie below a row's K-th distance", FB_CAP);
  }
  if (stats) {
    stats[0] = exact ? 1 : 0;
    stats[1] = nfail;
    stats[2] = sa.KP;
    stats[3] = 0;
  }
  ssg_internal_clear_error();
  return SSG_OK;
}

}  // extern "C"
