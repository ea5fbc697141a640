// ssg_build.hip -- the two pruning loops of the indexing algorithm (Alg. 3)
// on the device: for every node, candidates from the kNN graph, the SSG
// angular rule over them (at most R out-edges, pairwise angles >= alpha),
// then reverse-neighbour checking.
//
// Readings (the same as the reference implementation used for testing):
//   * candidates of node i: for each kNN neighbour u of i in ascending order,
//     u and then u's whole kNN list are added (i itself and repeats skipped);
//     the expansion stops once at least l candidates are held;
//   * candidates at distance 0 from i are dropped (the angle is undefined);
//   * candidates are taken in ascending (squared distance, id) order; one is
//     kept unless a kept edge makes an angle below alpha with it, i.e. unless
//     <c - i, k - i> > 0 and <c - i, k - i>^2 > cos^2(alpha) |c - i|^2 |k - i|^2,
//     all in FP64 with every operation rounded on its own;
//   * reverse step, order-independent: node j re-selects from its own
//     out-edges plus every i with an edge i -> j, by the same rule.
//
// Work mapping: one wavefront per node. The forward step keeps its
// candidates in LDS (open-addressing hash for the repeats, then a rank sort);
// the reverse step gathers each node's in-edges with a count / scan / fill
// pass and sorts them in a workspace.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "ssg.h"
#include "ssg_device.h"
#include "ssg_internal.h"

namespace {

constexpr uint32_t kSent = 0xFFFFFFFFu;
constexpr int PCAP = 1024;       // forward candidates per node: l + Kk + 2 <= PCAP
constexpr int RMAX = 64;         // out-degree bound
constexpr int SCAN_B = 1024;     // elements per scan block

struct Cand {
  double dist;
  uint32_t id;
  uint32_t pad;
};

__device__ __forceinline__ bool cand_less(const Cand& a, const Cand& b) {
  return a.dist < b.dist || (a.dist == b.dist && a.id < b.id);
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint32_t mbcnt64(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Writes in[0..nc) to out[0..nc) in ascending (dist, id) order (ids are
// distinct, so every key has its own rank).
__device__ void wave_rank_sort(const Cand* in, Cand* out, int nc, int lane) {
  for (int e = lane; e < nc; e += 64) {
    const Cand ce = in[e];
    int r = 0;
    for (int f = 0; f < nc; ++f) r += cand_less(in[f], ce);
    out[r] = ce;
  }
  wave_sync();
}

// NB sums s[b] = sum_j (p[b]_j - c_j) (q_j - c_j), each in FP64 in index
// order with every operation rounded on its own: the operation sequence of
// ssgdev::dot_rel(p[b], q, c, d) for every b, the NB chains interleaved so
// that their latencies overlap. (q_j - c_j) is formed once and shared.
template <int NB>
__device__ __forceinline__ void dot_rel_multi(const float* const (&p)[NB], const float* q,
                                              const float* c, int d, double (&s)[NB]) {
#pragma clang fp contract(off)
#pragma unroll
  for (int b = 0; b < NB; ++b) s[b] = 0.0;
  int j = 0;
  uintptr_t al = reinterpret_cast<uintptr_t>(q) | reinterpret_cast<uintptr_t>(c);
#pragma unroll
  for (int b = 0; b < NB; ++b) al |= reinterpret_cast<uintptr_t>(p[b]);
  if ((al & 15) == 0) {
    for (; j + 4 <= d; j += 4) {
      const float4 y = *reinterpret_cast<const float4*>(q + j);
      const float4 z = *reinterpret_cast<const float4*>(c + j);
      const double yz0 = (double)y.x - (double)z.x, yz1 = (double)y.y - (double)z.y;
      const double yz2 = (double)y.z - (double)z.z, yz3 = (double)y.w - (double)z.w;
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const float4 x = *reinterpret_cast<const float4*>(p[b] + j);
        s[b] = s[b] + ((double)x.x - (double)z.x) * yz0;
        s[b] = s[b] + ((double)x.y - (double)z.y) * yz1;
        s[b] = s[b] + ((double)x.z - (double)z.z) * yz2;
        s[b] = s[b] + ((double)x.w - (double)z.w) * yz3;
      }
    }
  }
  for (; j < d; ++j) {
    const double yz = (double)q[j] - (double)c[j];
#pragma unroll
    for (int b = 0; b < NB; ++b) s[b] = s[b] + ((double)p[b][j] - (double)c[j]) * yz;
  }
}

// Greedy SSG selection over sorted candidates cs[0..nc) of node i. Writes the
// kept ids to kid[] and returns their number (<= R). Candidates are taken up
// to SEL_NB at a time: lane k < kept computes the batch members' dot products
// against kept edge k in interleaved chains, and the next lanes test each
// later member against each earlier one (needed if the earlier one is kept).
// The batch is then resolved in candidate order, member by member, with the
// same tests and the same FP64 values as taking one candidate at a time.
constexpr int SEL_NB = 4;

__device__ int wave_select(const float* __restrict__ base, int d, int64_t i, const Cand* cs,
                           int nc, double cos2a, int R, uint32_t* kid, double* klen, int lane) {
#pragma clang fp contract(off)
  const float* xi = base + i * d;
  int kept = 0;
  for (int c = 0; c < nc && kept < R;) {
    int nb = min(SEL_NB, nc - c);
    while (nb > 1 && kept + nb * (nb - 1) / 2 > 64) --nb;  // one lane per member pair
    const int kept0 = kept, npair = nb * (nb - 1) / 2;
    const float* p[SEL_NB];
    const float* q = xi;
    int pb = -1, pa = -1;  // pair lane: member pb tested against member pa
    if (lane < kept0) {
      q = base + (int64_t)kid[lane] * d;
#pragma unroll
      for (int b = 0; b < SEL_NB; ++b) p[b] = base + (int64_t)cs[c + min(b, nb - 1)].id * d;
    } else if (lane < kept0 + npair) {
      int t = lane - kept0, b = 1;
      while (t >= b) { t -= b; ++b; }  // lane kept0 + b (b - 1) / 2 + a holds pair (a, b)
      pb = b;
      pa = t;
      q = base + (int64_t)cs[c + pa].id * d;
#pragma unroll
      for (int k = 0; k < SEL_NB; ++k) p[k] = base + (int64_t)cs[c + pb].id * d;
    } else {
#pragma unroll
      for (int b = 0; b < SEL_NB; ++b) p[b] = xi;
    }
    double s[SEL_NB];
    dot_rel_multi<SEL_NB>(p, q, xi, d, s);
    uint32_t conf = 0;  // bit b: an edge kept before the batch conflicts with member b
#pragma unroll
    for (int b = 0; b < SEL_NB; ++b) {
      if (b >= nb) break;
      const double dc = cs[c + b].dist;
      const bool cf = lane < kept0 && s[b] > 0.0 && s[b] * s[b] > cos2a * dc * klen[lane];
      if (__ballot(cf) != 0) conf |= 1u << b;
    }
    bool pcf = false;
    if (pb >= 0) {
      const double dc = cs[c + pb].dist, dk = cs[c + pa].dist;
      pcf = s[0] > 0.0 && s[0] * s[0] > cos2a * dc * dk;
    }
    const uint64_t pmask = __ballot(pcf);
    uint32_t acc = 0;  // bit b: member b kept
    for (int b = 0; b < nb && kept < R; ++b) {
      bool ok = !((conf >> b) & 1u);
      for (int a0 = 0; a0 < b; ++a0)
        if (((acc >> a0) & 1u) && ((pmask >> (kept0 + b * (b - 1) / 2 + a0)) & 1ull)) ok = false;
      if (ok) {
        acc |= 1u << b;
        if (lane == 0) {
          kid[kept] = cs[c + b].id;
          klen[kept] = cs[c + b].dist;
        }
        ++kept;
      }
    }
    wave_sync();
    c += nb;
  }
  return kept;
}


// ------------------------------------------------------------- forward step
struct PruneArgs {
  const float* base;
  int64_t n;
  int d;
  const uint32_t* knn;
  int Kk, l, R;
  double cos2a;
  uint32_t* out;
};

// PC: candidate capacity (>= l + Kk + 2); the repeat filter is a hash of 4 PC
// slots, so it is at most a quarter full.
template <int PC>
__global__ __launch_bounds__(64) void prune_kernel(PruneArgs a) {
  constexpr int HSLOTS = 4 * PC;
  constexpr int HBITS = PC == 256 ? 10 : 12;
  static_assert((1 << HBITS) == HSLOTS, "hash size");
  __shared__ union {
    uint32_t hash[HSLOTS];
    Cand sorted[PC];
  } u;
  __shared__ Cand cand[PC];
  __shared__ uint32_t kid[RMAX];
  __shared__ double klen[RMAX];
  const int lane = threadIdx.x;
  const int64_t i = blockIdx.x;
  for (int s = lane; s < HSLOTS; s += 64) u.hash[s] = kSent;
  wave_sync();
  // test-and-insert; true when v was not yet present
  auto insert = [&](uint32_t v) -> bool {
    uint32_t h = (v * 2654435761u) >> (32 - HBITS);
    for (;;) {
      const uint32_t old = atomicCAS(&u.hash[h], kSent, v);
      if (old == kSent) return true;
      if (old == v) return false;
      h = (h + 1) & (HSLOTS - 1);
    }
  };
  if (lane == 0) insert((uint32_t)i);  // never a candidate of itself
  wave_sync();
  int np = 0;
  const uint32_t* row = a.knn + i * a.Kk;
  for (int t = 0; t < a.Kk; ++t) {
    const uint32_t u0 = row[t];
    if (u0 == kSent) break;
    // the neighbour itself, then its kNN list
    for (int e0 = 0; e0 <= a.Kk; e0 += 64) {
      const int e = e0 + lane;
      uint32_t v = kSent;
      if (e == 0) v = u0;
      else if (e <= a.Kk) v = a.knn[(int64_t)u0 * a.Kk + e - 1];
      const bool fresh = v != kSent && (int64_t)v < a.n && insert(v);
      const uint64_t m = __ballot(fresh);
      const int pos = np + (int)mbcnt64(m);
      if (fresh && pos < PC) cand[pos].id = v;
      np += __popcll(m);
      wave_sync();
    }
    if (np >= a.l) break;
  }
  np = min(np, PC);  // cannot bind: the host checks l + Kk + 2 <= PC
  // FP64 distances; distance-0 candidates sort last and are cut
  const float* xi = a.base + i * a.d;
  int zeros = 0;
  for (int c0 = 0; c0 < np; c0 += 64) {
    const int c = c0 + lane;
    bool z = false;
    if (c < np) {
      const double dd = ssgdev::exact_l2(xi, a.base + (int64_t)cand[c].id * a.d, a.d);
      z = dd == 0.0;
      cand[c].dist = z ? INFINITY : dd;
    }
    zeros += __popcll(__ballot(z));
  }
  wave_sync();
  wave_rank_sort(cand, u.sorted, np, lane);
  const int kept = wave_select(a.base, a.d, i, u.sorted, np - zeros, a.cos2a, a.R, kid, klen, lane);
  for (int t = lane; t < a.R; t += 64) a.out[i * a.R + t] = t < kept ? kid[t] : kSent;
}

// ------------------------------------------------------------- reverse step
__global__ void rev_count(const uint32_t* __restrict__ g1, int64_t n, int R, uint32_t* cnt) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const uint32_t j = g1[e];
  if (j != kSent) atomicAdd(&cnt[j], 1u);
}

// exclusive prefix of cnt[0..n) -> off[0..n], in blocks of SCAN_B
__global__ __launch_bounds__(SCAN_B) void scan_blocks(const uint32_t* cnt, int64_t n, uint32_t* off,
                                                      uint32_t* bsum) {
  __shared__ uint32_t s[SCAN_B];
  const int t = threadIdx.x;
  const int64_t g = (int64_t)blockIdx.x * SCAN_B + t;
  const uint32_t v = g < n ? cnt[g] : 0u;
  s[t] = v;
  __syncthreads();
  for (int o = 1; o < SCAN_B; o <<= 1) {
    const uint32_t add = t >= o ? s[t - o] : 0u;
    __syncthreads();
    s[t] += add;
    __syncthreads();
  }
  if (g < n) off[g] = s[t] - v;
  if (t == SCAN_B - 1) bsum[blockIdx.x] = s[t];
}

// one workgroup: exclusive prefix of the block sums, in place; bsum[nb] = total
__global__ __launch_bounds__(SCAN_B) void scan_sums(uint32_t* bsum, int64_t nb) {
  __shared__ uint32_t s[SCAN_B];
  __shared__ uint32_t carry;
  const int t = threadIdx.x;
  if (t == 0) carry = 0;
  __syncthreads();
  for (int64_t b0 = 0; b0 < nb; b0 += SCAN_B) {
    const int64_t g = b0 + t;
    const uint32_t v = g < nb ? bsum[g] : 0u;
    s[t] = v;
    __syncthreads();
    for (int o = 1; o < SCAN_B; o <<= 1) {
      const uint32_t add = t >= o ? s[t - o] : 0u;
      __syncthreads();
      s[t] += add;
      __syncthreads();
    }
    const uint32_t c = carry;
    if (g < nb) bsum[g] = c + s[t] - v;
    __syncthreads();
    if (t == SCAN_B - 1) carry = c + s[t];
    __syncthreads();
  }
  if (t == 0) bsum[nb] = carry;
}

__global__ void scan_add(uint32_t* off, int64_t n, const uint32_t* bsum, int64_t nb) {
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (g < n) off[g] += bsum[g / SCAN_B];
  if (g == 0) off[n] = bsum[nb];
}

__global__ void rev_fill(const uint32_t* __restrict__ g1, int64_t n, int R, const uint32_t* off,
                         uint32_t* fill, uint32_t* rev) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * R) return;
  const uint32_t j = g1[e];
  if (j != kSent) rev[off[j] + atomicAdd(&fill[j], 1u)] = (uint32_t)(e / R);
}

struct ReverseArgs {
  const float* base;
  int64_t n;
  int d;
  const uint32_t* g1;
  int R;
  double cos2a;
  const uint32_t* off;
  const uint32_t* rev;
  Cand* scratch;  // node j owns [2 (off[j] + j R), 2 (off[j + 1] + (j + 1) R))
  uint32_t* out;
};

__global__ __launch_bounds__(64) void reverse_kernel(ReverseArgs a) {
  __shared__ uint32_t own[RMAX];
  __shared__ uint32_t kid[RMAX];
  __shared__ double klen[RMAX];
  const int lane = threadIdx.x;
  const int64_t j = blockIdx.x;
  const uint32_t r0 = a.off[j], r1 = a.off[j + 1];
  const int64_t cap = (int64_t)(r1 - r0) + a.R;
  Cand* cs = a.scratch + 2 * ((int64_t)r0 + j * a.R);
  Cand* srt = cs + cap;
  const float* xj = a.base + j * a.d;
  // own out-edges, in order (a row is ids followed by padding)
  uint32_t v = lane < a.R ? a.g1[j * a.R + lane] : kSent;
  const int deg = __popcll(__ballot(v != kSent));
  if (lane < deg) {
    own[lane] = v;
    cs[lane].id = v;
    cs[lane].dist = ssgdev::exact_l2(xj, a.base + (int64_t)v * a.d, a.d);
  }
  wave_sync();
  // in-edges not already out-edges, distance 0 dropped
  int nc = deg;
  for (uint32_t e0 = r0; e0 < r1; e0 += 64) {
    const uint32_t e = e0 + lane;
    bool keep = false;
    uint32_t w = 0;
    double dd = 0.0;
    if (e < r1) {
      w = a.rev[e];
      keep = true;
      for (int k = 0; k < deg; ++k) keep = keep && own[k] != w;
      if (keep) {
        dd = ssgdev::exact_l2(xj, a.base + (int64_t)w * a.d, a.d);
        keep = dd != 0.0;
      }
    }
    const uint64_t m = __ballot(keep);
    if (keep) {
      const int pos = nc + (int)mbcnt64(m);
      cs[pos].id = w;
      cs[pos].dist = dd;
    }
    nc += __popcll(m);
  }
  wave_sync();
  wave_rank_sort(cs, srt, nc, lane);
  const int kept = wave_select(a.base, a.d, j, srt, nc, a.cos2a, a.R, kid, klen, lane);
  for (int t = lane; t < a.R; t += 64) a.out[j * a.R + t] = t < kept ? kid[t] : kSent;
}

// ------------------------------------------------------------- exact SSG
// Alg. 2 over all pairs: node i's candidates are all other points in
// ascending (distance, id) order (distance 0 dropped), selected by the rule
// of wave_select without a degree bound. One wavefront per node; the
// candidates are sorted by a bitonic network in a workspace slice, and lane k
// tests a candidate against kept edges k, k + 64, ...
struct ExactArgs {
  const float* base;
  int64_t n;
  int d;
  double cos2a;
  int cap;
  int64_t first;       // first node of this launch
  int64_t npad;        // sort length (power of two >= n)
  Cand* scratch;       // [nodes per launch][npad]
  uint32_t* kept_id;   // [nodes per launch][n]
  double* kept_len;    // [nodes per launch][n]
  uint32_t* out;       // n x cap
  int32_t* deg;        // n
};

__global__ __launch_bounds__(64) void exact_ssg_kernel(ExactArgs a) {
#pragma clang fp contract(off)
  const int lane = threadIdx.x;
  const int64_t slot = blockIdx.x;
  const int64_t i = a.first + slot;
  if (i >= a.n) return;
  Cand* c = a.scratch + slot * a.npad;
  uint32_t* kid = a.kept_id + slot * a.n;
  double* klen = a.kept_len + slot * a.n;
  const float* xi = a.base + i * a.d;
  for (int64_t j = lane; j < a.npad; j += 64) {
    Cand v;
    v.id = (uint32_t)j;
    v.pad = 0;
    v.dist = INFINITY;  // padding, itself and distance 0 sort last and are cut
    if (j < a.n && j != i) {
      const double dd = ssgdev::exact_l2(xi, a.base + j * a.d, a.d);
      if (dd != 0.0) v.dist = dd;
    }
    if (j >= a.n) v.id = kSent;
    c[j] = v;
  }
  __syncthreads();  // one wavefront per block; orders its global scratch accesses
  // bitonic sort of npad entries by (dist, id)
  for (int64_t k = 2; k <= a.npad; k <<= 1) {
    for (int64_t jj = k >> 1; jj > 0; jj >>= 1) {
      for (int64_t t = lane; t < a.npad; t += 64) {
        const int64_t u = t ^ jj;
        if (u > t) {
          const Cand x = c[t], y = c[u];
          const bool up = (t & k) == 0;
          if (up ? cand_less(y, x) : cand_less(x, y)) {
            c[t] = y;
            c[u] = x;
          }
        }
      }
      __syncthreads();  // one wavefront per block; orders its global scratch accesses
    }
  }
  int kept = 0;
  for (int64_t cc = 0; cc < a.n; ++cc) {
    const Cand cd = c[cc];
    if (cd.dist == INFINITY) break;
    const float* xc = a.base + (int64_t)cd.id * a.d;
    bool conflict = false;
    for (int k = lane; k < kept && !conflict; k += 64) {
      const double dot = ssgdev::dot_rel(xc, a.base + (int64_t)kid[k] * a.d, xi, a.d);
      conflict = dot > 0.0 && dot * dot > a.cos2a * cd.dist * klen[k];
    }
    if (__ballot(conflict) == 0) {
      if (lane == 0) {
        kid[kept] = cd.id;
        klen[kept] = cd.dist;
      }
      ++kept;
      __syncthreads();  // one wavefront per block; orders its global scratch accesses
    }
  }
  for (int t = lane; t < a.cap; t += 64) a.out[i * a.cap + t] = t < kept ? kid[t] : kSent;
  if (lane == 0) a.deg[i] = kept;
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

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr int64_t EXACT_CHUNK = 1024;  // nodes per exact-SSG launch

int64_t pow2_at_least(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

struct RevLayout {
  size_t cnt, fill, off, bsum, rev, scratch, total;
};

RevLayout rev_layout(int64_t n, int R) {
  RevLayout L{};
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  size_t o = 0;
  auto take = [&](size_t b) { size_t r = o; o = align256(o + b); return r; };
  L.cnt = take((size_t)n * 4);
  L.fill = take((size_t)n * 4);
  L.off = take((size_t)(n + 1) * 4);
  L.bsum = take((size_t)(nb + 1) * 4);
  L.rev = take((size_t)n * R * 4);
  L.scratch = take((size_t)4 * n * R * sizeof(Cand));
  L.total = o;
  return L;
}

}  // namespace

extern "C" {

size_t ssg_exact_ssg_workspace_bytes(int64_t n) {
  if (n < 2) return 0;
  const int64_t npad = pow2_at_least(n);
  return align256((size_t)EXACT_CHUNK * npad * sizeof(Cand)) + align256((size_t)EXACT_CHUNK * n * 4) +
         align256((size_t)EXACT_CHUNK * n * 8);
}

int ssg_exact_ssg(const float* base, int64_t n, int32_t d, double cos2a, int32_t cap, uint32_t* out,
                  int32_t* deg, void* workspace, size_t workspace_bytes, void* stream) {
  if (!base || !out || !deg || !workspace) return fail_msg(SSG_EINVAL, "ssg_exact_ssg: null pointer argument");
  if (n < 2 || n > (1 << 20) || d < 1 || cap < 1)
    return fail_msg(SSG_EINVAL, "ssg_exact_ssg: n=%lld d=%d cap=%d out of range (n <= 2^20)", (long long)n, d, cap);
  if (!(cos2a >= 0.0 && cos2a <= 1.0)) return fail_msg(SSG_EINVAL, "ssg_exact_ssg: cos2a outside [0, 1]");
  const size_t need = ssg_exact_ssg_workspace_bytes(n);
  if (workspace_bytes < need)
    return fail_msg(SSG_EINVAL, "ssg_exact_ssg: workspace of %zu bytes, %zu needed", workspace_bytes, need);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail_msg(SSG_EINVAL, "ssg_exact_ssg: workspace not 256-byte aligned");
  const int64_t npad = pow2_at_least(n);
  char* w = static_cast<char*>(workspace);
  ExactArgs a{};
  a.base = base;
  a.n = n;
  a.d = d;
  a.cos2a = cos2a;
  a.cap = cap;
  a.npad = npad;
  a.scratch = reinterpret_cast<Cand*>(w);
  a.kept_id = reinterpret_cast<uint32_t*>(w + align256((size_t)EXACT_CHUNK * npad * sizeof(Cand)));
  a.kept_len = reinterpret_cast<double*>(w + align256((size_t)EXACT_CHUNK * npad * sizeof(Cand)) +
                                         align256((size_t)EXACT_CHUNK * n * 4));
  a.out = out;
  a.deg = deg;
  hipStream_t s = static_cast<hipStream_t>(stream);
  for (int64_t f = 0; f < n; f += EXACT_CHUNK) {
    a.first = f;
    const int64_t m = n - f < EXACT_CHUNK ? n - f : EXACT_CHUNK;
    hipLaunchKernelGGL(exact_ssg_kernel, dim3((unsigned)m), dim3(64), 0, s, a);
  }
  if (hipGetLastError() != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_exact_ssg: launch failed: %s", hipGetErrorString(hipGetLastError()));
  ssg_internal_clear_error();
  return SSG_OK;
}

int ssg_nssg_prune(const float* base, int64_t n, int32_t d, const uint32_t* knn, int32_t Kk,
                   int32_t l, int32_t R, double cos2a, uint32_t* out, void* stream) {
  if (!base || !knn || !out) return fail_msg(SSG_EINVAL, "ssg_nssg_prune: null pointer argument");
  if (n < 1 || n >= (int64_t)kSent || d < 1 || Kk < 1 || l < 1 || R < 1 || R > RMAX)
    return fail_msg(SSG_EINVAL, "ssg_nssg_prune: n=%lld d=%d Kk=%d l=%d R=%d out of range", (long long)n,
                    d, Kk, l, R);
  if (l + Kk + 2 > PCAP)
    return fail_msg(SSG_EUNSUPPORTED, "ssg_nssg_prune: l + Kk = %d exceeds %d candidates", l + Kk, PCAP - 2);
  if (!(cos2a >= 0.0 && cos2a <= 1.0)) return fail_msg(SSG_EINVAL, "ssg_nssg_prune: cos2a outside [0, 1]");
  hipStream_t s = static_cast<hipStream_t>(stream);
  PruneArgs a{base, n, d, knn, Kk, l, R, cos2a, out};
  if (l + Kk + 2 <= 256)
    hipLaunchKernelGGL(prune_kernel<256>, dim3((unsigned)n), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL(prune_kernel<PCAP>, dim3((unsigned)n), dim3(64), 0, s, a);
  if (hipGetLastError() != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_nssg_prune: launch failed: %s", hipGetErrorString(hipGetLastError()));
  ssg_internal_clear_error();
  return SSG_OK;
}

size_t ssg_nssg_reverse_workspace_bytes(int64_t n, int32_t R) {
  if (n < 1 || R < 1) return 0;
  return rev_layout(n, R).total;
}

int ssg_nssg_reverse(const float* base, int64_t n, int32_t d, const uint32_t* g1, int32_t R,
                     double cos2a, uint32_t* out, void* workspace, size_t workspace_bytes,
                     void* stream) {
  if (!base || !g1 || !out || !workspace)
    return fail_msg(SSG_EINVAL, "ssg_nssg_reverse: null pointer argument");
  if (n < 1 || n >= (int64_t)kSent || d < 1 || R < 1 || R > RMAX || n * R >= (int64_t)kSent)
    return fail_msg(SSG_EINVAL, "ssg_nssg_reverse: n=%lld d=%d R=%d out of range", (long long)n, d, R);
  if (!(cos2a >= 0.0 && cos2a <= 1.0)) return fail_msg(SSG_EINVAL, "ssg_nssg_reverse: cos2a outside [0, 1]");
  const RevLayout L = rev_layout(n, R);
  if (workspace_bytes < L.total)
    return fail_msg(SSG_EINVAL, "ssg_nssg_reverse: workspace of %zu bytes, %zu needed", workspace_bytes, L.total);
  if (reinterpret_cast<uintptr_t>(workspace) & 255)
    return fail_msg(SSG_EINVAL, "ssg_nssg_reverse: workspace not 256-byte aligned");
  hipStream_t s = static_cast<hipStream_t>(stream);
  char* w = static_cast<char*>(workspace);
  uint32_t* cnt = reinterpret_cast<uint32_t*>(w + L.cnt);
  uint32_t* fill = reinterpret_cast<uint32_t*>(w + L.fill);
  uint32_t* off = reinterpret_cast<uint32_t*>(w + L.off);
  uint32_t* bsum = reinterpret_cast<uint32_t*>(w + L.bsum);
  uint32_t* rev = reinterpret_cast<uint32_t*>(w + L.rev);
  Cand* scratch = reinterpret_cast<Cand*>(w + L.scratch);
  const int64_t edges = n * R;
  const int64_t nb = (n + SCAN_B - 1) / SCAN_B;
  if (hipMemsetAsync(cnt, 0, (size_t)n * 4, s) != hipSuccess || hipMemsetAsync(fill, 0, (size_t)n * 4, s) != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_nssg_reverse: memset failed");
  hipLaunchKernelGGL(rev_count, dim3((unsigned)((edges + 255) / 256)), dim3(256), 0, s, g1, n, R, cnt);
  hipLaunchKernelGGL(scan_blocks, dim3((unsigned)nb), dim3(SCAN_B), 0, s, cnt, n, off, bsum);
  hipLaunchKernelGGL(scan_sums, dim3(1), dim3(SCAN_B), 0, s, bsum, nb);
  hipLaunchKernelGGL(scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, off, n, bsum, nb);
  hipLaunchKernelGGL(rev_fill, dim3((unsigned)((edges + 255) / 256)), dim3(256), 0, s, g1, n, R, off, fill, rev);
  ReverseArgs a{base, n, d, g1, R, cos2a, off, rev, scratch, out};
  hipLaunchKernelGGL(reverse_kernel, dim3((unsigned)n), dim3(64), 0, s, a);
  if (hipGetLastError() != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_nssg_reverse: launch failed: %s", hipGetErrorString(hipGetLastError()));
  ssg_internal_clear_error();
  return SSG_OK;
}

}  // extern "C"
