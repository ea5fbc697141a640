// ssg_merge.hip -- the aggregation step of the partitioned search (Sec. 6.5):
// the data set is split into S random shards with one graph each, every
// query is searched in every shard, and the S per-shard result lists are
// merged into one list by (distance, global id).
//
// One wavefront per query. Its S x K candidates go to LDS as 64-bit keys
// ord(dist) << 32 | global id (padding gets distinct keys above every real
// one); each shard's list is rank-sorted (a shard orders equal distances by
// its local ids, which need not follow the global ones), then every candidate
// finds its output position as its index in its own list plus, for each
// other list, the number of smaller keys there (binary search).

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cstdarg>
#include <cstdio>

#include "ssg.h"
#include "ssg_internal.h"

namespace {

constexpr uint32_t kSent = 0xFFFFFFFFu;
constexpr int MAX_KEYS = 4096;  // S * K per query (LDS: 16 bytes per key)

__device__ __forceinline__ uint32_t ord_f32(float f) {
  uint32_t b = __float_as_uint(f);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
  const uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(b);
}
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct MergeArgs {
  const uint32_t* ids;    // [S][nq][K] shard-local ids
  const float* dists;     // [S][nq][K]
  int S;
  int64_t nq;
  int K;
  const uint32_t* id_map;  // shard s, local id l -> id_map[map_off[s] + l]
  const int64_t* map_off;  // [S]
  int64_t map_len;         // entries of id_map
  int K_out;
  uint32_t* out_ids;       // [nq][K_out]
  float* out_dists;        // [nq][K_out]
};

__global__ __launch_bounds__(64) void merge_kernel(MergeArgs a) {
  extern __shared__ uint64_t dyn[];  // 2 S K keys
  const int lane = threadIdx.x;
  const int64_t q = blockIdx.x;
  const int K = a.K, S = a.S, tot = S * K;
  uint64_t* raw = dyn;
  uint64_t* srt = dyn + tot;
  for (int e = lane; e < tot; e += 64) {
    const int s = e / K, i = e % K;
    const int64_t src = ((int64_t)s * a.nq + q) * K + i;
    const uint32_t l = a.ids[src];
    uint64_t key;
    const int64_t at = a.map_off[s] + (int64_t)l;
    if (l == kSent || at < 0 || at >= a.map_len) {
      key = ~0ull - (uint64_t)e;  // padding (or an id outside the map): above every real key
    } else {
      const uint32_t g = a.id_map[at];
      key = ((uint64_t)ord_f32(a.dists[src]) << 32) | g;
    }
    raw[e] = key;
  }
  wave_sync();
  // sort each shard's list by (dist, global id)
  for (int e = lane; e < tot; e += 64) {
    const int s = e / K;
    const uint64_t k = raw[e];
    int r = 0;
    for (int f = s * K; f < s * K + K; ++f) r += raw[f] < k;
    srt[s * K + r] = k;
  }
  wave_sync();
  for (int e = lane; e < tot; e += 64) {
    const int s = e / K, i = e % K;
    const uint64_t k = srt[e];
    int pos = i;
    for (int t = 0; t < S && pos < a.K_out; ++t) {
      if (t == s) continue;
      const uint64_t* lt = srt + t * K;
      int lo = 0, hi = K;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (lt[mid] < k) lo = mid + 1; else hi = mid;
      }
      pos += lo;
    }
    if (pos < a.K_out) {
      const bool pad = (k >> 32) > 0xFF800000ull;  // above ord(+inf): padding
      a.out_ids[q * a.K_out + pos] = pad ? kSent : (uint32_t)k;
      a.out_dists[q * a.K_out + pos] = pad ? INFINITY : unord_f32((uint32_t)(k >> 32));
    }
  }
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

extern "C" int ssg_merge_shards(const uint32_t* ids, const float* dists, int32_t S, int64_t nq,
                                int32_t K, const uint32_t* id_map, const int64_t* map_off,
                                int64_t map_len, int32_t K_out, uint32_t* out_ids, float* out_dists,
                                void* stream) {
  if (nq < 0 || S < 1 || K < 1 || K_out < 1 || map_len < 0)
    return fail_msg(SSG_EINVAL, "ssg_merge_shards: S=%d K=%d K_out=%d nq=%lld map_len=%lld", S, K,
                    K_out, (long long)nq, (long long)map_len);
  if ((int64_t)S * K > MAX_KEYS)
    return fail_msg(SSG_EUNSUPPORTED, "ssg_merge_shards: S * K = %d exceeds %d", S * K, MAX_KEYS);
  if (K_out > S * K) return fail_msg(SSG_EINVAL, "ssg_merge_shards: K_out above S * K");
  if (nq == 0) { ssg_internal_clear_error(); return SSG_OK; }
  if (!ids || !dists || !id_map || !map_off || !out_ids || !out_dists)
    return fail_msg(SSG_EINVAL, "ssg_merge_shards: null pointer argument");
  if (nq > 0x7FFFFFFF) return fail_msg(SSG_EINVAL, "ssg_merge_shards: nq too large for one launch");
  MergeArgs a{ids, dists, S, nq, K, id_map, map_off, map_len, K_out, out_ids, out_dists};
  hipLaunchKernelGGL(merge_kernel, dim3((unsigned)nq), dim3(64), (size_t)16 * S * K,
                     static_cast<hipStream_t>(stream), a);
  if (hipGetLastError() != hipSuccess)
    return fail_msg(SSG_EDEVICE, "ssg_merge_shards: launch failed");
  ssg_internal_clear_error();
  return SSG_OK;
}
