// ssg_search_common.h -- device helpers, storage decoders and the kernel
// argument block shared by the search kernels (one query per wavefront in
// ssg_search.hip, several queries per wavefront in ssg_groups.hip). The
// argument block has one layout for every kernel (namespace ssgk); every
// other definition sits in an unnamed namespace, so each translation unit
// keeps its own copy. Nothing here is part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// The kernels' argument block (passed by value; one layout for every search
// kernel of the library).
namespace ssgk {
struct Args {
  const unsigned char* base;  // n x (DC * 16) bytes
  int64_t n;
  int32_t d;
  int32_t dc;                 // 16-byte chunks per vector
  const float* dim_scale;     // fp8 only
  const uint32_t* graph;
  int32_t R;
  const uint32_t* entry;
  int32_t s;
  const float* queries;
  int64_t nq;
  int32_t K, L, metric;
  uint32_t* out_ids;
  float* out_d;
  int32_t* out_ndc;
  int32_t* out_hops;
  int32_t vmode;       // visited form: 0 exact bitset, 1 hash, 2 tag cache
  int32_t hash_log2;   // hash / cache: log2 of the number of entries
  int32_t id_bits;     // cache: k, with every id < 2^k (k - (hash_log2 - 2) <= 15)
  int32_t lds_per_wave;
  const float* base_f32;  // FP32 vectors for the final rerank, or null
  int32_t rerank;         // pool entries to rerank (<= 64 * PREG); -1: K of each query
  // batched / persistent mode
  const int32_t* qlist;   // query indices processed by this launch, or null (0..nlist)
  int64_t nlist;          // number of entries of qlist (or queries)
  const int32_t* L_arr;   // per-query pool size, or null (L)
  const int32_t* K_arr;   // per-query result count, or null (K)
  int32_t kstride;        // output row stride (>= every K)
  uint32_t* counter;      // persistent work queue head, or null (one query per wave)
  int64_t entry_group;    // > 0: query i uses entry[(i / entry_group) * s ...]; 0: all share
  uint32_t* out_trace;    // nq x trace_cap expanded ids in expansion order, or null
  int32_t trace_cap;
};
using KernelFn = void (*)(Args);
}  // namespace ssgk

namespace {

constexpr uint32_t kSent = 0xFFFFFFFFu;
constexpr uint64_t kNoKey = ~0ull;

// ------------------------------------------------------------------ helpers
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Monotone map of a float to uint32 (negative zero folded onto positive zero).
__device__ __forceinline__ uint32_t ord_f32(float f) {
  uint32_t b = __float_as_uint(f);
  if (b == 0x80000000u) b = 0u;
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o & 0x7FFFFFFFu) : ~o;
  return __uint_as_float(b);
}
__device__ __forceinline__ uint64_t make_key(float dist, uint32_t id) {
  return ((uint64_t)ord_f32(dist) << 32) | (uint32_t)(id << 1);
}
// The same key for a distance known to be >= +0 (a sum of squares that
// starts at +0 is never -0): its order code is its bits with the sign set.
__device__ __forceinline__ uint64_t make_key_nonneg(float dist, uint32_t id) {
  return ((uint64_t)(__float_as_uint(dist) | 0x80000000u) << 32) | (uint32_t)(id << 1);
}
__device__ __forceinline__ uint32_t key_id(uint64_t k) { return (uint32_t)(k >> 1) & 0x7FFFFFFFu; }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int lane) {
  uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor64(uint64_t v, int m) {
  uint32_t lo = __shfl_xor((int)(uint32_t)v, m, 64);
  uint32_t hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)hi << 32) | lo;
}
// x + the value of lane ^ OFF. Within a row of 16 lanes the partner comes
// from a DPP lane move (VALU; row_shr:n reads lane i - n, row_shl:n lane
// i + n, quad_perm permutes each quad), across rows from a lane shuffle.
// Call with every lane active.
template <int CTRL>
__device__ __forceinline__ float dpp_f32(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int OFF>
__device__ __forceinline__ float add_xor_lane(float x, int lane) {
  if constexpr (OFF == 1) return x + dpp_f32<0xB1>(x);  // quad_perm [1,0,3,2]
  if constexpr (OFF == 2) return x + dpp_f32<0x4E>(x);  // quad_perm [2,3,0,1]
  if constexpr (OFF == 4 || OFF == 8) {
    const float lo = dpp_f32<0x110 + OFF>(x);  // row_shr: lane - OFF
    const float hi = dpp_f32<0x100 + OFF>(x);  // row_shl: lane + OFF
    return x + ((lane & OFF) ? lo : hi);
  }
  if constexpr (OFF >= 16) return x + __shfl_xor(x, OFF, 64);
}
// Sum over each aligned group of G lanes, on every lane of the group; the
// same additions in the same order as a butterfly of lane shuffles from
// offset G/2 down to 1.
template <int G>
__device__ __forceinline__ float group_sum(float x, int lane) {
  if constexpr (G >= 64) x = add_xor_lane<32>(x, lane);
  if constexpr (G >= 32) x = add_xor_lane<16>(x, lane);
  if constexpr (G >= 16) x = add_xor_lane<8>(x, lane);
  if constexpr (G >= 8) x = add_xor_lane<4>(x, lane);
  if constexpr (G >= 4) x = add_xor_lane<2>(x, lane);
  if constexpr (G >= 2) x = add_xor_lane<1>(x, lane);
  return x;
}

// Minimum of a 64-bit value over the wavefront, read back on every lane.
// Row-local DPP shifts (VALU latency, not the LDS pipe of lane shuffles)
// reduce each row of 16 into its lane 15; row broadcasts fold the four rows
// into lane 63.
template <int CTRL>
__device__ __forceinline__ uint64_t dpp_min64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_update_dpp(0xFFFFFFFFu, (uint32_t)v, CTRL, 0xF, 0xF, false);
  const uint32_t hi = __builtin_amdgcn_update_dpp(0xFFFFFFFFu, (uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
  const uint64_t o = ((uint64_t)hi << 32) | lo;
  return o < v ? o : v;
}
// Minimum of a 32-bit value over the wavefront: row shifts and row
// broadcasts of the DPP unit, each folded into one v_min with its DPP
// operand; a lane without a source lane keeps its own value.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_min32(uint32_t v) {
  return min(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ uint32_t wave_min32(uint32_t v) {
  v = dpp_min32<0x111>(v);
  v = dpp_min32<0x112>(v);
  v = dpp_min32<0x114>(v);
  v = dpp_min32<0x118>(v);
  v = dpp_min32<0x142>(v);
  v = dpp_min32<0x143>(v);
  return __builtin_amdgcn_readlane(v, 63);
}
// 64-bit minimum as two 32-bit ones: the high words, then the low words of
// the lanes holding the smallest high word.
__device__ __forceinline__ uint64_t wave_min64_split(uint64_t v) {
  const uint32_t hi = wave_min32((uint32_t)(v >> 32));
  const uint32_t lo = wave_min32((uint32_t)(v >> 32) == hi ? (uint32_t)v : 0xFFFFFFFFu);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t wave_min64(uint64_t v) {
  v = dpp_min64<0x111>(v);  // row_shr:1
  v = dpp_min64<0x112>(v);  // row_shr:2
  v = dpp_min64<0x114>(v);  // row_shr:4
  v = dpp_min64<0x118>(v);  // row_shr:8
  v = dpp_min64<0x142>(v);  // row_bcast:15
  v = dpp_min64<0x143>(v);  // row_bcast:31
  return readlane64(v, 63);
}

__device__ __forceinline__ int lane_prefix(uint64_t mask) {  // set bits below this lane
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}
__device__ __forceinline__ uint32_t hash_slot(uint32_t id, uint32_t mask) {
  return (id * 0x9E3779B1u) >> 7 & mask;
}

// ------------------------------------------------------------------ vector types
// A "chunk" is 16 bytes of a stored vector: 4 f32, 8 bf16 or 16 fp8 values.
struct F32T {
  static constexpr int kEpc = 4;
  static constexpr bool kScaled = false;
  __device__ static __forceinline__ void decode(uint4 c, float* x) {
    x[0] = __uint_as_float(c.x);
    x[1] = __uint_as_float(c.y);
    x[2] = __uint_as_float(c.z);
    x[3] = __uint_as_float(c.w);
  }
};
struct BF16T {
  static constexpr int kEpc = 8;
  static constexpr bool kScaled = false;
  __device__ static __forceinline__ void decode(uint4 c, float* x) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      x[2 * i] = __uint_as_float(w[i] << 16);
      x[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
  }
};
// OCP FP8 E4M3 (bias 7, no infinities, S.1111.111 is NaN): exact decode by
// bit placement for normal codes and by one multiply for subnormal codes.
struct FP8T {
  static constexpr int kEpc = 16;
  static constexpr bool kScaled = true;
  __device__ static __forceinline__ float one(uint32_t b) {
    uint32_t s = (b & 0x80u) << 24;
    uint32_t e = (b >> 3) & 0xFu;
    uint32_t m = b & 0x7u;
    float v = (e == 0u) ? (float)m * 0.001953125f  // m * 2^-9
                        : __uint_as_float(((e + 120u) << 23) | (m << 20));
    return __uint_as_float(__float_as_uint(v) | s);
  }
  __device__ static __forceinline__ void decode(uint4 c, float* x) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
#pragma unroll
      for (int b = 0; b < 4; ++b) x[4 * i + b] = one((w[i] >> (8 * b)) & 0xFFu);
    }
  }
};

// The same E4M3 decode through gfx950's packed conversion instruction (two
// codes per instruction instead of a dozen integer operations per code).
struct FP8HwT {
  static constexpr int kEpc = 16;
  static constexpr bool kScaled = true;
  __device__ static __forceinline__ void decode(uint4 c, float* x) {
    const uint32_t w[4] = {c.x, c.y, c.z, c.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], false);
      const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8((int)w[i], true);
      x[4 * i] = lo[0];
      x[4 * i + 1] = lo[1];
      x[4 * i + 2] = hi[0];
      x[4 * i + 3] = hi[1];
    }
  }
};



using ssgk::Args;
using ssgk::KernelFn;

}  // namespace
