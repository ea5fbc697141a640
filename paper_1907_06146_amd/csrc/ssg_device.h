// ssg_device.h -- FP64 pair arithmetic shared by the index-building kernels.
// Every operation is rounded on its own (no fused multiply-add) and the
// dimensions are summed in order, so the values do not depend on the launch
// shape.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssgdev {

// Squared Euclidean distance: sum over j of (a_j - b_j)^2.
__device__ inline double exact_l2(const float* __restrict__ a, const float* __restrict__ b, int d) {
#pragma clang fp contract(off)
  double s = 0.0;
  int j = 0;
  if (((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0) {
    for (; j + 4 <= d; j += 4) {
      const float4 x = *reinterpret_cast<const float4*>(a + j);
      const float4 y = *reinterpret_cast<const float4*>(b + j);
      double t;
      t = (double)x.x - (double)y.x; s = s + t * t;
      t = (double)x.y - (double)y.y; s = s + t * t;
      t = (double)x.z - (double)y.z; s = s + t * t;
      t = (double)x.w - (double)y.w; s = s + t * t;
    }
  }
  for (; j < d; ++j) {
    const double t = (double)a[j] - (double)b[j];
    s = s + t * t;
  }
  return s;
}

// <a - c, b - c>: the inner product of two edge vectors leaving c.
__device__ inline double dot_rel(const float* __restrict__ a, const float* __restrict__ b,
                                 const float* __restrict__ c, int d) {
#pragma clang fp contract(off)
  double s = 0.0;
  int j = 0;
  if (((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b) | reinterpret_cast<uintptr_t>(c)) & 15) == 0) {
    for (; j + 4 <= d; j += 4) {
      const float4 x = *reinterpret_cast<const float4*>(a + j);
      const float4 y = *reinterpret_cast<const float4*>(b + j);
      const float4 z = *reinterpret_cast<const float4*>(c + j);
      s = s + ((double)x.x - (double)z.x) * ((double)y.x - (double)z.x);
      s = s + ((double)x.y - (double)z.y) * ((double)y.y - (double)z.y);
      s = s + ((double)x.z - (double)z.z) * ((double)y.z - (double)z.z);
      s = s + ((double)x.w - (double)z.w) * ((double)y.w - (double)z.w);
    }
  }
  for (; j < d; ++j) s = s + ((double)a[j] - (double)c[j]) * ((double)b[j] - (double)c[j]);
  return s;
}

}  // namespace ssgdev
