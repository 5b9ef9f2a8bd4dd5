// zsort_mlp.h -- device functions of the learned partition map: a monotone
// multilayer perceptron 1 -> 32 -> 32 -> 1 that approximates the keys' CDF.
// With non-negative weights and the clamp to [0, 1] as activation, every
// operation is non-decreasing in its input, so the map
//   cluster(x) = min(B - 1, floor(B * clamp(f(u(x)), 0, 1)))
// never puts a larger key into a smaller cluster, which is what zSort's
// distribution pass needs of its map (Section III: clusters must be ordered
// so that concatenating the sorted clusters sorts the array).
//
// Precision, fixed so that every implementation computes the same bits:
//   u(x)   = 0 below the range, 1 above it, else (x - smin) / (smax - smin)
//            in binary64;
//   layer 1: binary64 weights, product and sum, rounded once to binary32;
//   layers 2 and 3: binary32, every product and every sum rounded on its
//            own (no fused multiply-add), sums taken in index order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "zsort_internal.h"

namespace zs {

__device__ __forceinline__ double mlp_norm(uint64_t x, uint64_t smin, uint64_t smax) {
  if (x <= smin) return 0.0;
  if (x >= smax) return 1.0;
  return __ddiv_rn(__ull2double_rn(x - smin), __ull2double_rn(smax - smin));
}

__device__ __forceinline__ float clamp01(float a) { return a < 0.0f ? 0.0f : (a > 1.0f ? 1.0f : a); }

// f(u) (p in LDS or global memory)
__device__ inline float mlp_forward(const MlpP& p, double u) {
  float h1[kH];
#pragma unroll
  for (int i = 0; i < kH; ++i) {
    double a = __dmul_rn(p.w1[i], u);
    a = __dadd_rn(a, p.b1[i]);
    h1[i] = clamp01(__double2float_rn(a));
  }
  float f = p.b3;
#pragma unroll 1
  for (int j = 0; j < kH; ++j) {
    float acc = p.b2[j];
#pragma unroll
    for (int i = 0; i < kH; ++i) acc = __fadd_rn(acc, __fmul_rn(p.w2[j * kH + i], h1[i]));
    f = __fadd_rn(f, __fmul_rn(p.w3[j], clamp01(acc)));
  }
  return f;
}

__device__ __forceinline__ uint32_t mlp_cluster_of_f(float f, int B) {
  const float t = __fmul_rn((float)B, clamp01(f));
  const float fl = floorf(t);
  if (fl >= (float)(B - 1)) return (uint32_t)(B - 1);
  return (uint32_t)fl;
}

__device__ __forceinline__ uint32_t mlp_cluster(const MlpP& p, uint64_t x, uint64_t smin,
                                                uint64_t smax, int B) {
  return mlp_cluster_of_f(mlp_forward(p, mlp_norm(x, smin, smax)), B);
}

// copies the parameters into LDS (all threads of the workgroup take part)
__device__ __forceinline__ void mlp_load(MlpP& dst, const MlpP* src) {
  const uint32_t* s = reinterpret_cast<const uint32_t*>(src);
  uint32_t* d = reinterpret_cast<uint32_t*>(&dst);
  for (uint32_t i = threadIdx.x; i < sizeof(MlpP) / 4; i += blockDim.x) d[i] = s[i];
}

// number of thresholds <= x, i.e. the cluster of x under a non-decreasing
// map with thresholds t[0..nt) (ascending); fixed trip count, no divergence
__device__ __forceinline__ uint32_t thr_cluster(const uint64_t* t, uint32_t nt, uint32_t top,
                                                uint64_t x) {
  uint32_t pos = 0;
  for (uint32_t st = top; st; st >>= 1)
    if (pos + st <= nt && t[pos + st - 1] <= x) pos += st;
  return pos;
}

__device__ __forceinline__ uint32_t top_pow2(uint32_t nt) {
  return nt ? (1u << (31 - __clz(nt))) : 0u;
}

}  // namespace zs
