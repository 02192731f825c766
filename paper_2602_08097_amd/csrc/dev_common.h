// dev_common.h -- device helpers shared by the HIP kernels.
#pragma once

#include "rp_internal.h"

namespace rp {

// Canonical FP64 squared distance of two float32 rows: t = (double)a - (double)b
// rounded once, accumulated with a correctly rounded fused multiply-add in
// ascending k.  Built with -ffp-contract=off so no other fusion happens.
__device__ __forceinline__ double canon_sq_f32(const float* __restrict__ a,
                                               const float* __restrict__ b, int d) {
  double acc = 0.0;
  for (int k = 0; k < d; ++k) {
    double t = (double)a[k] - (double)b[k];
    acc = __fma_rn(t, t, acc);
  }
  return acc;
}

// Exact squared distance of two uint8 rows (d <= 4096 keeps it below 2^31).
__device__ __forceinline__ uint32_t sq_u8(const uint8_t* __restrict__ a,
                                          const uint8_t* __restrict__ b, int d) {
  uint32_t acc = 0;
  for (int k = 0; k < d; ++k) {
    int t = (int)a[k] - (int)b[k];
    acc += (uint32_t)(t * t);
  }
  return acc;
}

// FP32 direct-difference squared distance (approximate).
__device__ __forceinline__ float sq_f32(const float* __restrict__ a,
                                        const float* __restrict__ b, int d) {
  float acc = 0.f;
  for (int k = 0; k < d; ++k) {
    float t = a[k] - b[k];
    acc = __fmaf_rn(t, t, acc);
  }
  return acc;
}

// Pruning condition of Algorithm 1 on squares, exact for integers:
// num^2 * s_star <= den^2 * s_p.
__device__ __forceinline__ bool alpha_test_int(uint32_t num2, uint32_t den2, uint32_t s_star,
                                               uint32_t s_p) {
  return (uint64_t)num2 * s_star <= (uint64_t)den2 * s_p;
}

// Same condition for float32 data, as defined on canonical FP64 values.
__device__ __forceinline__ bool alpha_test_f64(uint32_t num2, uint32_t den2, double s_star,
                                               double s_p) {
  double lhs = (double)num2 * s_star;
  double rhs = (double)den2 * s_p;
  return lhs <= rhs;
}

// (S, id) lexicographic "strictly before".
__device__ __forceinline__ bool before_f64(double sa, int ia, double sb, int ib) {
  return sa < sb || (sa == sb && ia < ib);
}

// Decide the float32 pruning condition from an approximate S~ of S(p*, p')
// known to satisfy |S~ - S_canonical| <= rel * S_canonical.  Returns 1 (prune),
// 0 (keep) or -1 (too close to call: recheck in canonical FP64).
__device__ __forceinline__ int decide_approx(uint32_t num2, uint32_t den2, double s_approx,
                                             double s_p, double rel) {
  if (!(s_approx >= 1e-25 && s_approx <= 1e30)) return -1;
  double lhs = (double)num2 * s_approx;
  double rhs = (double)den2 * s_p;
  if (lhs * (1.0 + rel) <= rhs) return 1;
  if (lhs * (1.0 - rel) > rhs) return 0;
  return -1;
}

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace rp
