// dev_common.h -- device helpers shared by the HIP kernels.
#pragma once

#include "rp_internal.h"

namespace rp {

// Canonical FP64 squared distance of two float32 rows: t = (double)a - (double)b
// rounded once, accumulated with a correctly rounded fused multiply-add in
// ascending k.  Built with -ffp-contract=off so no other fusion happens.
// (16-byte loads when both rows are 16-byte aligned and d % 4 == 0; the
// evaluation order is the same.)
__device__ __forceinline__ double canon_sq_f32(const float* __restrict__ a,
                                               const float* __restrict__ b, int d) {
  double acc = 0.0;
  int k = 0;
  if ((((uintptr_t)a | (uintptr_t)b) & 15) == 0 && (d & 3) == 0) {
    // unrolled so that several 16-byte loads are in flight before the
    // multiply-add chain consumes them (one round trip per 32 dimensions)
#pragma unroll 8
    for (; k < d; k += 4) {
      const float4 x = *(const float4*)(a + k);
      const float4 y = *(const float4*)(b + k);
      double t = (double)x.x - (double)y.x;
      acc = __fma_rn(t, t, acc);
      t = (double)x.y - (double)y.y;
      acc = __fma_rn(t, t, acc);
      t = (double)x.z - (double)y.z;
      acc = __fma_rn(t, t, acc);
      t = (double)x.w - (double)y.w;
      acc = __fma_rn(t, t, acc);
    }
  }
  for (; k < d; ++k) {
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

// FP32 direct-difference squared distance (approximate), sequential in k;
// 16-byte loads when both rows are 16-byte aligned and d % 4 == 0.
__device__ __forceinline__ float sq_f32(const float* __restrict__ a,
                                        const float* __restrict__ b, int d) {
  float acc = 0.f;
  int k = 0;
  if ((((uintptr_t)a | (uintptr_t)b) & 15) == 0 && (d & 3) == 0) {
#pragma unroll 8
    for (; k < d; k += 4) {
      const float4 x = *(const float4*)(a + k);
      const float4 y = *(const float4*)(b + k);
      float t = x.x - y.x;
      acc = __fmaf_rn(t, t, acc);
      t = x.y - y.y;
      acc = __fmaf_rn(t, t, acc);
      t = x.z - y.z;
      acc = __fmaf_rn(t, t, acc);
      t = x.w - y.w;
      acc = __fmaf_rn(t, t, acc);
    }
  }
  for (; k < d; ++k) {
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

// Lane exchange with partner lane ^ J (J a power of two).
template <int J>
__device__ __forceinline__ int xchg(int v) {
  if constexpr (J == 1) return __builtin_amdgcn_update_dpp(0, v, 0xB1, 0xF, 0xF, false);
  else if constexpr (J == 2) return __builtin_amdgcn_update_dpp(0, v, 0x4E, 0xF, 0xF, false);
  else if constexpr (J == 4) return __builtin_amdgcn_ds_swizzle(v, 0x101F);
  else if constexpr (J == 8) return __builtin_amdgcn_update_dpp(0, v, 0x128, 0xF, 0xF, false);
  else if constexpr (J == 16) return __builtin_amdgcn_ds_swizzle(v, 0x401F);
  else return __shfl_xor(v, 32, 64);
}

template <int K, int J>
__device__ __forceinline__ uint64_t bitonic_step(uint64_t key, int lane) {
  const int lo = xchg<J>((int)(uint32_t)key);
  const int hi = xchg<J>((int)(uint32_t)(key >> 32));
  const uint64_t other = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
  const bool take_min = ((lane & J) == 0) == ((lane & K) == 0);
  const uint64_t mn = key < other ? key : other;
  const uint64_t mx = key < other ? other : key;
  return take_min ? mn : mx;
}

// Ascending bitonic sort of one 64-bit key per lane across the wavefront.
__device__ __forceinline__ uint64_t wave_sort(uint64_t k, int lane) {
  k = bitonic_step<2, 1>(k, lane);
  k = bitonic_step<4, 2>(k, lane);
  k = bitonic_step<4, 1>(k, lane);
  k = bitonic_step<8, 4>(k, lane);
  k = bitonic_step<8, 2>(k, lane);
  k = bitonic_step<8, 1>(k, lane);
  k = bitonic_step<16, 8>(k, lane);
  k = bitonic_step<16, 4>(k, lane);
  k = bitonic_step<16, 2>(k, lane);
  k = bitonic_step<16, 1>(k, lane);
  k = bitonic_step<32, 16>(k, lane);
  k = bitonic_step<32, 8>(k, lane);
  k = bitonic_step<32, 4>(k, lane);
  k = bitonic_step<32, 2>(k, lane);
  k = bitonic_step<32, 1>(k, lane);
  k = bitonic_step<64, 32>(k, lane);
  k = bitonic_step<64, 16>(k, lane);
  k = bitonic_step<64, 8>(k, lane);
  k = bitonic_step<64, 4>(k, lane);
  k = bitonic_step<64, 2>(k, lane);
  k = bitonic_step<64, 1>(k, lane);
  return k;
}

// Ascending bitonic sort of (hi, lo) pairs across the wavefront, compared
// lexicographically.
template <int K, int J>
__device__ __forceinline__ void bitonic_step2(uint64_t& hi, uint32_t& lo, int lane) {
  const int oh0 = xchg<J>((int)(uint32_t)hi);
  const int oh1 = xchg<J>((int)(uint32_t)(hi >> 32));
  const uint32_t olo = (uint32_t)xchg<J>((int)lo);
  const uint64_t ohi = ((uint64_t)(uint32_t)oh1 << 32) | (uint32_t)oh0;
  const bool mine_less = hi < ohi || (hi == ohi && lo < olo);
  const bool take_min = ((lane & J) == 0) == ((lane & K) == 0);
  if (take_min != mine_less) {
    hi = ohi;
    lo = olo;
  }
}

__device__ __forceinline__ void wave_sort2(uint64_t& hi, uint32_t& lo, int lane) {
  bitonic_step2<2, 1>(hi, lo, lane);
  bitonic_step2<4, 2>(hi, lo, lane);
  bitonic_step2<4, 1>(hi, lo, lane);
  bitonic_step2<8, 4>(hi, lo, lane);
  bitonic_step2<8, 2>(hi, lo, lane);
  bitonic_step2<8, 1>(hi, lo, lane);
  bitonic_step2<16, 8>(hi, lo, lane);
  bitonic_step2<16, 4>(hi, lo, lane);
  bitonic_step2<16, 2>(hi, lo, lane);
  bitonic_step2<16, 1>(hi, lo, lane);
  bitonic_step2<32, 16>(hi, lo, lane);
  bitonic_step2<32, 8>(hi, lo, lane);
  bitonic_step2<32, 4>(hi, lo, lane);
  bitonic_step2<32, 2>(hi, lo, lane);
  bitonic_step2<32, 1>(hi, lo, lane);
  bitonic_step2<64, 32>(hi, lo, lane);
  bitonic_step2<64, 16>(hi, lo, lane);
  bitonic_step2<64, 8>(hi, lo, lane);
  bitonic_step2<64, 4>(hi, lo, lane);
  bitonic_step2<64, 2>(hi, lo, lane);
  bitonic_step2<64, 1>(hi, lo, lane);
}

// Orders the LDS accesses of one wavefront's lanes around this point (a
// workgroup holds several independent wavefronts, each on its own vertex and
// its own LDS region, so no workgroup barrier is needed).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Power-of-two scale of a float32 vertex frame: |x_jk - x_pk| <= bound <
// 2^ex, e = 14 - ex, so every scaled difference is below 2^14 in magnitude.
// The bound is a sum of two finite floats taken in FP64 (below 2^129), so
// ex <= 129 and e >= -115: 2^e stays a normal float.  The cap at 100 only
// shrinks the scaled values further.
__device__ __forceinline__ int frame_exponent(double bound) {
  int e = 0;
  if (bound > 0.0) {
    int ex;
    frexp(bound, &ex);
    e = min(100, max(-115, 14 - ex));
  }
  return e;
}

// A wave-uniform 64-bit value pinned to scalar registers.
__device__ __forceinline__ uint64_t uniform_u64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  int lo = __shfl((int)(uint32_t)v, src, 64);
  int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

}  // namespace rp
