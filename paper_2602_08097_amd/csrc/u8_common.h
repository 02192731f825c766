// u8_common.h -- device helpers of the uint8 kernels (int8 matrix-unit
// operands, exact alpha thresholds and decision codes).
#pragma once

#include "dev_common.h"

namespace rp {
namespace u8 {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// floor(den2 * s / num2) for s < 2^28, exact, from M = floor(2^60 den2 / num2) + 1:
// 0 < s (M / 2^60 - den2 / num2) < 2^-32 < 1 / num2, less than the gap between a
// non-integer quotient and the next integer, so floor(16 s M / 2^64) is the
// floor (two 32 x 32 -> 64-bit multiply-adds).
__device__ __forceinline__ int32_t alpha_threshold(uint64_t M, uint32_t s) {
  const uint64_t s16 = (uint64_t)(s << 4);
  const uint64_t lo = s16 * (uint64_t)(uint32_t)M;
  const uint64_t hi = s16 * (M >> 32) + (lo >> 32);
  return (int32_t)(uint32_t)(hi >> 32);
}

// The decision bounds of this lane's tile column j.  Pair (i, j) is pruned at
// alpha_k  <=>  S(i, j) <= T_k(j)  <=>  y = 2 G(i, j) - |u_i|^2 >= U_k = |u_j|^2 - T_k(j).
// On Y = 16 y with B_k = 16 U_k and A_k = B_k - w_k, w_k = 2^(k mod 4), the median
// med3(Y, A_k, B_k) - A_k is w_k when Y >= B_k and 0 otherwise (Y and B_k are
// multiples of 16 > w_k), so the code 2^c - 1 is a sum of medians offset by
// -sum A_k: alphas 0..3 in the low nibble, 4..7 in the high one.
template <int NA>
struct ColBounds {
  int32_t A[NA], B[NA];
  int32_t off_lo, off_hi;
};

template <int NA>
__device__ __forceinline__ ColBounds<NA> col_bounds(int32_t ncol16, const int32_t (&T)[NA]) {
  ColBounds<NA> cb;
  cb.off_lo = 0;
  cb.off_hi = 0;
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    cb.B[k] = ncol16 - 16 * T[k];
    cb.A[k] = cb.B[k] - (1 << (k & 3));
    if (k < 4) cb.off_lo -= cb.A[k];
    else cb.off_hi -= cb.A[k];
  }
  return cb;
}

// One v_med3_i32 (the compiler keeps min(max()) of register bounds as two).
__device__ __forceinline__ int32_t med3_i32(int32_t x, int32_t lo, int32_t hi) {
  int32_t r;
  asm("v_med3_i32 %0, %1, %2, %3" : "=v"(r) : "v"(x), "v"(lo), "v"(hi));
  return r;
}

__device__ __forceinline__ v4i shift_u8(v4i x) {
  x.x ^= 0x80808080;
  x.y ^= 0x80808080;
  x.z ^= 0x80808080;
  x.w ^= 0x80808080;
  return x;
}

__device__ __forceinline__ v4i shfl_v4i(v4i x, int src) {
  v4i y;
  y.x = __shfl(x.x, src, 64);
  y.y = __shfl(x.y, src, 64);
  y.z = __shfl(x.z, src, 64);
  y.w = __shfl(x.w, src, 64);
  return y;
}

__device__ __forceinline__ int sdot16(v4i a, v4i b, int acc) {
  acc = __builtin_amdgcn_sdot4(a.x, b.x, acc, false);
  acc = __builtin_amdgcn_sdot4(a.y, b.y, acc, false);
  acc = __builtin_amdgcn_sdot4(a.z, b.z, acc, false);
  acc = __builtin_amdgcn_sdot4(a.w, b.w, acc, false);
  return acc;
}

}  // namespace u8
}  // namespace rp
