// f32_common.h -- pieces shared by the two float32 prune kernels: rounding
// helpers, the canonical FP64 row distance, and the proven rounding band of
// the split-FP16 Gram.
#pragma once

#include <math.h>

#include "dev_common.h"

namespace rp {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

constexpr int kDC = 32;  // dimensions per accumulator chunk of the Gram

struct F32Args {
  double c1, c2, c3;  // rounding band of S~ (scaled units)
  int32_t nr;         // outputs per alpha (outputs are alpha-major)
  // measurement mode: only the listed vertices, S~ compared with canonical FP64
  const int32_t* nodes;
  int64_t n_nodes;
  GramErrorStats* stats;
};

// Next float toward -inf / +inf (finite inputs).
__device__ __forceinline__ float next_down(float f) {
  if (f == 0.f) return -1.401298464e-45f;
  const int b = __float_as_int(f);
  return __int_as_float(f > 0.f ? b - 1 : b + 1);
}

__device__ __forceinline__ float next_up(float f) {
  if (f == 0.f) return 1.401298464e-45f;
  const int b = __float_as_int(f);
  return __int_as_float(f > 0.f ? b + 1 : b - 1);
}

// FP32 value <= x (round down) and >= x (round up).
__device__ __forceinline__ float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = next_down(f);
  return f;
}

__device__ __forceinline__ float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = next_up(f);
  return f;
}

// Canonical FP64 squared distance of two float32 rows in global memory.
template <bool VEC>
__device__ __forceinline__ double canon_rows(const float* __restrict__ a,
                                             const float* __restrict__ b, int d) {
  double acc = 0.0;
  int k = 0;
  if (VEC) {
    for (; k + 4 <= d; k += 4) {
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
    const double t = (double)a[k] - (double)b[k];
    acc = __fma_rn(t, t, acc);
  }
  return acc;
}

__device__ __forceinline__ bool key_less(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah < bh || (ah == bh && al < bl);
}

__device__ __forceinline__ int ff1_u64(uint64_t v) {
  const uint64_t u = uniform_u64(v);
  int i;
  asm("s_ff1_i32_b64 %0, %1" : "=s"(i) : "s"(u));
  return i;  // -1 for an empty mask
}

// Power-of-two scale of the frame centred on p: |x_jk - x_pk| <= bound < 2^ex,
// e = 14 - ex, so every scaled difference is below 2^14 in magnitude.
__device__ __forceinline__ int frame_exponent(float bound) {
  int e = 0;
  if (bound > 0.f) {
    int ex;
    frexpf(bound, &ex);
    e = min(100, max(-100, 14 - ex));
  }
  return e;
}

// Bound of |S~ - S(i, j) 2^2e| for every rank i before j (S(p, i) <= S(p, j)),
// s = S(p, j) 2^2e, U = (x - x_p) 2^e exact:
//   e1 = 2^-22 + 2^-23  relative error of hi + lo against U (FP32 subtraction
//                       2^-24, rounding of lo 2^-22);
//   ea = 2^-14          absolute error of one element whose hi or lo is an
//                       FP16 subnormal, even if the matrix unit flushes it;
//   dropped lo lo'      <= 2^-22 (1 + 2^-9) s;
//   FP32 accumulation   gamma over the additions into one accumulator, with
//                       unit 2^-23 (covers truncating hardware), plus the
//                       gamma of the chunk sums (unit 2^-24);
//   |G~ - G| <= (2 e1 + e1^2 + lo lo' + acc) s + 2 ea sqrt(d) (1 + e1)(1 + acc) sqrt(s)
//               + d ea^2 (1 + acc);
//   S~ = (S(p,i) + S(p,j)) 2^2e - 2 G~ in FP32 adds 8 * 2^-24 s, and the
//   canonical FP64 values differ from the exact ones by at most 12 d 2^-53 s.
// Every coefficient is doubled; the FP64 threshold's own rounding is covered
// by the (1 -/+ 2^-50) factors.  csum: the accumulator is restarted every kDC
// dimensions and the chunk results are summed in FP32.
inline void f32_bound_constants(int d, bool csum, double* c1, double* c2, double* c3) {
  auto gam = [](double n, double u) { return n * u / (1.0 - n * u); };
  const double u24 = 0x1p-24;
  const double e1 = 0x1p-22 + 0x1p-23;
  const double ea = 0x1p-14;
  const double nadd = csum ? 3.0 * kDC + 1.0 : 3.0 * d + 1.0;
  const double g1 = gam(nadd, 0x1p-23);
  const double g2 = csum ? gam((double)((d + kDC - 1) / kDC), u24) : 0.0;
  const double acc = (g1 + g2 + g1 * g2) * (1.0 + 0x1p-9);
  const double lolo = 0x1p-22 * (1.0 + 0x1p-9);
  const double sd = sqrt((double)d);
  *c1 = 2.0 * (2.0 * (2.0 * e1 + e1 * e1 + lolo + acc) + 8.0 * u24 + 12.0 * d * 0x1p-53);
  *c2 = 2.0 * (2.0 * 2.0 * ea * sd * (1.0 + e1) * (1.0 + acc));
  *c3 = 2.0 * (2.0 * d * ea * ea * (1.0 + acc));
}

// Sorts the alphas of a sweep in descending order (num_a^2 den_b^2 against
// num_b^2 den_a^2) and moves every output with its alpha (outputs are
// alpha-major: o = alpha * nr + iR).
inline SweepArgs alphas_descending(const SweepArgs& a_in, int nr) {
  SweepArgs a = a_in;
  int order[kMaxAlphas];
  for (int i = 0; i < a_in.n_alpha; ++i) order[i] = i;
  for (int i = 1; i < a_in.n_alpha; ++i) {
    const int v = order[i];
    int j = i - 1;
    while (j >= 0 && (uint64_t)a_in.num2[v] * a_in.den2[order[j]] >
                         (uint64_t)a_in.num2[order[j]] * a_in.den2[v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  for (int k = 0; k < a_in.n_alpha; ++k) {
    a.num2[k] = a_in.num2[order[k]];
    a.den2[k] = a_in.den2[order[k]];
    a.ratio[k] = a_in.ratio[order[k]];
    for (int ir = 0; ir < nr; ++ir) {
      a.out[k * nr + ir] = a_in.out[order[k] * nr + ir];
      a.out[k * nr + ir].alpha_idx = k;
    }
  }
  return a;
}

}  // namespace rp
