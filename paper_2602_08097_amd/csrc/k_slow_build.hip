// k_slow_build.hip -- the "slow preprocessing" construction of Section 2.1:
// RobustPrune(p, P \ {p}, alpha, R) (Algorithm 1) for every point p.  With
// R >= n - 1 the result is alpha-reachable (Lemma 2.2); it is the rebuild
// that RP-Tuning (Section 3) is compared with.
//
// One 256-thread workgroup per vertex (the grid strides over the vertices):
//  - S(p, j) of every other point j (exact integers for uint8 points, the
//    canonical FP64 value for float32 points) into the workgroup's slice of
//    a workspace, with the list of candidates still in V;
//  - each round takes p* = the (S(p, .), id)-smallest candidate left (a
//    workgroup reduction), keeps it, stops at R, and rebuilds the candidate
//    list from the points p* does not prune (alpha D(p*, p') <= D(p, p') on
//    squares, evaluated as in Algorithm 1), so later rounds scan only what is
//    left.  The list order is arbitrary; the argmin makes the result unique.
#include "dev_common.h"

namespace rp {

namespace {

constexpr int kSlowThreads = 256;

struct SlowArgs {
  const void* X;
  int64_t n;
  int32_t d;
  uint32_t num2, den2;
  int32_t R;
  int32_t* out_nbr;  // n x R
  int32_t* out_deg;  // n
  double* S;         // gridDim.x x n
  int32_t* ids;      // gridDim.x x 2n
};

template <int DT>
__device__ __forceinline__ double dist(const void* X, int d, int64_t a, int64_t b) {
  if (DT == RP_U8) {
    const uint8_t* x = (const uint8_t*)X;
    return (double)sq_u8(x + a * d, x + b * d, d);
  }
  const float* x = (const float*)X;
  return canon_sq_f32(x + a * d, x + b * d, d);
}

template <int DT>
__device__ __forceinline__ bool prunes(uint32_t num2, uint32_t den2, double s_star, double s_p) {
  if (DT == RP_U8) return alpha_test_int(num2, den2, (uint32_t)s_star, (uint32_t)s_p);
  return alpha_test_f64(num2, den2, s_star, s_p);
}

template <int DT>
__global__ __launch_bounds__(kSlowThreads) void slow_build_kernel(SlowArgs A) {
  __shared__ double red_s[kSlowThreads / 64];
  __shared__ int32_t red_id[kSlowThreads / 64];
  __shared__ int32_t s_cnt, s_best;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wv = tid >> 6;
  const int64_t n = A.n;
  double* S = A.S + (int64_t)blockIdx.x * n;
  int32_t* cur = A.ids + (int64_t)blockIdx.x * 2 * n;
  int32_t* nxt = cur + n;
  for (int64_t p = blockIdx.x; p < n; p += gridDim.x) {
    // V <- P \ {p}, with S(p, .)
    for (int64_t j = tid; j < n; j += kSlowThreads) {
      if (j == p) continue;
      S[j] = dist<DT>(A.X, A.d, p, j);
      cur[j < p ? j : j - 1] = (int32_t)j;
    }
    int cnt = (int)(n - 1);
    int kept = 0;
    __syncthreads();
    while (cnt > 0) {
      // p* <- argmin over V of (S(p, .), id)
      double bs = 0.0;
      int bi = -1;
      for (int t = tid; t < cnt; t += kSlowThreads) {
        const int j = cur[t];
        const double s = S[j];
        if (bi < 0 || before_f64(s, j, bs, bi)) {
          bs = s;
          bi = j;
        }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double os = __shfl_xor(bs, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (oi >= 0 && (bi < 0 || before_f64(os, oi, bs, bi))) {
          bs = os;
          bi = oi;
        }
      }
      if (lane == 0) {
        red_s[wv] = bs;
        red_id[wv] = bi;
      }
      __syncthreads();
      if (tid == 0) {
        double s0 = red_s[0];
        int i0 = red_id[0];
        for (int w = 1; w < kSlowThreads / 64; ++w)
          if (red_id[w] >= 0 && (i0 < 0 || before_f64(red_s[w], red_id[w], s0, i0))) {
            s0 = red_s[w];
            i0 = red_id[w];
          }
        s_best = i0;
        s_cnt = 0;
        A.out_nbr[p * A.R + kept] = i0;
      }
      __syncthreads();
      const int pstar = s_best;
      ++kept;
      if (kept == A.R) break;
      // V <- the candidates p* does not prune (p* itself leaves V explicitly)
      for (int t = tid; t < cnt; t += kSlowThreads) {
        const int j = cur[t];
        if (j == pstar) continue;
        if (!prunes<DT>(A.num2, A.den2, dist<DT>(A.X, A.d, pstar, j), S[j]))
          nxt[atomicAdd(&s_cnt, 1)] = j;
      }
      __syncthreads();
      cnt = s_cnt;
      int32_t* t = cur;
      cur = nxt;
      nxt = t;
      __syncthreads();
    }
    for (int t = kept + tid; t < A.R; t += kSlowThreads) A.out_nbr[p * A.R + t] = -1;
    if (tid == 0) A.out_deg[p] = kept;
    __syncthreads();
  }
}

}  // namespace

// Workgroups for n points: at most 2,048, and a workspace of at most 1 GiB
// (16 bytes per point and workgroup).
int slow_build_groups(int64_t n) {
  int64_t g = min((int64_t)2048, n);
  const int64_t cap = ((int64_t)1 << 30) / (16 * n);
  return (int)max((int64_t)1, min(g, cap));
}

size_t slow_build_workspace_bytes(int64_t n, int groups) {
  return (size_t)groups * (size_t)n * (8 + 8);
}

hipError_t launch_slow_build(const void* X, int32_t dtype, int64_t n, int32_t d, uint32_t num2,
                             uint32_t den2, int32_t R, int32_t* out_nbr, int32_t* out_deg,
                             void* workspace, int groups, hipStream_t s) {
  SlowArgs A;
  A.X = X;
  A.n = n;
  A.d = d;
  A.num2 = num2;
  A.den2 = den2;
  A.R = R;
  A.out_nbr = out_nbr;
  A.out_deg = out_deg;
  A.S = (double*)workspace;
  A.ids = (int32_t*)((char*)workspace + (size_t)groups * n * 8);
  if (dtype == RP_U8)
    hipLaunchKernelGGL(slow_build_kernel<RP_U8>, dim3(groups), dim3(kSlowThreads), 0, s, A);
  else
    hipLaunchKernelGGL(slow_build_kernel<RP_F32>, dim3(groups), dim3(kSlowThreads), 0, s, A);
  return hipGetLastError();
}

}  // namespace rp
