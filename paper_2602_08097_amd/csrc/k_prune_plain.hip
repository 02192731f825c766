// k_prune_plain.hip -- plain baseline RP-Tuning kernel.
//
// One 64-lane workgroup per vertex p runs RobustPrune(p, N_out(p), alpha, R)
// (Algorithm 1) as written: the candidate list is read, p itself and repeated
// ids are dropped, D(p, .) is computed once per candidate, the candidates are
// ranked by (S(p, .), id) (the repeated argmin of Algorithm 1 over a set that
// only loses members visits them in this order), and the greedy loop walks
// that order (UnsortedRobustPrune, Section 3: the stored list order instead):
// each survivor p* is kept, the loop stops at the R-th keep, and
// the lanes evaluate alpha * D(p*, p') <= D(p, p') for every later survivor,
// computing D(p*, p') on demand from the rows in global memory.
//   uint8  : exact int32 distances, exact integer test.
//   float32: FP32 direct differences decided against a rounding bound, with a
//            canonical FP64 recheck of the pairs inside the bound.
#include "dev_common.h"

namespace rp {

template <int DT>
__global__ __launch_bounds__(64) void prune_plain_kernel(GraphView g, uint32_t num2,
                                                         uint32_t den2, int32_t R,
                                                         int32_t* __restrict__ out_nbr,
                                                         int32_t* __restrict__ out_deg,
                                                         double rel, DevCounters* ctr,
                                                         bool unsorted) {
  __shared__ int32_t ids[kMaxRmax];
  __shared__ double sp[kMaxRmax];      // S(p, candidate)
  __shared__ int16_t order[kMaxRmax];  // rank -> candidate slot
  __shared__ uint8_t valid[kMaxRmax];
  __shared__ uint8_t alive[kMaxRmax];  // by rank
  __shared__ int32_t s_nvalid;

  const int lane = threadIdx.x;
  const int64_t p = blockIdx.x;
  const int d = g.d;
  const int m = g.deg[p];
  const int32_t* row = g.nbr + p * g.r_max;

  for (int t = lane; t < m; t += kWave) ids[t] = row[t];
  if (lane == 0) s_nvalid = 0;
  __syncthreads();

  // V <- N_out(p) \ {p}, each id once.
  for (int t = lane; t < m; t += kWave) {
    int id = ids[t];
    bool ok = id != (int)p;
    for (int u = 0; u < t && ok; ++u) ok = ids[u] != id;
    valid[t] = ok;
    if (ok) {
      if (DT == RP_U8) {
        const uint8_t* X = (const uint8_t*)g.X;
        sp[t] = (double)sq_u8(X + p * d, X + (int64_t)id * d, d);
      } else {
        const float* X = (const float*)g.X;
        sp[t] = canon_sq_f32(X + p * d, X + (int64_t)id * d, d);
      }
      atomicAdd(&s_nvalid, 1);
    }
  }
  __syncthreads();

  // Rank by (S(p, .), id); UnsortedRobustPrune keeps the list order.
  for (int t = lane; t < m; t += kWave) {
    if (!valid[t]) continue;
    int r = 0;
    for (int u = 0; u < m; ++u)
      if (valid[u] && (unsorted ? u < t : before_f64(sp[u], ids[u], sp[t], ids[t]))) ++r;
    order[r] = (int16_t)t;
  }
  const int nv = s_nvalid;
  for (int r = lane; r < nv; r += kWave) alive[r] = 1;
  __syncthreads();

  unsigned long long rechecks = 0;
  int kept = 0;
  for (int r = 0; r < nv; ++r) {
    if (!alive[r]) continue;  // uniform: read after the barrier
    const int i = order[r];
    const int pid = ids[i];
    if (lane == 0) out_nbr[p * R + kept] = pid;
    ++kept;
    if (kept == R) break;
    for (int u = r + 1 + lane; u < nv; u += kWave) {
      if (!alive[u]) continue;
      const int j = order[u];
      const int jid = ids[j];
      bool prune;
      if (DT == RP_U8) {
        const uint8_t* X = (const uint8_t*)g.X;
        uint32_t s = sq_u8(X + (int64_t)pid * d, X + (int64_t)jid * d, d);
        prune = alpha_test_int(num2, den2, s, (uint32_t)sp[j]);
      } else {
        const float* X = (const float*)g.X;
        const float* a = X + (int64_t)pid * d;
        const float* b = X + (int64_t)jid * d;
        int dec = decide_approx(num2, den2, (double)sq_f32(a, b, d), sp[j], rel);
        if (dec < 0) {
          ++rechecks;
          prune = alpha_test_f64(num2, den2, canon_sq_f32(a, b, d), sp[j]);
        } else {
          prune = dec == 1;
        }
      }
      if (prune) alive[u] = 0;
    }
    __syncthreads();
  }
  for (int t = kept + lane; t < R; t += kWave) out_nbr[p * R + t] = -1;
  if (lane == 0) out_deg[p] = kept;

  if (DT == RP_F32) {
    rechecks = wave_sum_u64(rechecks);
    if (lane == 0 && rechecks) atomicAdd(&ctr->rechecks, rechecks);
  }
}

hipError_t launch_prune_plain(const GraphView& g, uint32_t num2, uint32_t den2, int32_t R,
                              int32_t* out_nbr, int32_t* out_deg, DevCounters* ctr,
                              hipStream_t s, bool unsorted) {
  const double rel = f32_rel_bound(g.d);
  dim3 grid((unsigned)g.n), block(kWave);
  if (g.dtype == RP_U8)
    hipLaunchKernelGGL(prune_plain_kernel<RP_U8>, grid, block, 0, s, g, num2, den2, R, out_nbr,
                       out_deg, rel, ctr, unsorted);
  else
    hipLaunchKernelGGL(prune_plain_kernel<RP_F32>, grid, block, 0, s, g, num2, den2, R, out_nbr,
                       out_deg, rel, ctr, unsorted);
  return hipGetLastError();
}

}  // namespace rp
