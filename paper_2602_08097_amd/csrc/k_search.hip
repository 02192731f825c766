// k_search.hip -- GreedySearch(s, q, k, L) (Algorithm 2), one wavefront per query.
//
// The search list is kept in LDS sorted by (S(q, .), id) with a visited flag
// per entry, in two ping-pong buffers.  One expansion:
//   1. p* = the first unvisited entry of the sorted list (= argmin over L \ V);
//   2. the lanes read N_out(p*) (64 ids per pass), compute S(q, j) exactly
//      (integers for uint8, canonical FP64 for float32), drop repeated ids and
//      ids already in the list (binary search on (S, id): S is a function of
//      the id), and, once the list is full, ids that fall behind its L-th
//      entry (the truncation would drop them at once);
//   3. the survivors are ranked and merged into the list, which is cut to L.
// Algorithm 2 also remembers visited vertices that the truncation evicted.
// Such a vertex can never re-enter the list: once the list holds L entries
// its L-th entry only moves closer, and the evicted vertex was behind it.
// The per-entry flags therefore carry the whole visited set that matters.
#include "dev_common.h"

namespace rp {

template <int DT>
__device__ __forceinline__ double query_sq(const GraphView& g, const void* q, int64_t j) {
  if (DT == RP_U8) {
    const uint8_t* X = (const uint8_t*)g.X;
    return (double)sq_u8((const uint8_t*)q, X + j * g.d, g.d);
  } else {
    const float* X = (const float*)g.X;
    return canon_sq_f32((const float*)q, X + j * g.d, g.d);
  }
}

template <int DT>
__global__ __launch_bounds__(64) void search_kernel(GraphView g, const void* __restrict__ Q,
                                                    int32_t k, int32_t L,
                                                    int32_t* __restrict__ out_ids,
                                                    double* __restrict__ out_dist,
                                                    int32_t* __restrict__ out_hops) {
  extern __shared__ double smem[];
  const int cap = L + kWave;
  double* bS0 = smem;
  double* bS1 = bS0 + cap;
  double* cS = bS1 + cap;        // 64 new candidates (compacted)
  double* sS = cS + kWave;       // 64 new candidates (sorted)
  int32_t* bI0 = (int32_t*)(sS + kWave);
  int32_t* bI1 = bI0 + cap;
  int32_t* cI = bI1 + cap;
  int32_t* cLb = cI + kWave;
  int32_t* sI = cLb + kWave;
  int32_t* sLb = sI + kWave;
  uint8_t* bV0 = (uint8_t*)(sLb + kWave);
  uint8_t* bV1 = bV0 + cap;

  const int lane = threadIdx.x;
  const int64_t qi = blockIdx.x;
  const size_t esz = DT == RP_U8 ? 1 : 4;
  const void* q = (const char*)Q + (size_t)qi * g.d * esz;

  double* bS = bS0;
  int32_t* bI = bI0;
  uint8_t* bV = bV0;
  double* nS = bS1;
  int32_t* nI = bI1;
  uint8_t* nV = bV1;

  if (lane == 0) {
    bS[0] = query_sq<DT>(g, q, g.start);
    bI[0] = g.start;
    bV[0] = 0;
  }
  int cnt = 1;
  int hops = 0;
  __syncthreads();

  // At most n distinct vertices can be expanded; the bound also guarantees
  // termination.
  while (hops < g.n) {
    // 1. first unvisited entry
    int pos = -1;
    for (int c = 0; c < cnt; c += kWave) {
      int t = c + lane;
      unsigned long long mask = __ballot(t < cnt && !bV[t]);
      if (mask) {
        pos = c + __ffsll((long long)mask) - 1;
        break;
      }
    }
    if (pos < 0) break;
    const int pstar = bI[pos];
    __syncthreads();
    if (lane == 0) bV[pos] = 1;
    ++hops;
    const int m = g.deg[pstar];
    const int32_t* row = g.nbr + (int64_t)pstar * g.r_max;

    for (int c0 = 0; c0 < m; c0 += kWave) {
      const int t = c0 + lane;
      int j = t < m ? row[t] : -1;
      // repeated ids within this pass: keep the first occurrence
      bool keep = j >= 0;
      for (int u = 0; u < kWave; ++u) {
        int other = __shfl(j, u, 64);
        if (u < lane && other == j) keep = false;
      }
      double s = 0.0;
      int lb = 0;
      if (keep) {
        s = query_sq<DT>(g, q, j);
        // lower bound: number of list entries strictly before (s, j)
        int lo = 0, hi = cnt;
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (before_f64(bS[mid], bI[mid], s, j)) lo = mid + 1;
          else hi = mid;
        }
        lb = lo;
        if (lb < cnt && bI[lb] == j) keep = false;            // already in the list
        if (keep && cnt == L && lb >= L) keep = false;        // behind the L-th entry
      }
      unsigned long long km = __ballot(keep);
      const int nc = __popcll(km);
      if (keep) {
        int slot = __popcll(km & ((1ull << lane) - 1ull));
        cS[slot] = s;
        cI[slot] = j;
        cLb[slot] = lb;
      }
      __syncthreads();
      if (nc == 0) continue;
      // rank the new candidates by (S, id)
      if (lane < nc) {
        double ms = cS[lane];
        int mi = cI[lane];
        int r = 0;
        for (int u = 0; u < nc; ++u) r += before_f64(cS[u], cI[u], ms, mi) ? 1 : 0;
        sS[r] = ms;
        sI[r] = mi;
        sLb[r] = cLb[lane];
      }
      __syncthreads();
      // merge into the other buffer, cut at L
      for (int i = lane; i < cnt; i += kWave) {
        double es = bS[i];
        int ei = bI[i];
        int lo = 0, hi = nc;  // new candidates strictly before entry i
        while (lo < hi) {
          int mid = (lo + hi) >> 1;
          if (before_f64(sS[mid], sI[mid], es, ei)) lo = mid + 1;
          else hi = mid;
        }
        int dst = i + lo;
        if (dst < L) {
          nS[dst] = es;
          nI[dst] = ei;
          nV[dst] = bV[i];
        }
      }
      if (lane < nc) {
        int dst = lane + sLb[lane];
        if (dst < L) {
          nS[dst] = sS[lane];
          nI[dst] = sI[lane];
          nV[dst] = 0;
        }
      }
      cnt = min(L, cnt + nc);
      __syncthreads();
      double* ts = bS; bS = nS; nS = ts;
      int32_t* ti = bI; bI = nI; nI = ti;
      uint8_t* tv = bV; bV = nV; nV = tv;
    }
    __syncthreads();
  }

  for (int t = lane; t < k; t += kWave) {
    out_ids[qi * k + t] = t < cnt ? bI[t] : -1;
    if (out_dist) out_dist[qi * k + t] = t < cnt ? bS[t] : -1.0;
  }
  if (lane == 0 && out_hops) out_hops[qi] = hops;
}

hipError_t launch_search(const GraphView& g, const void* Q, int64_t nq, int32_t k, int32_t L,
                         int32_t* out_ids, double* out_dist, int32_t* out_hops,
                         hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const size_t cap = (size_t)L + kWave;
  const size_t shmem = cap * 2 * sizeof(double) + 2 * kWave * sizeof(double) +
                       cap * 2 * sizeof(int32_t) + 4 * kWave * sizeof(int32_t) + cap * 2;
  dim3 grid((unsigned)nq), block(kWave);
  if (g.dtype == RP_U8)
    hipLaunchKernelGGL(search_kernel<RP_U8>, grid, block, shmem, s, g, Q, k, L, out_ids,
                       out_dist, out_hops);
  else
    hipLaunchKernelGGL(search_kernel<RP_F32>, grid, block, shmem, s, g, Q, k, L, out_ids,
                       out_dist, out_hops);
  return hipGetLastError();
}

}  // namespace rp
