// k_search.hip -- GreedySearch(s, q, k, L) (Algorithm 2), one wavefront per query.
//
// The search list lives in LDS, sorted by the key (S(q, v), v) with a visited
// flag per entry, in two ping-pong buffers.  One expansion:
//   1. p* = the first unvisited entry of the sorted list (= argmin over L \ V);
//   2. the lanes read N_out(p*) (64 ids per pass) and compute S(q, j) exactly:
//      uint8 points as |q|^2 + |x_j|^2 - 2 <q, x_j> with 4-way byte dot
//      products on 16-byte row loads (|x_j|^2 precomputed per point);
//      float32 points as the canonical FP64 value;
//   3. the 64 keys are sorted across the wavefront (DPP bitonic network), so
//      repeated ids become adjacent; ids already in the list are found by a
//      lower-bound search of their key (S is a function of the id), and once
//      the list is full, ids behind its L-th entry are dropped (the truncation
//      would drop them at once);
//   4. the survivors, still in key order after compaction, are merged into
//      the list, which is cut at L.
// Algorithm 2 also remembers visited vertices that the truncation evicted.
// Such a vertex can never re-enter the list: once the list holds L entries
// its L-th entry only moves closer, and the evicted vertex was behind it.
// The per-entry flags therefore carry the whole visited set that matters.
//
// Keys are (hi, lo) pairs compared lexicographically: hi = S (uint8 points) or
// the bit pattern of the non-negative FP64 S (float32 points, which orders as
// an unsigned integer); lo = the vertex id.
#include "dev_common.h"

namespace rp {

namespace {

// Byte offset of the query row in the search kernel's LDS (16-byte aligned).
__host__ __device__ inline size_t search_query_offset(int cap) {
  const size_t off = (size_t)cap * 2 * 8 + kWave * 8 + (size_t)cap * 2 * 4 + kWave * 4 +
                     kWave * 4 + (size_t)cap * 2;
  return (off + 15) & ~(size_t)15;
}

__device__ __forceinline__ bool key_less(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah < bh || (ah == bh && al < bl);
}

// S(q, x_j) for uint8 points: q in LDS (broadcast reads), 16-byte row loads.
__device__ __forceinline__ uint32_t sq_u8_q(const uint8_t* __restrict__ qs,
                                            const uint8_t* __restrict__ x, int d, uint32_t qq,
                                            uint32_t xx) {
  uint32_t dot = 0;
  int k = 0;
  if (((d & 15) | ((uintptr_t)x & 15)) == 0)  // 16-byte aligned rows
#pragma unroll 8
  for (; k + 16 <= d; k += 16) {
    const uint4 a = *(const uint4*)(qs + k);
    const uint4 b = *(const uint4*)(x + k);
    dot = __builtin_amdgcn_udot4(a.x, b.x, dot, false);
    dot = __builtin_amdgcn_udot4(a.y, b.y, dot, false);
    dot = __builtin_amdgcn_udot4(a.z, b.z, dot, false);
    dot = __builtin_amdgcn_udot4(a.w, b.w, dot, false);
  }
  for (; k < d; ++k) dot += (uint32_t)qs[k] * x[k];
  return qq + xx - 2u * dot;
}

// Queries come either as one contiguous nq x d array with contiguous outputs,
// or (jobs != null) as one descriptor per query with its own row and outputs.
template <int DT>
__global__ __launch_bounds__(64) void search_kernel(GraphView g, const void* __restrict__ Q,
                                                    const SearchJob* __restrict__ jobs,
                                                    int32_t k, int32_t L,
                                                    int32_t* __restrict__ out_ids,
                                                    double* __restrict__ out_dist,
                                                    int32_t* __restrict__ out_hops) {
  extern __shared__ __align__(16) uint64_t smem[];
  const int cap = L + kWave;
  uint8_t* base = (uint8_t*)smem;
  uint64_t* bH0 = (uint64_t*)base;
  uint64_t* bH1 = bH0 + cap;
  uint64_t* nH = bH1 + cap;                 // new candidates, compacted (sorted)
  uint32_t* bL0 = (uint32_t*)(nH + kWave);
  uint32_t* bL1 = bL0 + cap;
  uint32_t* nL = bL1 + cap;
  int32_t* nLb = (int32_t*)(nL + kWave);    // insertion position in the old list
  uint8_t* bV0 = (uint8_t*)(nLb + kWave);
  uint8_t* bV1 = bV0 + cap;
  uint8_t* qs = base + search_query_offset(cap);  // query row, 16-byte aligned

  const int lane = threadIdx.x;
  const int64_t qi = blockIdx.x;
  const int d = g.d;
  const size_t esz = DT == RP_U8 ? 1 : 4;
  const uint8_t* qg = (const uint8_t*)Q + (size_t)qi * d * esz;
  int32_t* o_ids = out_ids + qi * k;
  double* o_dist = out_dist ? out_dist + qi * k : nullptr;
  int32_t* o_hops = out_hops ? out_hops + qi : nullptr;
  if (jobs) {
    const SearchJob jb = jobs[qi];
    qg = (const uint8_t*)jb.q;
    o_ids = jb.ids;
    o_dist = jb.dist;
    o_hops = jb.hops;
  }
  for (int t = lane; t < (int)(d * esz); t += kWave) qs[t] = qg[t];
  __syncthreads();
  uint32_t qq = 0;
  if (DT == RP_U8) {
    for (int t = 0; t < d; ++t) qq += (uint32_t)qs[t] * qs[t];
  }

  auto dist = [&](int64_t j) -> uint64_t {
    if (DT == RP_U8) {
      return (uint64_t)sq_u8_q(qs, (const uint8_t*)g.X + j * d, d, qq, g.norms[j]);
    } else {
      const double s = canon_sq_f32((const float*)qs, (const float*)g.X + j * d, d);
      return (uint64_t)__double_as_longlong(s);
    }
  };

  uint64_t* bH = bH0;
  uint32_t* bL = bL0;
  uint8_t* bV = bV0;
  uint64_t* oH = bH1;
  uint32_t* oL = bL1;
  uint8_t* oV = bV1;
  if (lane == 0) {
    bH[0] = dist(g.start);
    bL[0] = (uint32_t)g.start;
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
      const int t = c + lane;
      const uint64_t mask = __ballot(t < cnt && !bV[t]);
      if (mask) {
        pos = c + __ffsll((long long)mask) - 1;
        break;
      }
    }
    if (pos < 0) break;
    const int pstar = (int)bL[pos];
    __syncthreads();
    if (lane == 0) bV[pos] = 1;
    ++hops;
    const int m = g.deg[pstar];
    const int32_t* row = g.nbr + (int64_t)pstar * g.r_max;

    for (int c0 = 0; c0 < m; c0 += kWave) {
      const int t = c0 + lane;
      const int j = t < m ? row[t] : -1;
      // 2. distances
      uint64_t kh = ~0ull;
      uint32_t kl = ~0u;
      if (j >= 0) {
        kh = dist(j);
        kl = (uint32_t)j;
      }
      // 3. sort the keys; repeats become adjacent
      wave_sort2(kh, kl, lane);
      const uint64_t ph = shfl_u64(kh, lane > 0 ? lane - 1 : 0);
      const uint32_t pl = (uint32_t)__shfl((int)kl, lane > 0 ? lane - 1 : 0, 64);
      bool keep = kl != ~0u && !(lane > 0 && ph == kh && pl == kl);
      int lb = 0;
      if (keep) {
        int lo = 0, hi = cnt;  // entries strictly before (kh, kl)
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (key_less(bH[mid], bL[mid], kh, kl)) lo = mid + 1;
          else hi = mid;
        }
        lb = lo;
        if (lb < cnt && bL[lb] == kl) keep = false;          // already in the list
        if (keep && cnt == L && lb >= L) keep = false;        // behind the L-th entry
      }
      const uint64_t km = __ballot(keep);
      const int nc = __popcll(km);
      if (nc == 0) continue;  // uniform
      if (keep) {
        const int slot = __popcll(km & ((1ull << lane) - 1ull));
        nH[slot] = kh;
        nL[slot] = kl;
        nLb[slot] = lb;
      }
      __syncthreads();
      // 4. merge into the other buffer, cut at L
      for (int i = lane; i < cnt; i += kWave) {
        int lo = 0, hi = nc;  // new candidates whose insertion position is <= i
        while (lo < hi) {
          const int mid = (lo + hi) >> 1;
          if (nLb[mid] <= i) lo = mid + 1;
          else hi = mid;
        }
        const int dst = i + lo;
        if (dst < L) {
          oH[dst] = bH[i];
          oL[dst] = bL[i];
          oV[dst] = bV[i];
        }
      }
      if (lane < nc) {
        const int dst = lane + nLb[lane];
        if (dst < L) {
          oH[dst] = nH[lane];
          oL[dst] = nL[lane];
          oV[dst] = 0;
        }
      }
      cnt = min(L, cnt + nc);
      __syncthreads();
      uint64_t* th = bH; bH = oH; oH = th;
      uint32_t* tl = bL; bL = oL; oL = tl;
      uint8_t* tv = bV; bV = oV; oV = tv;
    }
    __syncthreads();
  }

  for (int t = lane; t < k; t += kWave) {
    o_ids[t] = t < cnt ? (int32_t)bL[t] : -1;
    if (o_dist) {
      double dv = -1.0;
      if (t < cnt) dv = DT == RP_U8 ? (double)bH[t] : __longlong_as_double((long long)bH[t]);
      o_dist[t] = dv;
    }
  }
  if (lane == 0 && o_hops) *o_hops = hops;
}

}  // namespace

static hipError_t launch_search_any(const GraphView& g, const void* Q, const SearchJob* jobs,
                                    int64_t nq, int32_t k, int32_t L, int32_t* out_ids,
                                    double* out_dist, int32_t* out_hops, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  const size_t cap = (size_t)L + kWave;
  const size_t esz = g.dtype == RP_U8 ? 1 : 4;
  // keys (hi, lo), insertion positions, visited flags, then the query row
  const size_t shmem = search_query_offset((int)cap) + (size_t)g.d * esz;
  dim3 grid((unsigned)nq), block(kWave);
  if (g.dtype == RP_U8)
    hipLaunchKernelGGL(search_kernel<RP_U8>, grid, block, shmem, s, g, Q, jobs, k, L, out_ids,
                       out_dist, out_hops);
  else
    hipLaunchKernelGGL(search_kernel<RP_F32>, grid, block, shmem, s, g, Q, jobs, k, L, out_ids,
                       out_dist, out_hops);
  return hipGetLastError();
}

hipError_t launch_search(const GraphView& g, const void* Q, int64_t nq, int32_t k, int32_t L,
                         int32_t* out_ids, double* out_dist, int32_t* out_hops,
                         hipStream_t s) {
  return launch_search_any(g, Q, nullptr, nq, k, L, out_ids, out_dist, out_hops, s);
}

hipError_t launch_search_jobs(const GraphView& g, const SearchJob* jobs, int64_t n, int32_t k,
                              int32_t L, hipStream_t s) {
  return launch_search_any(g, nullptr, jobs, n, k, L, nullptr, nullptr, nullptr, s);
}

}  // namespace rp
