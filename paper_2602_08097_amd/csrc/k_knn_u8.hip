// k_knn_u8.hip -- exact K nearest neighbours of uint8 points by (S, id), on
// int8 MFMA with a per-query top-K kept in LDS.
//
// The base graphs of the experiments are RobustPrune (Algorithm 1) over each
// point's K nearest points: the stand-in used here for the paper's Vamana
// base index (Section 4.1).  This kernel builds those lists.
//
// One wavefront owns 32 queries (one MFMA row block) and streams candidates
// in tiles of 32 (one column block):
//  - rows go straight from global memory into the operand registers of
//    v_mfma_i32_32x32x32_i8, shifted to int8 u = x - 128, so the inner
//    products are exact; |u_c|^2 comes from 4-way byte dot products on the
//    same registers;
//  - per (query q, candidate c) the key is (S'', c) with
//    S'' = |u_c|^2 - 2 <u_q, u_c> + 16384 d = S(q, c) - |u_q|^2 + 16384 d, a
//    shift of S(q, c) that is constant along a query's row, non-negative and
//    below 2^25 for d <= 256, so ordering keys orders (S, id);
//  - a candidate whose S'' is at most the query's current K-th S'' goes to an
//    insertion buffer in LDS; full buffers are merged into the sorted top-128
//    by bitonic merges across the wavefront (the 128 smallest of a sorted T
//    and new keys b are T[0..63] plus the 64 smallest of T[64..127] and b).
// The query itself is never a candidate of its own list.  Large candidate
// sets can be split into slices (blockIdx.y) whose partial top-128 lists go
// to a workspace and are merged by a second kernel.
#include "u8_common.h"

namespace rp {

using namespace u8;

namespace {

constexpr int kQB = 32;    // queries per wavefront
constexpr int kCB = 32;    // candidates per tile
constexpr int kTop = 128;  // keys kept per query (K <= kTop)
constexpr int kBuf = 64;   // insertion buffer per query
constexpr size_t kKnnLds =
    (size_t)kQB * kTop * 8 + (size_t)kQB * kBuf * 8 + kQB * 4 + kQB * 4 + kQB * 4;

struct KnnArgs {
  const uint8_t* X;
  int64_t n;
  int32_t d;
  const int32_t* qids;  // nq query rows (null: rows 0 .. nq - 1)
  int64_t nq;
  const int32_t* cids;  // nc candidate rows (null: rows 0 .. nc - 1)
  int64_t nc;
  int64_t per_slice;    // candidates per slice (a multiple of kCB)
  int32_t K;
  int32_t* out;         // nq x K ids (slices == 1)
  uint64_t* part;       // slices x nq x kTop keys (slices > 1)
};

// Ascending order of a bitonic sequence of 64 keys, one per lane.
__device__ __forceinline__ uint64_t bitonic_merge64(uint64_t k, int lane) {
  k = bitonic_step<64, 32>(k, lane);
  k = bitonic_step<64, 16>(k, lane);
  k = bitonic_step<64, 8>(k, lane);
  k = bitonic_step<64, 4>(k, lane);
  k = bitonic_step<64, 2>(k, lane);
  k = bitonic_step<64, 1>(k, lane);
  return k;
}

// t0 (ranks 0..63) and t1 (ranks 64..127): a sorted list of 128 keys; b: 64
// keys in ascending order.  Afterwards t0, t1 hold the 128 smallest of both,
// in ascending order.  Every key of t0 is at most every key of t1, so the
// result is t0 with the 64 smallest of t1 and b.
__device__ __forceinline__ void merge128(uint64_t& t0, uint64_t& t1, uint64_t b, int lane) {
  const uint64_t br = shfl_u64(b, 63 - lane);
  uint64_t x = t1 < br ? t1 : br;  // bitonic: the 64 smallest of t1 and b
  x = bitonic_merge64(x, lane);
  const uint64_t xr = shfl_u64(x, 63 - lane);
  const uint64_t lo = t0 < xr ? t0 : xr;
  const uint64_t hi = t0 < xr ? xr : t0;
  t0 = bitonic_merge64(lo, lane);
  t1 = bitonic_merge64(hi, lane);
}

// Merges query row r's insertion buffer into its top-128 (whole wavefront).
__device__ __forceinline__ void flush_row(uint64_t* top, uint64_t* buf, int32_t* cnt,
                                          uint32_t* tau, int r, int K, int lane) {
  const int c = cnt[r];
  uint64_t b = lane < c ? buf[r * kBuf + lane] : ~0ull;
  b = wave_sort(b, lane);
  uint64_t t0 = top[r * kTop + lane];
  uint64_t t1 = top[r * kTop + 64 + lane];
  merge128(t0, t1, b, lane);
  top[r * kTop + lane] = t0;
  top[r * kTop + 64 + lane] = t1;
  // the K-th key's S'' bounds what can still enter (ties by id pass and are
  // settled by the next merge)
  const uint64_t kth = shfl_u64(K <= 64 ? t0 : t1, (K - 1) & 63);
  if (lane == 0) {
    cnt[r] = 0;
    tau[r] = (uint32_t)(kth >> 32);
  }
}

template <int NK>
__device__ __forceinline__ void load_rows(v4i (&f)[NK], const uint8_t* row, int d, int half) {
#pragma unroll
  for (int k = 0; k < NK; ++k) f[k] = *(const v4i*)(row + min(32 * k + 16 * half, d - 16));
}

template <int NK>
__device__ __forceinline__ void shift_zero(v4i (&f)[NK], int d, int half) {
  const v4i zero = {0, 0, 0, 0};
#pragma unroll
  for (int k = 0; k < NK; ++k) f[k] = 32 * k + 16 * half < d ? shift_u8(f[k]) : zero;
}

template <int NK>
__global__ __launch_bounds__(64) void knn_u8_kernel(KnnArgs A) {
  extern __shared__ __align__(16) uint8_t lds[];
  uint64_t* top = (uint64_t*)lds;                 // [kQB][kTop], ascending
  uint64_t* buf = top + kQB * kTop;               // [kQB][kBuf]
  int32_t* cnt = (int32_t*)(buf + kQB * kBuf);    // [kQB]
  uint32_t* tau = (uint32_t*)(cnt + kQB);         // [kQB]: S'' of the K-th key
  int32_t* qs = (int32_t*)(tau + kQB);            // [kQB]: query ids (-1: none)
  const int lane = threadIdx.x;
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int d = A.d;
  const int64_t q0 = (int64_t)blockIdx.x * kQB;
  const int slice = blockIdx.y;
  const int64_t c_begin = (int64_t)slice * A.per_slice;
  const int64_t c_end = min(A.nc, c_begin + A.per_slice);

  // queries: row l32 of the block in this lane's A-operand slices
  // (ids outside [0, n) are ignored: such a query gets a row of -1, such a
  // candidate is never listed)
  int qid = -1;
  if (q0 + l32 < A.nq) qid = A.qids ? A.qids[q0 + l32] : (int)(q0 + l32);
  if (qid >= A.n) qid = -1;
  v4i qf[NK];
  load_rows<NK>(qf, A.X + (int64_t)(qid >= 0 ? qid : 0) * d, d, half);
  shift_zero<NK>(qf, d, half);
  // the query id of each accumulator row of this lane: rows 8 (v / 4) + 4 half + v % 4
  int qr[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) qr[v] = __shfl(qid, 8 * (v >> 2) + 4 * half + (v & 3), 64);
  for (int i = lane; i < kQB * kTop; i += 64) top[i] = ~0ull;
  if (lane < kQB) {
    cnt[lane] = 0;
    tau[lane] = 0xFFFFFFFFu;
    qs[lane] = qid < 0 ? -1 : qid;
  }
  wave_sync();
  uint32_t tr[16];
#pragma unroll
  for (int v = 0; v < 16; ++v) tr[v] = 0xFFFFFFFFu;
  const int32_t bias = 16384 * d;

  // the first tile's rows, then each tile prefetches the next
  v4i cf[NK];
  int cid = -1;
  {
    const int64_t ci = c_begin + l32;
    if (ci < c_end) cid = A.cids ? A.cids[ci] : (int)ci;
    if (cid >= A.n) cid = -1;
    load_rows<NK>(cf, A.X + (int64_t)(cid >= 0 ? cid : 0) * d, d, half);
  }
  for (int64_t c0 = c_begin; c0 < c_end; c0 += kCB) {
    v4i cur[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) cur[k] = cf[k];
    const int ccur = cid;
    {
      const int64_t ci = c0 + kCB + l32;
      cid = -1;
      if (ci < c_end) cid = A.cids ? A.cids[ci] : (int)ci;
      if (cid >= A.n) cid = -1;
      if (c0 + kCB < c_end) load_rows<NK>(cf, A.X + (int64_t)(cid >= 0 ? cid : 0) * d, d, half);
    }
    shift_zero<NK>(cur, d, half);
    int nc = 0;
#pragma unroll
    for (int k = 0; k < NK; ++k) nc = sdot16(cur[k], cur[k], nc);
    nc += __shfl_xor(nc, 32, 64);
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(qf[k], cur[k], acc, 0, 0, 0);
    const int32_t ncb = nc + bias;
    uint32_t s[16];
    bool anyp = false;
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      s[v] = (uint32_t)(ncb - 2 * acc[v]);
      anyp = anyp || (s[v] <= tr[v]);
    }
    anyp = anyp && ccur >= 0;
    if (__ballot(anyp) == 0) continue;  // uniform
    bool over = false;
    if (anyp) {
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        if (s[v] <= tr[v] && ccur != qr[v]) {
          const int r = 8 * (v >> 2) + 4 * half + (v & 3);
          const int pos = atomicAdd(&cnt[r], 1);
          buf[r * kBuf + pos] = ((uint64_t)s[v] << 32) | (uint32_t)ccur;
          over = over || pos >= kBuf - kCB;
        }
      }
    }
    // a row that could overflow on the next tile is merged now (with the
    // other rows that hold new keys)
    if (__ballot(over) != 0) {
      wave_sync();
      for (int r = 0; r < kQB; ++r) {
        if (cnt[r] > 0) flush_row(top, buf, cnt, tau, r, A.K, lane);  // uniform
        wave_sync();
      }
#pragma unroll
      for (int v = 0; v < 16; ++v) tr[v] = tau[8 * (v >> 2) + 4 * half + (v & 3)];
    }
  }
  wave_sync();
  for (int r = 0; r < kQB; ++r) {
    if (cnt[r] > 0) flush_row(top, buf, cnt, tau, r, A.K, lane);
    wave_sync();
  }
  // outputs: the ids of the K smallest keys (-1 where fewer candidates), or
  // the slice's 128 keys for the merge kernel
  for (int r = 0; r < kQB; ++r) {
    const int64_t q = q0 + r;
    if (q >= A.nq) break;
    const bool none = qs[r] < 0;
    const uint64_t t0 = none ? ~0ull : top[r * kTop + lane];
    const uint64_t t1 = none ? ~0ull : top[r * kTop + 64 + lane];
    if (A.part) {
      uint64_t* o = A.part + ((int64_t)slice * A.nq + q) * kTop;
      o[lane] = t0;
      o[64 + lane] = t1;
    } else {
      int32_t* o = A.out + q * A.K;
      if (lane < A.K) o[lane] = t0 == ~0ull ? -1 : (int32_t)(uint32_t)t0;
      if (64 + lane < A.K) o[64 + lane] = t1 == ~0ull ? -1 : (int32_t)(uint32_t)t1;
    }
  }
}

// One wavefront per query: merges the slices' sorted 128-key lists.
__global__ __launch_bounds__(64) void knn_merge_kernel(const uint64_t* __restrict__ part,
                                                       int64_t nq, int slices, int K,
                                                       int32_t* __restrict__ out) {
  const int lane = threadIdx.x;
  const int64_t q = blockIdx.x;
  uint64_t t0 = part[q * kTop + lane];
  uint64_t t1 = part[q * kTop + 64 + lane];
  for (int s = 1; s < slices; ++s) {
    const uint64_t* o = part + ((int64_t)s * nq + q) * kTop;
    merge128(t0, t1, o[lane], lane);
    merge128(t0, t1, o[64 + lane], lane);
  }
  int32_t* dst = out + q * K;
  if (lane < K) dst[lane] = t0 == ~0ull ? -1 : (int32_t)(uint32_t)t0;
  if (64 + lane < K) dst[64 + lane] = t1 == ~0ull ? -1 : (int32_t)(uint32_t)t1;
}

template <int NK>
hipError_t launch_nk(const KnnArgs& A, int slices, hipStream_t s) {
  const dim3 grid((unsigned)((A.nq + kQB - 1) / kQB), (unsigned)slices);
  hipLaunchKernelGGL(knn_u8_kernel<NK>, grid, dim3(64), kKnnLds, s, A);
  return hipGetLastError();
}

}  // namespace

bool knn_u8_supported(int d) { return d >= 16 && d <= 256 && d % 16 == 0; }

// Slices of the candidate set: enough wavefronts for the chip (about 2,048),
// at least 4,096 candidates per slice, at most 64 slices.
int knn_u8_slices(int64_t nq, int64_t nc) {
  const int64_t blocks = (nq + kQB - 1) / kQB;
  int64_t s = (2048 + blocks - 1) / blocks;
  s = min(s, max((int64_t)1, nc / 4096));
  return (int)max((int64_t)1, min(s, (int64_t)64));
}

size_t knn_u8_workspace_bytes(int64_t nq, int slices) {
  return slices > 1 ? (size_t)slices * (size_t)nq * kTop * 8 : 0;
}

hipError_t launch_knn_u8(const uint8_t* X, int64_t n, int32_t d, const int32_t* qids, int64_t nq,
                         const int32_t* cids, int64_t nc, int32_t K, int32_t* out,
                         uint64_t* workspace, int slices, hipStream_t s) {
  if (nq == 0) return hipSuccess;
  KnnArgs A;
  A.X = X;
  A.n = n;
  A.d = d;
  A.qids = qids;
  A.nq = nq;
  A.cids = cids;
  A.nc = nc;
  const int64_t per = (nc + slices - 1) / slices;
  A.per_slice = (per + kCB - 1) / kCB * kCB;
  A.K = K;
  A.out = out;
  A.part = slices > 1 ? workspace : nullptr;
  hipError_t e;
  if (d <= 32) e = launch_nk<1>(A, slices, s);
  else if (d <= 64) e = launch_nk<2>(A, slices, s);
  else if (d <= 128) e = launch_nk<4>(A, slices, s);
  else e = launch_nk<8>(A, slices, s);
  if (e != hipSuccess || slices == 1) return e;
  hipLaunchKernelGGL(knn_merge_kernel, dim3((unsigned)nq), dim3(64), 0, s, workspace, nq,
                     slices, K, out);
  return hipGetLastError();
}

}  // namespace rp
