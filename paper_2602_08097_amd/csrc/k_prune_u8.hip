// k_prune_u8.hip -- batched RP-Tuning for uint8 points on int8 MFMA.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep from a single gather of the candidate
// rows.  For out-lists of at most 64 ids and d a multiple of 16 (d <= 256):
//
//  a1  read:   lane t holds the t-th listed id; p itself is dropped here.
//  a2  gather: rows are staged in LDS as int8 u = x - 128 (the shift leaves
//              every squared distance unchanged) with coalesced 16-byte loads:
//              d/16 consecutive lanes read one row.
//  a3  p-row:  S(p, j) = |u_p|^2 + |u_j|^2 - 2 <u_p, u_j>, exact in int32,
//              with 4-way int8 dot products.
//  a4  sort:   a 64-lane bitonic sort of keys (S(p, j), id, slot) packed in
//              64 bits.  The repeated argmin of Algorithm 1 over a shrinking
//              candidate set visits the candidates in this order; repeated
//              ids become adjacent and are dropped.
//  a5  Gram:   G = U U^T over the rank-ordered rows on
//              v_mfma_i32_32x32x32_i8 (exact int32 accumulation); only the
//              blocks on or above the diagonal are formed, and
//              S(i, j) = |u_i|^2 + |u_j|^2 - 2 G(i, j) is written to LDS.
//  a6  test:   alpha * D(p*, p') <= D(p, p') on squares is
//              num^2 S(p*, p') <= den^2 S(p, p')  <=>  S(p*, p') <= T(p'),
//              T(p') = floor(den^2 S(p, p') / num^2), exact for integer S.
//  a7  greedy: per alpha a 64-bit survivor mask in scalar registers:
//              p* = lowest surviving rank, kept; its S row is read from LDS
//              and one ballot of S(p*, .) <= T removes every candidate it
//              prunes.  All alphas advance in lockstep so their LDS reads
//              overlap.  The chain stops at the largest R requested for that
//              alpha; a smaller R is the prefix of the same chain.
//  a8  write:  the kept ranks of each output are scattered to their
//              positions (popcount of the kept ranks before them), -1 padded.
#include "dev_common.h"

namespace rp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

// LDS per wave: max(U tile, S tile) + per-rank squared norms.
//   U tile: 65 rows (64 candidates + p) of d + 16 bytes (padding staggers banks)
//   S tile: rows 0..31 x 64 columns, rows 32..63 x 32 columns (upper blocks)
constexpr int kSTileBytes = (32 * 64 + 32 * 32) * 4;  // 12 KiB
constexpr int kMaxDimU8 = 256;
constexpr int kGatherBatch = 9;  // 16-byte loads in flight per lane (65 rows x 128 B = 520)

__host__ __device__ constexpr int u_stride(int d) { return d + 16; }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  int lo = __shfl_xor((int)(uint32_t)v, m, 64);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  int lo = __shfl((int)(uint32_t)v, src, 64);
  int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Ascending bitonic sort of one 64-bit key per lane across the wavefront.
__device__ __forceinline__ uint64_t wave_sort(uint64_t key, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint64_t other = shfl_xor_u64(key, j);
      bool up = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      bool take_min = lower == up;
      uint64_t mn = key < other ? key : other;
      uint64_t mx = key < other ? other : key;
      key = take_min ? mn : mx;
    }
  }
  return key;
}

// floor(den2 * s / num2) for s < 2^28, exact.
__device__ __forceinline__ int32_t alpha_threshold(uint32_t num2, uint32_t den2, uint32_t s) {
  const uint64_t B = (uint64_t)den2 * s;
  int64_t t = (int64_t)((double)B / (double)num2);
  int64_t r = (int64_t)B - (int64_t)num2 * t;
  for (int it = 0; it < 4 && r < 0; ++it) { --t; r += num2; }
  for (int it = 0; it < 4 && r >= (int64_t)num2; ++it) { ++t; r -= num2; }
  return (int32_t)t;
}

template <int NA>
__global__ __launch_bounds__(64) void prune_u8_kernel(GraphView g, SweepArgs a, int32_t idbits,
                                                      DevCounters* ctr) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int lane = threadIdx.x;
  const int64_t p = blockIdx.x;
  const int d = g.d;
  const int stride = u_stride(d);
  int8_t* U = (int8_t*)lds;                       // U tile (rows 0..63 candidates, 64 = p)
  int32_t* Stile = (int32_t*)lds;                 // S tile (overlays U after the Gram)
  const int tile_bytes = max(65 * stride, kSTileBytes);
  int32_t* nr = (int32_t*)(lds + tile_bytes);     // |u|^2 by rank
  int32_t* idl = nr + 64;                          // listed ids (slot order), then p
  const uint8_t* X = (const uint8_t*)g.X;

  // ---- a1: read the list -------------------------------------------------
  const int m = g.deg[p];
  int id = lane < m ? g.nbr[p * g.r_max + lane] : -1;
  idl[lane] = id;
  if (lane == 0) idl[64] = (int)p;
  __syncthreads();

  // ---- a2: coalesced gather into LDS (u = x - 128) -----------------------
  // Every load of a batch is issued before any of its stores so that the
  // lane's loads are in flight together.
  {
    const int cpr = d >> 4;  // 16-byte chunks per row
    const int total = 65 * cpr;
    const float inv_cpr = 1.0f / (float)cpr;
    for (int base = 0; base < total; base += 64 * kGatherBatch) {
      uint4 buf[kGatherBatch];
      int dst[kGatherBatch];
#pragma unroll
      for (int t = 0; t < kGatherBatch; ++t) {
        const int c = base + lane + 64 * t;
        buf[t] = make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u);
        dst[t] = -1;
        if (c < total) {
          const int row = (int)(((float)c + 0.5f) * inv_cpr);
          const int col = c - row * cpr;
          const int rid = idl[row];
          dst[t] = row * stride + col * 16;
          if (rid >= 0) buf[t] = *(const uint4*)(X + (int64_t)rid * d + col * 16);
        }
      }
#pragma unroll
      for (int t = 0; t < kGatherBatch; ++t) {
        if (dst[t] >= 0) {
          uint4 v = buf[t];
          v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
          *(uint4*)(U + dst[t]) = v;
        }
      }
    }
  }
  __syncthreads();

  // ---- a3: p-row S(p, j) and |u_j|^2 ------------------------------------
  int32_t nj = 0, dotp = 0, np = 0;
  {
    const int8_t* uj = U + lane * stride;
    const int8_t* up = U + 64 * stride;
    for (int c = 0; c < d; c += 16) {
      int4 xj = *(const int4*)(uj + c);
      int4 xp = *(const int4*)(up + c);
      nj = __builtin_amdgcn_sdot4(xj.x, xj.x, nj, false);
      nj = __builtin_amdgcn_sdot4(xj.y, xj.y, nj, false);
      nj = __builtin_amdgcn_sdot4(xj.z, xj.z, nj, false);
      nj = __builtin_amdgcn_sdot4(xj.w, xj.w, nj, false);
      dotp = __builtin_amdgcn_sdot4(xj.x, xp.x, dotp, false);
      dotp = __builtin_amdgcn_sdot4(xj.y, xp.y, dotp, false);
      dotp = __builtin_amdgcn_sdot4(xj.z, xp.z, dotp, false);
      dotp = __builtin_amdgcn_sdot4(xj.w, xp.w, dotp, false);
      np = __builtin_amdgcn_sdot4(xp.x, xp.x, np, false);
      np = __builtin_amdgcn_sdot4(xp.y, xp.y, np, false);
      np = __builtin_amdgcn_sdot4(xp.z, xp.z, np, false);
      np = __builtin_amdgcn_sdot4(xp.w, xp.w, np, false);
    }
  }
  const uint32_t sp = (uint32_t)(np + nj - 2 * dotp);

  // ---- a4: sort by (S(p, j), id); drop p and repeated ids ---------------
  const uint64_t kInvalid = ~0ull;
  const int shift = idbits + 6;
  uint64_t key = (id >= 0 && id != (int)p)
                     ? (((uint64_t)sp << shift) | ((uint64_t)(uint32_t)id << 6) | (uint64_t)lane)
                     : kInvalid;
  key = wave_sort(key, lane);
  {
    uint64_t prev = shfl_u64(key, lane > 0 ? lane - 1 : 0);
    bool dup = lane > 0 && key != kInvalid && (key >> 6) == (prev >> 6);
    if (dup) key = kInvalid - 1;  // stays after every valid key; never alive
  }
  const bool valid = key < kInvalid - 1;
  const uint64_t valid_mask = __ballot(valid);
  const int slot = (int)(key & 63);
  const uint32_t s_rank = valid ? (uint32_t)(key >> shift) : 0u;
  const int id_rank = valid ? (int)((key >> 6) & ((1ull << idbits) - 1)) : -1;
  const int32_t n_rank = __shfl(nj, slot, 64);
  nr[lane] = n_rank;

  // ---- a5: Gram tile on MFMA (rank order) -------------------------------
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int sl0 = __shfl(slot, l32, 64);        // row of rank l32
  const int sl1 = __shfl(slot, 32 + l32, 64);   // row of rank 32 + l32
  v16i acc00 = {0}, acc01 = {0}, acc11 = {0};
  const int d32 = (d + 31) & ~31;
  for (int kk = 0; kk < d32; kk += 32) {
    const int off = kk + half * 16;
    v4i f0 = {0, 0, 0, 0}, f1 = {0, 0, 0, 0};
    if (off < d) {
      f0 = *(const v4i*)(U + sl0 * stride + off);
      f1 = *(const v4i*)(U + sl1 * stride + off);
    }
    acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0, f0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0, f1, acc01, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f1, f1, acc11, 0, 0, 0);
  }
  __syncthreads();  // every U read done before the S tile overwrites it

  // Accumulator layout of a 32x32 block: lane l holds column l % 32 of rows
  // 8 (v / 4) + 4 (l / 32) + v % 4 in register v.
  {
    const int32_t ncol0 = nr[l32];
    const int32_t ncol1 = nr[32 + l32];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v >> 2) + 4 * half + (v & 3);
      const int32_t nrow0 = nr[r];
      const int32_t nrow1 = nr[32 + r];
      Stile[r * 64 + l32] = nrow0 + ncol0 - 2 * acc00[v];
      Stile[r * 64 + 32 + l32] = nrow0 + ncol1 - 2 * acc01[v];
      Stile[32 * 64 + r * 32 + l32] = nrow1 + ncol1 - 2 * acc11[v];
    }
  }
  __syncthreads();

  // ---- a6: thresholds per alpha -----------------------------------------
  int32_t T[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) T[ai] = alpha_threshold(a.num2[ai], a.den2[ai], s_rank);

  // ---- a7: greedy keep / discard (all alphas in lockstep) ---------------
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) rmax[ai] = 0;
  for (int o = 0; o < a.n_out; ++o) {
#pragma unroll
    for (int ai = 0; ai < NA; ++ai)
      if (a.out[o].alpha_idx == ai) rmax[ai] = max(rmax[ai], a.out[o].R);
  }
  uint64_t alive[NA], kept[NA];
  int cnt[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    alive[ai] = valid_mask;
    kept[ai] = 0;
    cnt[ai] = 0;
  }
  // lane offset of the S-row read: rows < 32 span 64 columns, rows >= 32
  // hold columns 32..63 (lanes < 32 read a duplicate and their bits are
  // already dead: every rank below p*'s is settled).
  const int col_hi = 32 * 64 + (lane >= 32 ? lane - 32 : lane);
  for (;;) {
    bool any = false;
    int32_t row[NA];
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      row[ai] = 0;
      if (alive[ai] != 0 && cnt[ai] < rmax[ai]) {
        const int i = __ffsll((long long)alive[ai]) - 1;
        kept[ai] |= 1ull << i;
        alive[ai] &= ~(1ull << i);
        ++cnt[ai];
        if (cnt[ai] < rmax[ai] && alive[ai] != 0) {
          const int addr = i < 32 ? i * 64 + lane : col_hi + (i - 32) * 32;
          row[ai] = Stile[addr];
          any = true;
        } else {
          alive[ai] = 0;
        }
      }
    }
    if (!any) break;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      if (alive[ai] != 0) alive[ai] &= ~(uint64_t)__ballot(row[ai] <= T[ai]);
    }
  }

  // ---- a8: write every output -------------------------------------------
  for (int o = 0; o < a.n_out; ++o) {
    const SweepOut& out = a.out[o];
    uint64_t km = 0;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai)
      if (out.alpha_idx == ai) km = kept[ai];
    const int R = out.R;
    const int total = __popcll(km);
    const int cntR = total < R ? total : R;
    int32_t* orow = out.nbr + p * R;
    if ((km >> lane) & 1ull) {
      const int pos = __popcll(km & ((1ull << lane) - 1ull));
      if (pos < R) orow[pos] = id_rank;
    }
    for (int t = cntR + lane; t < R; t += 64) orow[t] = -1;
    if (lane == 0) out.deg[p] = cntR;
  }
}

}  // namespace

bool prune_u8_supported(const GraphView& g) {
  return g.dtype == RP_U8 && g.r_max <= 64 && (g.d % 16) == 0 && g.d <= kMaxDimU8 &&
         g.n <= (1ll << 30);
}

hipError_t launch_prune_u8(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                           hipStream_t s) {
  int idbits = 1;
  while ((1ll << idbits) < g.n) ++idbits;
  const int stride = u_stride(g.d);
  const size_t shmem = (size_t)max(65 * stride, kSTileBytes) + (64 + 68) * sizeof(int32_t);
  dim3 grid((unsigned)g.n), block(64);
#define RP_LAUNCH_U8(NA_)                                                                   \
  case NA_:                                                                                 \
    hipLaunchKernelGGL(prune_u8_kernel<NA_>, grid, block, shmem, s, g, a, idbits, ctr); \
    break;
  switch (a.n_alpha) {
    RP_LAUNCH_U8(1)
    RP_LAUNCH_U8(2)
    RP_LAUNCH_U8(3)
    RP_LAUNCH_U8(4)
    RP_LAUNCH_U8(5)
    RP_LAUNCH_U8(6)
    RP_LAUNCH_U8(7)
    RP_LAUNCH_U8(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RP_LAUNCH_U8
  return hipGetLastError();
}

}  // namespace rp
