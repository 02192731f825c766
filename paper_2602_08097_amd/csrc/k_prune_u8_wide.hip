// k_prune_u8_wide.hip -- batched RP-Tuning for uint8 points with out-lists of
// 65 to 128 ids (four row blocks of 32 slots), d <= 128: the base-graph
// prune of 128-NN lists and sweeps over graphs of degree up to 128.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex at every alpha of a sweep, as the 64-candidate kernel does, with
// rank masks of two 64-bit words (rank t is bit t % 64 of word t / 64, held
// by lane t % 64):
//  a1  read:   slot t's id in lane t % 64 of word t / 64.
//  a2  gather: row block b (slots 32 b .. 32 b + 31) goes straight from
//              global memory into the int8 MFMA operand registers: lane l
//              holds bytes 32 k + 16 (l / 32) .. + 15 of row 32 b + l % 32,
//              shifted to u = x - 128.
//  a3  p-row:  S(p, j) = |u_p|^2 + |u_j|^2 - 2 <u_p, u_j> exact in int32
//              (byte dot products for |u_j|^2, the matrix unit with x_p in
//              every row of the left operand for <u_p, u_j> and |u_p|^2).
//  a4  sort:   (S(p, j), id, slot) keys; a list in rank order (every K-NN
//              list and every RobustPrune output) is used as read, otherwise
//              two 64-key sorts and a merge order the 128 keys and the rows
//              are read again by rank.  UnsortedRobustPrune keeps the list
//              order.  p and repeated ids are dropped.
//  a5  Gram:   the ten 32 x 32 blocks on and above the diagonal on
//              v_mfma_i32_32x32x32_i8 (exact).
//  a6  test:   S(p*, p') <= T_k(p') = floor(den_k^2 S(p, p') / num_k^2), the
//              codes 2^c - 1 of the alphas that prune, one byte per pair.
//  a7  greedy: per alpha, the ranks not pruned so far and the candidates (not
//              pruned, after the last visited row, whose row can prune), two
//              words each; each step keeps the survivors up to the first
//              candidate, which removes what its row prunes.  A chain stops at
//              its largest R.
//  a8  write:  kept ids in rank order, -1 padded.
#include <type_traits>

#include "u8_common.h"

namespace rp {

using namespace u8;

namespace {

constexpr int kNB = 4;                      // row blocks
constexpr int kMS = 32 * kNB;               // slots
constexpr int kNK = 4;                      // 32-byte steps (d <= 128)
constexpr int kTileBytes = 1024 * 10;       // codes of the blocks on and above the diagonal
constexpr int kWaveLdsWide = kTileBytes + kMS * 4;  // + -16 |u|^2 by rank

// Column block cb of the code tile holds rows 0 .. 32 cb + 31, 32 bytes each:
// entry (i, j) sits at cbase(j / 32) + 32 i + j % 32.
__host__ __device__ constexpr int cbase(int cb) { return 512 * cb * (cb + 1); }

__device__ __forceinline__ int ff1(uint64_t v) {
  const uint64_t u = uniform_u64(v);
  int i;
  asm("s_ff1_i32_b64 %0, %1" : "=s"(i) : "s"(u));
  return i;  // -1 for an empty mask
}

// The codes of block (BI, BJ) from its Gram accumulator (lane l holds column
// l % 32 of rows 8 (v / 4) + 4 (l / 32) + v % 4 in register v).
template <int NA, int BI, int BJ>
__device__ __forceinline__ void decide_block(uint8_t* C, const int32_t* mnr, const v16i& acc,
                                             const ColBounds<NA>& cb, int l32, int half) {
  int4 nrow[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) nrow[q] = *(const int4*)(mnr + 32 * BI + 8 * q + 4 * half);
  uint8_t* base = C + cbase(BJ) + 32 * (32 * BI + 4 * half) + l32;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int rr = 8 * (v >> 2) + (v & 3);
    const int4 nq = nrow[v >> 2];
    const int32_t mn16 = (v & 3) == 0 ? nq.x : (v & 3) == 1 ? nq.y : (v & 3) == 2 ? nq.z : nq.w;
    const int32_t Y = acc[v] * 32 + mn16;
    int32_t lo = cb.off_lo;
#pragma unroll
    for (int k = 0; k < (NA < 4 ? NA : 4); ++k) lo += med3_i32(Y, cb.A[k], cb.B[k]);
    uint32_t t = (uint32_t)lo;
    if (NA > 4) {
      int32_t hi = cb.off_hi;
#pragma unroll
      for (int k = 4; k < NA; ++k) hi += med3_i32(Y, cb.A[k], cb.B[k]);
      t += (uint32_t)hi << 4;
    }
    base[32 * rr] = (uint8_t)t;
  }
}

// Rows of the four blocks for the ids held by word 0 / word 1 (absent slots
// read x_p; their keys are invalid).
__device__ __forceinline__ void load_blocks(v4i (&f)[kNB][kNK], const uint8_t* X, int d,
                                            int64_t p, const int (&idw)[2], int l32, int half) {
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    const int id = __shfl(idw[b >> 1], 32 * (b & 1) + l32, 64);
    const uint8_t* r = X + (int64_t)(id >= 0 ? id : (int)p) * d;
#pragma unroll
    for (int k = 0; k < kNK; ++k) f[b][k] = *(const v4i*)(r + min(32 * k + 16 * half, d - 16));
  }
}

__device__ __forceinline__ void shift_blocks(v4i (&f)[kNB][kNK], int d, int half) {
  const v4i zero = {0, 0, 0, 0};
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
#pragma unroll
    for (int k = 0; k < kNK; ++k) f[b][k] = 32 * k + 16 * half < d ? shift_u8(f[b][k]) : zero;
  }
}

// |u|^2 of each block's row l % 32 (both halves of the row combined).
__device__ __forceinline__ void block_norms(const v4i (&f)[kNB][kNK], int (&nb)[kNB]) {
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    int acc = 0;
#pragma unroll
    for (int k = 0; k < kNK; ++k) acc = sdot16(f[b][k], f[b][k], acc);
    nb[b] = acc + __shfl_xor(acc, 32, 64);
  }
}

template <int NA, bool CAP>
__global__ __launch_bounds__(256) void prune_u8_wide_kernel(GraphView g, SweepArgs a,
                                                            int32_t idbits, int32_t nr_out,
                                                            int32_t wave_lds) {
  extern __shared__ __align__(16) uint8_t lds_all[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (p >= g.n) return;
  uint8_t* C = lds_all + (size_t)wave * wave_lds;   // code tile
  int32_t* nr = (int32_t*)(C + kTileBytes);        // -16 |u|^2 by rank
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int d = g.d;
  const uint8_t* X = (const uint8_t*)g.X;

  // ---- a1 + a2 ---------------------------------------------------------------
  v4i fp[kNK];
  const uint8_t* rp_ = X + p * d;
#pragma unroll
  for (int k = 0; k < kNK; ++k) fp[k] = *(const v4i*)(rp_ + min(32 * k + 16 * half, d - 16));
  int idw[2];
  {
    const int m = g.deg[p];
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      const int t = lane + 64 * w;
      const int raw = t < g.r_max ? g.nbr[p * g.r_max + t] : -1;
      idw[w] = (t < m && raw != (int)p) ? raw : -1;
    }
  }
  v4i f[kNB][kNK];
  load_blocks(f, X, d, p, idw, l32, half);
  shift_blocks(f, d, half);
  {
    const v4i zero = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kNK; ++k) fp[k] = 32 * k + 16 * half < d ? shift_u8(fp[k]) : zero;
  }

  // ---- a3: p-row ---------------------------------------------------------------
  int nb[kNB];
  block_norms(f, nb);
  int qb[kNB];
#pragma unroll
  for (int b = 0; b < kNB; ++b) {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < kNK; ++k) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(fp[k], f[b][k], acc, 0, 0, 0);
    qb[b] = acc[0];
  }
  int np;
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < kNK; ++k) acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(fp[k], fp[k], acc, 0, 0, 0);
    np = acc[0];
  }
  // slot lane + 64 w lives in block 2 w + half
  uint64_t key[2];
  const int shift = idbits + 7;
  const uint64_t kInvalid = ~0ull;
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int b0 = 2 * w, b1 = 2 * w + 1;
    const int nj = half ? nb[b1] : nb[b0];
    const int qj = half ? qb[b1] : qb[b0];
    const uint32_t sp = (uint32_t)(np + nj - 2 * qj);
    key[w] = idw[w] >= 0 ? (((uint64_t)sp << shift) | ((uint64_t)(uint32_t)idw[w] << 7) |
                            (uint64_t)(lane + 64 * w))
                         : kInvalid;
  }

  // ---- a4: rank order; drop repeated ids ----------------------------------------
  bool dup[2] = {false, false};
  if (a.unsorted) {
    // UnsortedRobustPrune: ranks are the list order; a repeated id counts at
    // its first slot
#pragma unroll 1
    for (int t = 0; t < 64; ++t) {
      const int v = __builtin_amdgcn_readlane(idw[0], t);
      dup[0] = dup[0] || (t < lane && v >= 0 && v == idw[0]);
      dup[1] = dup[1] || (v >= 0 && v == idw[1]);
    }
#pragma unroll 1
    for (int t = 0; t < 63; ++t) {
      const int v = __builtin_amdgcn_readlane(idw[1], t);
      dup[1] = dup[1] || (t < lane && v >= 0 && v == idw[1]);
    }
  } else {
    uint64_t prev0 = shfl_u64(key[0], lane > 0 ? lane - 1 : 0);
    uint64_t prev1 = shfl_u64(key[1], lane > 0 ? lane - 1 : 0);
    const uint64_t last0 = shfl_u64(key[0], 63);
    if (lane == 0) prev1 = last0;
    const bool out_of_order = (lane > 0 && key[0] < prev0) || key[1] < prev1;
    if (__ballot(out_of_order) != 0) {
      // sort each word, then merge: b reversed makes a ++ b bitonic, the
      // elementwise minimum holds the 64 smallest
      uint64_t ka = wave_sort(key[0], lane);
      uint64_t kb = wave_sort(key[1], lane);
      const uint64_t rb = shfl_u64(kb, 63 - lane);
      const uint64_t lo = ka < rb ? ka : rb;
      const uint64_t hi = ka < rb ? rb : ka;
      key[0] = lo;
      key[1] = hi;
#pragma unroll
      for (int w = 0; w < 2; ++w) {
        key[w] = bitonic_step<64, 32>(key[w], lane);
        key[w] = bitonic_step<64, 16>(key[w], lane);
        key[w] = bitonic_step<64, 8>(key[w], lane);
        key[w] = bitonic_step<64, 4>(key[w], lane);
        key[w] = bitonic_step<64, 2>(key[w], lane);
        key[w] = bitonic_step<64, 1>(key[w], lane);
      }
      // the rows again, by rank
      int idr[2];
#pragma unroll
      for (int w = 0; w < 2; ++w)
        idr[w] = key[w] != kInvalid ? (int)((key[w] >> 7) & ((1ull << idbits) - 1)) : -1;
      load_blocks(f, X, d, p, idr, l32, half);
      shift_blocks(f, d, half);
      block_norms(f, nb);
      prev0 = shfl_u64(key[0], lane > 0 ? lane - 1 : 0);
      prev1 = shfl_u64(key[1], lane > 0 ? lane - 1 : 0);
      const uint64_t l0 = shfl_u64(key[0], 63);
      if (lane == 0) prev1 = l0;
    }
    dup[0] = lane > 0 && key[0] != kInvalid && (key[0] >> 7) == (prev0 >> 7);
    dup[1] = key[1] != kInvalid && (key[1] >> 7) == (prev1 >> 7);
  }
  uint64_t vm[2];
  int id_rank[2];
  uint32_t s_rank[2];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const bool valid = key[w] != kInvalid && !dup[w];
    vm[w] = __ballot(valid);
    id_rank[w] = valid ? (int)((key[w] >> 7) & ((1ull << idbits) - 1)) : -1;
    s_rank[w] = valid ? (uint32_t)(key[w] >> shift) : 0u;
    // -16 |u|^2 of rank lane + 64 w: its row sits in block 2 w + half (the
    // rows are in rank order now, or the list was)
    nr[lane + 64 * w] = -16 * (half ? nb[2 * w + 1] : nb[2 * w]);
  }
  wave_sync();

  // ---- a5 + a6: Gram blocks and codes, column block by column block ------------
  int32_t Tw[2][NA];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
#pragma unroll
    for (int k = 0; k < NA; ++k) Tw[w][k] = alpha_threshold(a.thr_mul[k], s_rank[w]);
  }
  auto column = [&](auto BJc) {
    constexpr int BJ = decltype(BJc)::value;
    int32_t T[NA];
#pragma unroll
    for (int k = 0; k < NA; ++k) T[k] = __shfl(Tw[BJ >> 1][k], 32 * (BJ & 1) + l32, 64);
    const ColBounds<NA> cb = col_bounds<NA>(-nr[32 * BJ + l32], T);  // 16 |u_j|^2
    auto blockc = [&](auto BIc) {
      constexpr int BI = decltype(BIc)::value;
      v16i acc = {0};
#pragma unroll
      for (int k = 0; k < kNK; ++k)
        acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(f[BI][k], f[BJ][k], acc, 0, 0, 0);
      decide_block<NA, BI, BJ>(C, nr, acc, cb, l32, half);
    };
    blockc(std::integral_constant<int, 0>{});
    if constexpr (BJ >= 1) blockc(std::integral_constant<int, 1>{});
    if constexpr (BJ >= 2) blockc(std::integral_constant<int, 2>{});
    if constexpr (BJ >= 3) blockc(std::integral_constant<int, 3>{});
  };
  column(std::integral_constant<int, 0>{});
  column(std::integral_constant<int, 1>{});
  column(std::integral_constant<int, 2>{});
  column(std::integral_constant<int, 3>{});
  wave_sync();

  // ---- a7: greedy --------------------------------------------------------------
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    rmax[ai] = kMS;
    if (CAP) {
      rmax[ai] = 0;
      for (int ir = 0; ir < nr_out; ++ir) rmax[ai] = max(rmax[ai], a.out[ai * nr_out + ir].R);
    }
  }
  // rows that can prune at each alpha: the OR of row i's codes over the
  // columns after i (row i = lane + 64 w)
  uint64_t vis[NA][2];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    const int i = lane + 64 * w;
    const int ib = i >> 5;
    uint32_t acc;
    {
      const uint8_t* drow = C + cbase(ib) + 32 * i;
      const uint4 d0 = *(const uint4*)drow;
      const uint4 d1 = *(const uint4*)(drow + 16);
      const uint64_t q[4] = {(uint64_t)d0.y << 32 | d0.x, (uint64_t)d0.w << 32 | d0.z,
                             (uint64_t)d1.y << 32 | d1.x, (uint64_t)d1.w << 32 | d1.z};
      const int drop = 8 * ((i & 31) + 1);  // bits of the columns up to i
      uint64_t a64 = 0;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int h = min(max(drop - 64 * t, 0), 64) >> 1;
        a64 |= (q[t] >> h) >> h;
      }
      acc = (uint32_t)a64 | (uint32_t)(a64 >> 32);
    }
#pragma unroll
    for (int cb = 1; cb < kNB; ++cb) {
      if (cb > ib) {
        const uint4 r0 = *(const uint4*)(C + cbase(cb) + 32 * i);
        const uint4 r1 = *(const uint4*)(C + cbase(cb) + 32 * i + 16);
        acc |= r0.x | r0.y | r0.z | r0.w | r1.x | r1.y | r1.z | r1.w;
      }
    }
    acc |= acc >> 16;
    acc |= acc >> 8;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) vis[ai][w] = __ballot((acc >> ai) & 1u) & vm[w];
  }
  uint64_t rem[NA][2], cand[NA][2];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
#pragma unroll
    for (int w = 0; w < 2; ++w) {
      rem[ai][w] = vm[w];
      cand[ai][w] = vis[ai][w];
    }
  }
  // tile column of this lane in word w: rank lane + 64 w
  const int lb0 = cbase(half) + l32;
  const int lb1 = cbase(2 + half) + l32;
  // Chains with larger alpha prune less and visit fewer rows: phase s0
  // advances chains 0..s0 while chain s0 has a candidate (a finished chain
  // repeats harmless empty steps).
#pragma unroll
  for (int s0 = NA - 1; s0 >= 0; --s0) {
    if ((uniform_u64(cand[s0][0]) | uniform_u64(cand[s0][1])) == 0) continue;
    do {
#pragma unroll
      for (int ai = 0; ai <= s0; ++ai) {
        const int i0 = ff1(cand[ai][0]);
        const int i1 = ff1(cand[ai][1]);
        const int i = i0 >= 0 ? i0 : (i1 >= 0 ? 64 + i1 : 0);
        // ranks after the candidate i (none if the chain has no candidate)
        uint64_t ab0 = i0 >= 0 ? (0xFFFFFFFFFFFFFFFEull << i0) : 0ull;
        uint64_t ab1 = i0 >= 0 ? ~0ull : (i1 >= 0 ? (0xFFFFFFFFFFFFFFFEull << i1) : 0ull);
        const uint32_t row0 = C[32 * i + lb0];
        const uint32_t row1 = C[32 * i + lb1];
        const uint64_t b0 = __ballot(row0 >= (1u << ai));
        const uint64_t b1 = __ballot(row1 >= (1u << ai));
        uint64_t r0 = uniform_u64(rem[ai][0]) & ~(b0 & ab0);
        uint64_t r1 = uniform_u64(rem[ai][1]) & ~(b1 & ab1);
        if (CAP && __popcll(r0 & ~ab0) + __popcll(r1 & ~ab1) >= rmax[ai]) {  // R kept: stop
          r0 &= ~ab0;
          r1 &= ~ab1;
          ab0 = 0;
          ab1 = 0;
        }
        rem[ai][0] = r0;
        rem[ai][1] = r1;
        cand[ai][0] = r0 & ab0 & vis[ai][0];
        cand[ai][1] = r1 & ab1 & vis[ai][1];
      }
    } while ((uniform_u64(cand[s0][0]) | uniform_u64(cand[s0][1])) != 0);
  }

  // a chain that reached its R keeps its first R ranks
  uint64_t kept[NA][2];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    const uint64_t k0 = rem[ai][0], k1 = rem[ai][1];
    kept[ai][0] = k0;
    kept[ai][1] = k1;
    if (CAP && __popcll(k0) + __popcll(k1) > rmax[ai]) {
      const int b0 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(k0 >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)k0, 0u));
      const int b1 = __popcll(k0) + (int)__builtin_amdgcn_mbcnt_hi(
                                        (uint32_t)(k1 >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)k1, 0u));
      kept[ai][0] = __ballot(((k0 >> lane) & 1ull) && b0 < rmax[ai]);
      kept[ai][1] = __ballot(((k1 >> lane) & 1ull) && b1 < rmax[ai]);
    }
  }

  // ---- a8: outputs -------------------------------------------------------------
  auto write_out = [&](const SweepOut& out, int ai) {
    const uint64_t k0 = kept[ai][0], k1 = kept[ai][1];
    const int c0 = __popcll(k0);
    const int tot = c0 + __popcll(k1);
    const int R = out.R;
    const int cntR = tot < R ? tot : R;
    int32_t* orow = out.nbr + p * R;
    const int pos0 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(k0 >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)k0, 0u));
    const int pos1 = c0 + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(k1 >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)k1, 0u));
    if (((k0 >> lane) & 1ull) && pos0 < R) orow[pos0] = id_rank[0];
    if (((k1 >> lane) & 1ull) && pos1 < R) orow[pos1] = id_rank[1];
    for (int t = cntR + lane; t < R; t += 64) orow[t] = -1;
    if (lane == 0) out.deg[p] = cntR;
  };
#pragma unroll
  for (int ai = 0; ai < NA; ++ai)
    for (int ir = 0; ir < nr_out; ++ir) write_out(a.out[ai * nr_out + ir], ai);
}

template <int NA>
hipError_t launch_na(const GraphView& g, const SweepArgs& a, int idbits, int waves,
                     hipStream_t s) {
  if (a.n_out % NA != 0 || a.n_out / NA > kMaxRs) return hipErrorInvalidValue;
  bool cap = false;
  for (int o = 0; o < a.n_out; ++o) cap = cap || a.out[o].R < g.r_max;
  const int nr_out = a.n_out / NA;
  const dim3 grid((unsigned)((g.n + waves - 1) / waves)), block(64 * waves);
  const size_t shmem = (size_t)kWaveLdsWide * waves;
  if (cap)
    hipLaunchKernelGGL((prune_u8_wide_kernel<NA, true>), grid, block, shmem, s, g, a, idbits,
                       nr_out, kWaveLdsWide);
  else
    hipLaunchKernelGGL((prune_u8_wide_kernel<NA, false>), grid, block, shmem, s, g, a, idbits,
                       nr_out, kWaveLdsWide);
  return hipGetLastError();
}

}  // namespace

int prune_u8_wide_wave_lds(const GraphView&) { return kWaveLdsWide; }

// 65..128 slots, d a multiple of 16 up to 128, 16-byte aligned points.
bool prune_u8_wide_supported(const GraphView& g) {
  return g.dtype == RP_U8 && g.r_max > 64 && g.r_max <= kMS && (g.d % 16) == 0 &&
         g.d <= 32 * kNK && g.n <= (1ll << 30) && (((uintptr_t)g.X) & 15) == 0;
}

// The alphas ascending (and thresholds) as the 64-slot kernel takes them.
SweepArgs u8_sweep_ascending(const SweepArgs& a_in);

hipError_t launch_prune_u8_wide(const GraphView& g, const SweepArgs& a_in, DevCounters* ctr,
                                hipStream_t s) {
  (void)ctr;
  const SweepArgs a = u8_sweep_ascending(a_in);
  int idbits = 1;
  while ((1ll << idbits) < g.n) ++idbits;
  const int waves = min(4, waves_for(TuneKey{kKernelU8Wide, g.dtype, g.d, g.r_max, a.n_alpha,
                                              a.n_out},
                                     kWaveLdsWide));
  switch (a.n_alpha) {
    case 1: return launch_na<1>(g, a, idbits, waves, s);
    case 2: return launch_na<2>(g, a, idbits, waves, s);
    case 3: return launch_na<3>(g, a, idbits, waves, s);
    case 4: return launch_na<4>(g, a, idbits, waves, s);
    case 5: return launch_na<5>(g, a, idbits, waves, s);
    case 6: return launch_na<6>(g, a, idbits, waves, s);
    case 7: return launch_na<7>(g, a, idbits, waves, s);
    case 8: return launch_na<8>(g, a, idbits, waves, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rp
