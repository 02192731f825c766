// k_prune_u8.hip -- batched RP-Tuning for uint8 points on int8 MFMA.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep from a single read of the candidate
// rows.  For out-lists of at most 64 ids and d a multiple of 16 (d <= 256):
//
//  a1  read:   lane t holds the t-th listed id (its slot).
//  a2  gather: the rows go straight from global memory into the registers
//              the matrix instruction takes: for row block b (slots
//              32 b .. 32 b + 31) lane l holds bytes 32 k + 16 (l / 32) .. + 15
//              of row 32 b + l % 32 for every 32-byte step k -- one 16-byte
//              load each, all in flight together -- shifted to int8
//              u = x - 128 (the shift leaves every difference unchanged).
//              No LDS staging.
//  a3  p-row:  S(p, j) = |u_p|^2 + |u_j|^2 - 2 <u_p, u_j>, exact in int32:
//              |u_j|^2 by 4-way int8 dot products on the same registers (the
//              two halves of a row combined across lanes l and l + 32),
//              <u_p, u_j> and |u_p|^2 on the matrix unit with x_p in every row
//              of the left operand.
//  a4  sort:   keys (S(p, j), id, slot) packed in 64 bits (UnsortedRobustPrune,
//              Section 3, keeps the list order and skips this step).  A list already in
//              (S, id) order -- every RobustPrune output is -- keeps its rows
//              where they are; otherwise a 64-lane bitonic sort (DPP and
//              swizzle exchanges) orders the keys and the rows move to their
//              ranks by lane permutes.  The repeated argmin of Algorithm 1
//              over a shrinking candidate set visits the candidates in this
//              order; p and repeated ids are dropped.
//  a5  Gram:   G = U U^T over the rank-ordered rows on
//              v_mfma_i32_32x32x32_i8 (exact int32 accumulation), one 32 x 32
//              block at a time, blocks on and above the diagonal only.
//  a6  test:   alpha * D(p*, p') <= D(p, p') on squares is
//              num^2 S(p*, p') <= den^2 S(p, p')  <=>  S(p*, p') <= T(p'),
//              T(p') = floor(den^2 S(p, p') / num^2), exact for integer S
//              (one 64-bit reciprocal multiply).  With the alphas ascending,
//              the alphas that prune p' from p* are a prefix 0..c-1; the
//              3 KiB decision tile stores 2^c - 1, summed from one median per
//              alpha.
//  a7  greedy: per alpha a 64-bit survivor mask.  Survivors whose row prunes
//              nothing at that alpha are kept in runs; each survivor whose row
//              can prune is kept and one ballot over its tile row removes what
//              it prunes.  A chain stops at the largest R requested for its
//              alpha; a smaller R is a prefix.
//  a8  write:  kept ranks are scattered to their positions (popcount of the
//              kept ranks before them), -1 padded.
#include "u8_common.h"

namespace rp {

using namespace u8;

namespace {

constexpr int kDecisionBytes = 3072;  // decision tile: the blocks on and above the diagonal
constexpr int kMaxDimU8 = 256;
constexpr int kWaveLdsU8 = kDecisionBytes + 64 * 4;  // + -16 |u|^2 by rank

// a1: the list of p (row and degree loads in flight together).
__device__ __forceinline__ int load_list(const GraphView& g, int64_t p, int lane) {
  const int raw = lane < g.r_max ? g.nbr[p * g.r_max + lane] : -1;
  const int m = g.deg[p];
  return lane < m ? raw : -1;
}

struct Front {
  uint64_t valid_mask;
  int id_rank;
};

// The decision codes of one 32 x 32 block (rows of block BI, columns of block
// BJ) from its Gram accumulator.  The diagonal blocks also code the columns up
// to the row: the greedy masks them off (those ranks are decided before the
// row is visited) and its row scan drops them.  Tile layout: columns 0..31 of
// rows 0..31 at byte 32 i + c; columns 32..63 of rows 0..63 at byte
// 1024 + 32 i + (c - 32).  Accumulator layout:
// lane l holds column l % 32 of rows 8 (v / 4) + 4 (l / 32) + v % 4 in
// register v.
template <int NA, int BI, int BJ>
__device__ __forceinline__ void decide_block(uint8_t* C, const int32_t* mnr, const v16i& acc,
                                             const ColBounds<NA>& cb, int l32, int half) {
  // -16 |u|^2 of this lane's 16 rows: rows 8 q + 4 half + 0..3 are consecutive
  int4 nrow[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) nrow[q] = *(const int4*)(mnr + 32 * BI + 8 * q + 4 * half);
  // row r = 8 q + 4 half + j of the block is byte base + 32 (8 q + j)
  uint8_t* base = C + (BJ == 0 ? 0 : 1024 + 32 * 32 * BI) + 128 * half + l32;
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int rr = 8 * (v >> 2) + (v & 3);  // r - 4 half, a constant
    const int4 nq = nrow[v >> 2];
    const int32_t mn16 = (v & 3) == 0 ? nq.x : (v & 3) == 1 ? nq.y : (v & 3) == 2 ? nq.z : nq.w;
    const int32_t Y = acc[v] * 32 + mn16;  // 16 y
    // U_k ascends with k, so the alphas that prune are 0..c-1 and the sum of
    // medians is the code 2^c - 1
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

// a1..a6 for vertex p: rows into registers, p-row, sort, Gram, decision tile.
template <int NA, int NK>
__device__ __forceinline__ Front node_front(uint8_t* C, int32_t* nr, const GraphView& g,
                                            const SweepArgs& a, int64_t p, int lane,
                                            int idbits) {
  const int d = g.d;
  const uint8_t* X = (const uint8_t*)g.X;
  const int l32 = lane & 31;
  const int half = lane >> 5;

  // ---- a1 ----------------------------------------------------------------
  const int id = load_list(g, p, lane);

  // ---- a2: 16-byte slices of every row, straight into registers ----------
  // every load reads valid memory (absent rows read x_p, slices past d read
  // the row's last 16 bytes) and is issued unconditionally; x_p's slices go
  // out while the list is still in flight
  v4i f0[NK], f1[NK], fp[NK];
  const uint8_t* rp = X + p * d;
#pragma unroll
  for (int k = 0; k < NK; ++k) fp[k] = *(const v4i*)(rp + min(32 * k + 16 * half, d - 16));
  __builtin_amdgcn_sched_barrier(0);
  const int usable = (id >= 0 && id != (int)p) ? id : -1;
  const int id0 = __shfl(usable, l32, 64);        // row of block 0 in this lane
  const int id1 = __shfl(usable, 32 + l32, 64);   // row of block 1
  const uint8_t* r0 = X + (int64_t)(id0 >= 0 ? id0 : (int)p) * d;
  const uint8_t* r1 = X + (int64_t)(id1 >= 0 ? id1 : (int)p) * d;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    const int off = min(32 * k + 16 * half, d - 16);
    f0[k] = *(const v4i*)(r0 + off);
    f1[k] = *(const v4i*)(r1 + off);
  }
  __builtin_amdgcn_sched_barrier(0);  // no use of x_p's slices before every load is out
  // (rows of absent slots hold x_p: their sort keys are invalid, and the codes
  // they produce only ever meet dead survivors)
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    f0[k] = shift_u8(f0[k]);
    f1[k] = shift_u8(f1[k]);
    fp[k] = shift_u8(fp[k]);
  }
  if (d != 32 * NK) {  // uniform: zero the slices past d
    const v4i zero = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      const bool in = 32 * k + 16 * half < d;
      f0[k] = in ? f0[k] : zero;
      f1[k] = in ? f1[k] : zero;
      fp[k] = in ? fp[k] : zero;
    }
  }

  // ---- a3: p-row S(p, j) and |u_j|^2 -------------------------------------
  // <u_p, u_j> and |u_p|^2 on the matrix unit: with x_p in every row of the
  // left operand, every row of the product is the p-row of inner products
  int n0 = 0, n1 = 0;
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    n0 = sdot16(f0[k], f0[k], n0);
    n1 = sdot16(f1[k], f1[k], n1);
  }
  n0 += __shfl_xor(n0, 32, 64);
  n1 += __shfl_xor(n1, 32, 64);
  int q0, q1, np;
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(fp[k], f0[k], acc, 0, 0, 0);
    q0 = acc[0];
  }
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(fp[k], f1[k], acc, 0, 0, 0);
    q1 = acc[0];
  }
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(fp[k], fp[k], acc, 0, 0, 0);
    np = acc[0];
  }
  // lane l is slot l: block 0 for l < 32, block 1 for l >= 32
  const int32_t nj = half ? n1 : n0;
  const uint32_t sp = (uint32_t)(np + nj - 2 * (half ? q1 : q0));

  // ---- a4: sort by (S(p, j), id); drop p and repeated ids ---------------
  const uint64_t kInvalid = ~0ull;
  const int shift = idbits + 6;
  uint64_t key = usable >= 0
                     ? (((uint64_t)sp << shift) | ((uint64_t)(uint32_t)id << 6) | (uint64_t)lane)
                     : kInvalid;
  bool dup = false;
  if (a.unsorted) {
    // UnsortedRobustPrune: the ranks are the list order (no sort); a repeated
    // id counts at its first slot
#pragma unroll 1
    for (int t = 0; t < 63; ++t) {
      const int v = __builtin_amdgcn_readlane(usable, t);
      dup = dup || (t < lane && v >= 0 && v == usable);
    }
  } else {
    uint64_t prev = shfl_u64(key, lane > 0 ? lane - 1 : 0);
    if (__ballot(lane > 0 && key < prev)) {
      key = wave_sort(key, lane);
      prev = shfl_u64(key, lane > 0 ? lane - 1 : 0);
      // rows to their ranks: row of rank 32 b + l32 comes from slot sl_b,
      // held by lane (sl_b % 32) + 32 half of block sl_b / 32
      const int slot = (int)(key & 63);
      const int sl0 = __shfl(slot, l32, 64);
      const int sl1 = __shfl(slot, 32 + l32, 64);
      const int src0 = (sl0 & 31) + 32 * half;
      const int src1 = (sl1 & 31) + 32 * half;
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const v4i a0 = shfl_v4i(f0[k], src0), b0 = shfl_v4i(f1[k], src0);
        const v4i a1 = shfl_v4i(f0[k], src1), b1 = shfl_v4i(f1[k], src1);
        f0[k] = sl0 >= 32 ? b0 : a0;
        f1[k] = sl1 >= 32 ? b1 : a1;
      }
    }
    dup = lane > 0 && key != kInvalid && (key >> 6) == (prev >> 6);
  }
  if (dup) key = kInvalid - 1;  // never alive
  const bool valid = key < kInvalid - 1;
  Front f;
  f.valid_mask = __ballot(valid);
  const int slot = (int)(key & 63);
  const uint32_t s_rank = valid ? (uint32_t)(key >> shift) : 0u;
  f.id_rank = valid ? (int)((key >> 6) & ((1ull << idbits) - 1)) : -1;
  const int32_t n_rank = __shfl(nj, slot, 64);
  nr[lane] = -16 * n_rank;  // -16 |u|^2 by rank

  // ---- a6: thresholds of this rank, then the bounds of the lane's two tile
  // columns (l32 and 32 + l32)
  int32_t T0[NA], T1[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    const int32_t t = alpha_threshold(a.thr_mul[k], s_rank);
    T0[k] = __shfl(t, l32, 64);
    T1[k] = __shfl(t, 32 + l32, 64);
  }
  const ColBounds<NA> cb0 = col_bounds<NA>(16 * __shfl(n_rank, l32, 64), T0);
  const ColBounds<NA> cb1 = col_bounds<NA>(16 * __shfl(n_rank, 32 + l32, 64), T1);
  wave_sync();  // the |u|^2 table is visible

  // ---- a5: Gram blocks on MFMA (rank order), then their decision codes ----
  // (every step runs: slices past d are zero)
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0[k], f0[k], acc, 0, 0, 0);
    decide_block<NA, 0, 0>(C, nr, acc, cb0, l32, half);
  }
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0[k], f1[k], acc, 0, 0, 0);
    decide_block<NA, 0, 1>(C, nr, acc, cb1, l32, half);
  }
  {
    v16i acc = {0};
#pragma unroll
    for (int k = 0; k < NK; ++k)
      acc = __builtin_amdgcn_mfma_i32_32x32x32_i8(f1[k], f1[k], acc, 0, 0, 0);
    decide_block<NA, 1, 1>(C, nr, acc, cb1, l32, half);
  }
  return f;
}

// a7 + a8 on the decision tile: greedy, outputs of p.
template <int NA, bool CAP>
__device__ __forceinline__ void node_back(const uint8_t* C, const SweepArgs& a, int64_t p,
                                          const Front& f, int lane, int NR) {
  // ---- a7: greedy keep / discard, all alphas in lockstep ----------------
  // outputs are alpha-major: output ai * NR + ir has alpha ai, bound R_ir
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    rmax[ai] = 64;
    if (CAP) {
      rmax[ai] = 0;
      for (int ir = 0; ir < NR; ++ir) rmax[ai] = max(rmax[ai], a.out[ai * NR + ir].R);
    }
  }
  // Rows that prune anything, per chain: the OR of row i's codes (lane i) over
  // the columns after i.  Columns 0..31 of rows 0..31 are at bytes 32 i ..;
  // columns 32..63 of every row at 1024 + 32 i ...
  uint64_t vis[NA];
  {
    // the lane's row in its diagonal block, less its first (i % 32) + 1 bytes
    const uint8_t* drow = C + (lane < 32 ? 32 * lane : 1024 + 32 * lane);
    const uint4 d0 = *(const uint4*)drow;
    const uint4 d1 = *(const uint4*)(drow + 16);
    const uint64_t q[4] = {(uint64_t)d0.y << 32 | d0.x, (uint64_t)d0.w << 32 | d0.z,
                           (uint64_t)d1.y << 32 | d1.x, (uint64_t)d1.w << 32 | d1.z};
    const int drop = 8 * ((lane & 31) + 1);  // bits
    uint64_t acc64 = 0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (NA < 8) {
        // a word dropped whole keeps only its bit 63, code bit 7: unused below 8 alphas
        acc64 |= q[t] >> min(max(drop - 64 * t, 0), 63);
      } else {
        const int h = min(max(drop - 64 * t, 0), 64) >> 1;
        acc64 |= (q[t] >> h) >> h;
      }
    }
    uint32_t acc = (uint32_t)acc64 | (uint32_t)(acc64 >> 32);
    if (lane < 32) {
      const uint4 r0 = *(const uint4*)(C + 1024 + 32 * lane);
      const uint4 r1 = *(const uint4*)(C + 1024 + 32 * lane + 16);
      acc |= r0.x | r0.y | r0.z | r0.w | r1.x | r1.y | r1.z | r1.w;
    }
    acc |= acc >> 16;
    acc |= acc >> 8;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) vis[ai] = __ballot((acc >> ai) & 1u) & f.valid_mask;
  }
  // Per chain: rem, the ranks not pruned so far, and cand, the survivors after
  // the last visited row whose rows can prune.  Every rank up to the visited
  // row is decided, and a survivor after the last candidate prunes nothing,
  // so when cand is empty the chain's kept ranks are rem.
  uint64_t rem[NA], cand[NA], kept[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    rem[ai] = f.valid_mask;
    cand[ai] = vis[ai];
  }
  const int lbase = (lane & 31) + 1024 * (lane >> 5);
  // Chain k visits its first candidate i, keeps it with the survivors before
  // it (none of those prunes anything) and removes what row i prunes; the
  // chain stops at its largest R (trimmed below).  Chains with larger alpha
  // prune less and visit fewer rows, so phase s advances chains 0..s while
  // chain s (the largest alpha still running) has a candidate; a finished
  // chain repeats harmless empty steps.  The loops test at the bottom, so the
  // masks stay in place across steps.
#pragma unroll
  for (int s0 = NA - 1; s0 >= 0; --s0) {
    if (uniform_u64(cand[s0]) == 0) continue;
    do {
      uint32_t row[NA];
      uint64_t above[NA];
#pragma unroll
      for (int ai = 0; ai <= s0; ++ai) {
        int i;
        const uint64_t c = uniform_u64(cand[ai]);
        asm("s_ff1_i32_b64 %0, %1" : "=s"(i) : "s"(c));
        // ranks after i; with no candidate (i = -1, shift 63) none
        above[ai] = 0xFFFFFFFFFFFFFFFEull << (i & 63);
        row[ai] = C[(i & 63) * 32 + lbase];
      }
#pragma unroll
      for (int ai = 0; ai <= s0; ++ai) {
        const uint64_t b = __ballot(row[ai] >= (1u << ai));
        uint64_t ab = above[ai];
        uint64_t r = uniform_u64(rem[ai]) & ~(b & ab);
        if (CAP && __popcll(r & ~ab) >= rmax[ai]) {  // R kept up to i: stop
          r &= ~ab;
          ab = 0;
        }
        rem[ai] = r;
        cand[ai] = r & ab & vis[ai];
      }
    } while (uniform_u64(cand[s0]) != 0);
  }
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) kept[ai] = rem[ai];
  // a chain that reached its R keeps its first R ranks
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    const uint64_t k = kept[ai];
    if (CAP && __popcll(k) > rmax[ai]) {
      const int before = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(k >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)k, 0u));
      kept[ai] = __ballot(((k >> lane) & 1ull) && before < rmax[ai]);
    }
  }

  // ---- a8: write every output -------------------------------------------
  // One store per output row: a kept rank goes to its position (the kept
  // ranks before it), every other lane, in lane order, to the next -1 slot
  // after the kept ones (there are enough of them for the first 64 slots).
  auto write_out = [&](const SweepOut& out, int ai) {
    const uint64_t km = kept[ai];
    const int tot = __popcll(km);
    const bool mine = (km >> lane) & 1ull;
    const int before = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(km >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
    const int R = out.R;
    const int cntR = tot < R ? tot : R;
    int32_t* orow = out.nbr + p * R;
    const int pos = mine ? before : cntR + (lane - before);
    if (pos < R) orow[pos] = mine ? f.id_rank : -1;
    if (R > 64) {
      for (int t = 64 + lane; t < R; t += 64) orow[t] = -1;
    }
    if (lane == 0) out.deg[p] = cntR;
  };
  if (NR == 1) {  // one bound per alpha: fixed argument offsets, loaded together
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) write_out(a.out[ai], ai);
  } else {
#pragma unroll
    for (int ai = 0; ai < NA; ++ai)
      for (int ir = 0; ir < NR; ++ir) write_out(a.out[ai * NR + ir], ai);
  }
}

// One wavefront per vertex (any d multiple of 16 up to 32 NK), blockDim.x / 64
// vertices per workgroup, each wavefront with its own `wave_lds` bytes of LDS.
template <int NA, bool CAP, int NK>
__global__ __launch_bounds__(512) void prune_u8_kernel(GraphView g, SweepArgs a, int32_t idbits,
                                                       int32_t nr_out, int32_t wave_lds) {
  extern __shared__ __align__(16) uint8_t lds_all[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar vertex index
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (p >= g.n) return;
  uint8_t* lds = lds_all + (size_t)wave * wave_lds;
  uint8_t* C = lds;                                 // decision tile
  int32_t* nr = (int32_t*)(lds + kDecisionBytes);  // -16 |u|^2 by rank
  const Front f = node_front<NA, NK>(C, nr, g, a, p, lane, idbits);
  wave_sync();  // the decision tile is visible
  node_back<NA, CAP>(C, a, p, f, lane, nr_out);
}

struct Launch {
  int idbits;
  int wave_lds;  // LDS bytes per wavefront
  int waves;     // vertices per workgroup
};

template <int NA, int NK>
hipError_t launch_nk(const GraphView& g, const SweepArgs& a, const Launch& L, hipStream_t s) {
  bool cap = false;
  for (int o = 0; o < a.n_out; ++o) cap = cap || a.out[o].R < g.r_max;
  const int nr_out = a.n_out / NA;
  const dim3 grid((unsigned)((g.n + L.waves - 1) / L.waves)), block(64 * L.waves);
  const size_t shmem = (size_t)L.wave_lds * L.waves;
  if (cap)
    hipLaunchKernelGGL((prune_u8_kernel<NA, true, NK>), grid, block, shmem, s, g, a, L.idbits,
                       nr_out, L.wave_lds);
  else
    hipLaunchKernelGGL((prune_u8_kernel<NA, false, NK>), grid, block, shmem, s, g, a, L.idbits,
                       nr_out, L.wave_lds);
  return hipGetLastError();
}

template <int NA>
hipError_t launch_na(const GraphView& g, const SweepArgs& a, const Launch& L, hipStream_t s) {
  if (a.n_out % NA != 0 || a.n_out / NA > kMaxRs) return hipErrorInvalidValue;
  return g.d <= 128 ? launch_nk<NA, 4>(g, a, L, s) : launch_nk<NA, 8>(g, a, L, s);
}

}  // namespace

int prune_u8_wave_lds(const GraphView&) { return kWaveLdsU8; }

// 16-byte row slices need d % 16 == 0 and a 16-byte aligned point array.
bool prune_u8_supported(const GraphView& g) {
  return g.dtype == RP_U8 && g.r_max <= 64 && (g.d % 16) == 0 && g.d <= kMaxDimU8 &&
         g.n <= (1ll << 30) && (((uintptr_t)g.X) & 15) == 0;
}

// The kernels take the alphas in ascending order (num_a^2 den_b^2 against
// num_b^2 den_a^2), each with its reciprocal-multiply threshold constant; the
// outputs move with their alphas (outputs are alpha-major: o = alpha * nr + iR).
SweepArgs u8_sweep_ascending(const SweepArgs& a_in) {
  SweepArgs a = a_in;
  int order[kMaxAlphas];
  for (int i = 0; i < a_in.n_alpha; ++i) order[i] = i;
  for (int i = 1; i < a_in.n_alpha; ++i) {
    int v = order[i], j = i - 1;
    while (j >= 0 && (uint64_t)a_in.num2[v] * a_in.den2[order[j]] <
                         (uint64_t)a_in.num2[order[j]] * a_in.den2[v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  const int nr = a_in.n_out / a_in.n_alpha;
  for (int k = 0; k < a_in.n_alpha; ++k) {
    a.num2[k] = a_in.num2[order[k]];
    a.den2[k] = a_in.den2[order[k]];
    a.ratio[k] = a_in.ratio[order[k]];
    a.thr_mul[k] = (uint64_t)((((unsigned __int128)a.den2[k]) << 60) / a.num2[k]) + 1u;
    for (int ir = 0; ir < nr; ++ir) {
      a.out[k * nr + ir] = a_in.out[order[k] * nr + ir];
      a.out[k * nr + ir].alpha_idx = k;
    }
  }
  return a;
}

hipError_t launch_prune_u8(const GraphView& g, const SweepArgs& a_in, DevCounters* ctr,
                           hipStream_t s) {
  (void)ctr;
  const SweepArgs a = u8_sweep_ascending(a_in);
  int idbits = 1;
  while ((1ll << idbits) < g.n) ++idbits;
  Launch L;
  L.idbits = idbits;
  L.wave_lds = prune_u8_wave_lds(g);
  L.waves = waves_for(TuneKey{kKernelU8, g.dtype, g.d, g.r_max, a.n_alpha, a.n_out}, L.wave_lds);
  switch (a.n_alpha) {
    case 1: return launch_na<1>(g, a, L, s);
    case 2: return launch_na<2>(g, a, L, s);
    case 3: return launch_na<3>(g, a, L, s);
    case 4: return launch_na<4>(g, a, L, s);
    case 5: return launch_na<5>(g, a, L, s);
    case 6: return launch_na<6>(g, a, L, s);
    case 7: return launch_na<7>(g, a, L, s);
    case 8: return launch_na<8>(g, a, L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace rp
