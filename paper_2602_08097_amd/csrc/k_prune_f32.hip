// k_prune_f32.hip -- batched RP-Tuning for float32 points: rows streamed
// straight into FP16 matrix-unit registers, a proven rounding band, and a
// canonical FP64 recheck of the pairs inside it.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep, reading each candidate row once, for
// out-lists of up to 32 NB ids (NB = 2 or 3 row blocks) and any d:
//
//  a1  read:   the t-th listed id is slot t (lane t, and lane t - 64 of the
//              second word for t >= 64); p itself and -1 padding are empty.
//  a2  gather: 16 dimensions per step, straight from global memory into the
//              operand layout of the matrix instruction: for row block b
//              (slots 32 b .. 32 b + 31) lane l holds dimensions
//              16 s + 8 (l / 32) .. + 7 of row 32 b + l % 32, several steps in
//              flight.  x_p sits in LDS.
//  a3  p-row:  one lane swap (lanes 32..63 of block 0 with lanes 0..31 of
//              block 1) gives lane t all 16 dimensions of slot t's row (block 2
//              swaps with itself), and the lane accumulates the canonical FP64
//              S(p, t): t = (double)a - (double)b, fused multiply-add, k
//              ascending.
//  a4  sort:   (S(p, j), id) ascending -- the order in which the repeated
//              argmin of Algorithm 1 visits the candidates (UnsortedRobustPrune,
//              Section 3, keeps the list order instead).  A list already in
//              that order (every RobustPrune output is) is used as read;
//              otherwise the keys are sorted and the rows are streamed a
//              second time in rank order.  Repeated ids are dropped.
//  a5  Gram:   in the frame centred on p and scaled by 2^e (every scaled
//              difference below 2^14; e of each vertex is computed with the
//              graph from the max |x_k| of the vertex and its list), each
//              FP32 difference is split as hi + lo, two FP16 values, and
//              G~ = sum hi hi' + hi lo' + lo hi' runs on
//              v_mfma_f32_32x32x16_f16; for long rows the accumulator restarts
//              every 128 dimensions and the pieces are summed in FP32 in LDS.
//              S~(i, j) = (S(p, i) + S(p, j)) 2^2e - 2 G~(i, j) goes to an
//              FP32 tile of the blocks on and above the diagonal, by rank
//              (entries with j <= i hold +inf).
//  a6  test:   fl(num^2 S(i, j)) <= fl(den^2 S(p, j)) is decided from S~
//              outside [P_j, K_j], thresholds that carry the proven bound
//              |S~ - S(i, j) 2^2e| <= c1 s + c2 sqrt(s) + c3 (s = S(p, j) 2^2e)
//              and the FP64 rounding of both products; pairs inside are
//              recomputed in canonical FP64 from the rows.
//  a7  greedy: per alpha a survivor mask over the ranks.  A row-minimum scan
//              marks the rows that can prune at each alpha; survivors whose
//              row cannot are kept in runs (one shift mask per step), each
//              survivor whose row can prune is kept and one ballot over its
//              tile row removes what it prunes.  A chain stops at its largest R.
//  a8  write:  kept ranks are scattered to their positions, -1 padded.
#include <math.h>

#include <cmath>
#include <type_traits>

#include "dev_common.h"

namespace rp {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

namespace {

constexpr int kDC = 64;  // dimensions per accumulator chunk of the Gram (long rows)
constexpr int kMaxDimF32 = 4096;

template <int NB>
struct Shape {
  static constexpr int MS = 32 * NB;            // candidate slots
  static constexpr int NW = NB > 2 ? 2 : 1;     // 64-bit words of a rank mask
  static constexpr int NP = NB * (NB + 1) / 2;  // 32 x 32 blocks on and above the diagonal
  static constexpr int TILE = 1024 * NP;        // S~ entries
};

// S~ tile: column block cb holds rows 0 .. 32 cb + 31; entry (i, j) sits at
// cb_base(j / 32) + 32 i + j % 32.
__host__ __device__ constexpr int cb_base(int cb) { return 512 * cb * (cb + 1); }
// accumulator of block (bi, bj), bi <= bj
__host__ __device__ constexpr int blk(int bi, int bj) { return bj * (bj + 1) / 2 + bi; }

__host__ __device__ inline int xp_floats(int d) { return (d + 15) & ~15; }

// LDS of one wavefront: the S~ tile; x_p as FP64 (the canonical p-row's
// operand); and one FP32 region that holds x_p 2^e while the rows stream,
// then S(p, .) 2^2e by rank until the tile is written, then 1 / S(p, .) 2^2e
// by rank.  x_p arrays are zero padded to a multiple of 16 values.
__host__ __device__ inline int aux_floats(int d, int nw) {
  return xp_floats(d) > 64 * nw ? xp_floats(d) : 64 * nw;
}

template <int NB>
inline int wave_lds_bytes(int d) {
  return Shape<NB>::TILE * 4 + xp_floats(d) * 8 + aux_floats(d, Shape<NB>::NW) * 4;
}

struct F32Args {
  double c1, c2, c3;  // rounding band of S~ (scaled units)
  int32_t nr;         // outputs per alpha (outputs are alpha-major)
  // measurement mode: only the listed vertices, S~ compared with canonical FP64
  const int32_t* nodes;
  int64_t n_nodes;
  GramErrorStats* stats;
};

// Next float toward +inf (finite inputs).
__device__ __forceinline__ float next_up(float f) {
  if (f == 0.f) return 1.401298464e-45f;
  const int b = __float_as_int(f);
  return __int_as_float(f > 0.f ? b + 1 : b - 1);
}

// FP32 value >= x (round up).
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
#pragma unroll 4
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

// The same value computed by a whole wavefront, for one pair: the
// differences t_k = (double)a_k - (double)b_k of up to 1,024 dimensions are
// requested at once (coalesced) and staged in buf (LDS, >= d doubles, 16-byte
// aligned), then every lane sums t_k^2 in order k = 0 .. d - 1 from the
// broadcast reads, so the result is uniform and equal to canon_rows.  One
// memory round trip per 1,024 dimensions instead of one per 4 (a lane's own
// loop waits for each load before its fused multiply-add).
template <bool VEC>
__device__ __forceinline__ double canon_rows_wave(const float* __restrict__ a,
                                                  const float* __restrict__ b, int d,
                                                  double* buf, int lane) {
  if (VEC) {
    for (int k0 = 0; k0 < d; k0 += 1024) {
      float4 va[4], vb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 256 * u + 4 * lane;
        if (k < d) {
          va[u] = *(const float4*)(a + k);
          vb[u] = *(const float4*)(b + k);
        }
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int k = k0 + 256 * u + 4 * lane;
        if (k < d) {
          *(double2*)(buf + k) =
              make_double2((double)va[u].x - (double)vb[u].x, (double)va[u].y - (double)vb[u].y);
          *(double2*)(buf + k + 2) =
              make_double2((double)va[u].z - (double)vb[u].z, (double)va[u].w - (double)vb[u].w);
        }
      }
    }
  } else {
    for (int k0 = 0; k0 < d; k0 += 512) {
      float va[8], vb[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + 64 * u + lane;
        if (k < d) {
          va[u] = a[k];
          vb[u] = b[k];
        }
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int k = k0 + 64 * u + lane;
        if (k < d) buf[k] = (double)va[u] - (double)vb[u];
      }
    }
  }
  wave_sync();
  double acc = 0.0;
  int k = 0;
#pragma unroll 8
  for (; k + 2 <= d; k += 2) {
    const double2 t = *(const double2*)(buf + k);
    acc = __fma_rn(t.x, t.x, acc);
    acc = __fma_rn(t.y, t.y, acc);
  }
  if (k < d) {
    const double t = buf[k];
    acc = __fma_rn(t, t, acc);
  }
  wave_sync();  // every read is done before buf is written again
  return acc;
}

// Pairs of one ambiguous step that the wavefront rechecks one at a time
// (more go lane-parallel, one pair per lane).
constexpr int kWaveRechecks = 8;

__device__ __forceinline__ double readlane_f64(double v, int l) {
  const uint64_t u = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readlane((uint32_t)u, l);
  const uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(u >> 32), l);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
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

// Sort of up to 128 (hi, lo) keys held two per lane (a: ranks 0..63 after the
// call, b: ranks 64..127): each half is sorted, b is reversed so a ++ b is
// bitonic, a half-cleaner splits the 64 smallest from the rest, and each half
// is merged.
__device__ __forceinline__ void wave_sort128(uint64_t& ah, uint32_t& al, uint64_t& bh,
                                             uint32_t& bl, int lane) {
  wave_sort2(ah, al, lane);
  wave_sort2(bh, bl, lane);
  const uint64_t rh = shfl_u64(bh, 63 - lane);
  const uint32_t rl = (uint32_t)__shfl((int)bl, 63 - lane, 64);
  if (key_less(rh, rl, ah, al)) {
    bh = ah;
    bl = al;
    ah = rh;
    al = rl;
  } else {
    bh = rh;
    bl = rl;
  }
  bitonic_step2<64, 32>(ah, al, lane);
  bitonic_step2<64, 16>(ah, al, lane);
  bitonic_step2<64, 8>(ah, al, lane);
  bitonic_step2<64, 4>(ah, al, lane);
  bitonic_step2<64, 2>(ah, al, lane);
  bitonic_step2<64, 1>(ah, al, lane);
  bitonic_step2<64, 32>(bh, bl, lane);
  bitonic_step2<64, 16>(bh, bl, lane);
  bitonic_step2<64, 8>(bh, bl, lane);
  bitonic_step2<64, 4>(bh, bl, lane);
  bitonic_step2<64, 2>(bh, bl, lane);
  bitonic_step2<64, 1>(bh, bl, lane);
}

// u = x 2^e - x_p 2^e in one rounding (the scaled difference; x_p 2^e comes
// from LDS), hi = fp16(u), lo = fp16(u - hi), where u - hi is exact in FP32
// and formed by one mixed-precision fused multiply-add.
__device__ __forceinline__ void split8(const float (&x)[8], const float4& p0, const float4& p1,
                                       float scf, v8h& hi, v8h& lo) {
  float u[8];
  u[0] = __builtin_fmaf(x[0], scf, -p0.x);
  u[1] = __builtin_fmaf(x[1], scf, -p0.y);
  u[2] = __builtin_fmaf(x[2], scf, -p0.z);
  u[3] = __builtin_fmaf(x[3], scf, -p0.w);
  u[4] = __builtin_fmaf(x[4], scf, -p1.x);
  u[5] = __builtin_fmaf(x[5], scf, -p1.y);
  u[6] = __builtin_fmaf(x[6], scf, -p1.z);
  u[7] = __builtin_fmaf(x[7], scf, -p1.w);
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const _Float16 h = (_Float16)u[i];
    hi[i] = h;
    lo[i] = (_Float16)__builtin_fmaf((float)h, -1.f, u[i]);
  }
}

// C += A B^T over one 16-dimension step in three products: hi hi', hi lo', lo hi'
// (FRESH: C = A B^T, the first step of an accumulator chunk).
template <bool FRESH = false>
__device__ __forceinline__ void gram3(v16f& c, const v8h& ah, const v8h& al, const v8h& bh,
                                      const v8h& bl) {
  if constexpr (FRESH) {
    const v16f z = {};
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, z, 0, 0, 0);
  } else {
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, c, 0, 0, 0);
  }
  c = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, c, 0, 0, 0);
}

// Lanes 32..63 of a and lanes 0..31 of b trade places: afterwards `lo` holds
// the first and `hi` the second 8 of the 16 dimensions of one row.  With a =
// block 0 and b = block 1 that row is block 0's row l for lanes l < 32 and
// block 1's row l - 32 for lanes l >= 32; with a = b = block 2 it is block 2's
// row l % 32 in both halves.
__device__ __forceinline__ void swap_halves(float a, float b, float& lo, float& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}

// acc + the canonical terms of one row's 16 dimensions of a step (xq: x_p's,
// already FP64).
__device__ __forceinline__ double row_step(double acc, const float (&a)[8], const float (&b)[8],
                                           const double* __restrict__ xq) {
  float lo[8], hi[8];
#pragma unroll
  for (int e = 0; e < 8; ++e) swap_halves(a[e], b[e], lo[e], hi[e]);
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const double2 q = *(const double2*)(xq + e);
    double t = (double)lo[e] - q.x;
    acc = __fma_rn(t, t, acc);
    t = (double)lo[e + 1] - q.y;
    acc = __fma_rn(t, t, acc);
  }
#pragma unroll
  for (int e = 0; e < 8; e += 2) {
    const double2 q = *(const double2*)(xq + 8 + e);
    double t = (double)hi[e] - q.x;
    acc = __fma_rn(t, t, acc);
    t = (double)hi[e + 1] - q.y;
    acc = __fma_rn(t, t, acc);
  }
  return acc;
}

// The 8 dimensions 16 s + 8 half .. + 7 of one row block per lane.
template <int NB>
struct Step {
  float x[NB][8];
};

// Every load reads valid memory: slices past d read the row's first values
// and are zeroed before use.
template <int NB, bool VEC>
__device__ __forceinline__ Step<NB> fetch_step(const float* const (&rows)[NB], int d, int s,
                                               int half) {
  Step<NB> q;
  const int o0 = 16 * s + 8 * half;
  if (VEC) {
    const int c0 = o0 < d ? o0 : 0;
    const int c1 = o0 + 4 < d ? o0 + 4 : 0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const float4 v0 = *(const float4*)(rows[b] + c0);
      const float4 v1 = *(const float4*)(rows[b] + c1);
      q.x[b][0] = v0.x;
      q.x[b][1] = v0.y;
      q.x[b][2] = v0.z;
      q.x[b][3] = v0.w;
      q.x[b][4] = v1.x;
      q.x[b][5] = v1.y;
      q.x[b][6] = v1.z;
      q.x[b][7] = v1.w;
    }
  } else {
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int e = 0; e < 8; ++e) q.x[b][e] = rows[b][o0 + e < d ? o0 + e : 0];
    }
  }
  return q;
}

// The first PF steps of a pass, requested ahead of it (named buffers, so
// nothing is indexed at run time).
template <int NB>
struct Ring {
  Step<NB> a, b, c, d;
};

template <int NB, bool VEC, int PF>
__device__ __forceinline__ void ring_fill(Ring<NB>& r, const float* const (&rows)[NB], int d,
                                          int half) {
  r.a = fetch_step<NB, VEC>(rows, d, 0, half);
  r.b = fetch_step<NB, VEC>(rows, d, 1, half);
  if (PF > 2) r.c = fetch_step<NB, VEC>(rows, d, 2, half);
  if (PF > 3) r.d = fetch_step<NB, VEC>(rows, d, 3, half);
}

// Chunk sums of the Gram accumulators (CSUM) live in LDS, in the region the
// S~ tile takes afterwards: block c's 16 values of lane l sit at
// acc + 1024 c + 256 q + 4 l + (v % 4) for v = 4 q + (v % 4), so every access
// is a 16-byte vector load or store of consecutive lanes.  Each word has one
// owner lane.  Block (i, j) is in use when row block j holds listed slots
// (nbu > j): c = blk(i, j) is below 1, 3, 6, 10 for j = 0, 1, 2, 3.
template <int NB>
__device__ __forceinline__ bool block_in_use(int c, int nbu) {
  return c == 0 || (c < 3 ? nbu > 1 : c < 6 ? nbu > 2 : nbu > 3);
}

// acc += cur, then (ZERO) cur = 0 for the next chunk; without ZERO the next
// chunk's first products start from zero instead.
template <int NB, bool ZERO = true>
__device__ __forceinline__ void chunk_flush(v16f (&cur)[Shape<NB>::NP], float* acc, int lane,
                                            int nbu) {
  constexpr int NP = Shape<NB>::NP;
#pragma unroll
  for (int c = 0; c < NP; ++c) {
    if (!block_in_use<NB>(c, nbu)) continue;  // uniform
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      float4* a = (float4*)(acc + 1024 * c + 256 * q + 4 * lane);
      float4 t = *a;
      t.x += cur[c][4 * q];
      t.y += cur[c][4 * q + 1];
      t.z += cur[c][4 * q + 2];
      t.w += cur[c][4 * q + 3];
      *a = t;
    }
    if (ZERO) {
#pragma unroll
      for (int v = 0; v < 16; ++v) cur[c][v] = 0.f;
    }
  }
}

template <int NB>
__device__ __forceinline__ void chunk_zero(float* acc, int lane) {
#pragma unroll
  for (int c = 0; c < Shape<NB>::NP; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
      *(float4*)(acc + 1024 * c + 256 * q + 4 * lane) = make_float4(0.f, 0.f, 0.f, 0.f);
  }
}

// The chunk sums back into the accumulator registers (after the last flush).
template <int NB>
__device__ __forceinline__ void chunk_load(v16f (&cur)[Shape<NB>::NP], const float* acc,
                                           int lane) {
#pragma unroll
  for (int c = 0; c < Shape<NB>::NP; ++c) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float4 t = *(const float4*)(acc + 1024 * c + 256 * q + 4 * lane);
      cur[c][4 * q] = t.x;
      cur[c][4 * q + 1] = t.y;
      cur[c][4 * q + 2] = t.z;
      cur[c][4 * q + 3] = t.w;
    }
  }
}

// One pass over this lane's rows (rows[b]: block b's row l % 32) whose first
// PF steps are in `ring`: the Gram blocks into cur (chunk sums into acc with
// CSUM) and, with PROW, the canonical S(p, .) of slot lane (sp[0], rows of
// blocks 0 and 1) and of slot 64 + lane (sp[1], rows of blocks 2 and 3; with
// three blocks lanes 32..63 repeat block 2).  nbu: blocks in use.
template <int NB, bool CSUM, bool PROW, bool VEC, int PF>
__device__ __forceinline__ void gram_pass(Ring<NB>& ring, const float* const (&rows)[NB], int d,
                                          int nbu, const double* __restrict__ xq,
                                          const float* __restrict__ xs, float scf,
                                          int half, v16f (&cur)[Shape<NB>::NP],
                                          float* acc, int lane, double (&sp)[Shape<NB>::NW]) {
  static_assert(PF >= 2 && PF <= 4, "two to four steps in flight");
  const int nsteps = (d + 15) >> 4;
  const bool ragged = (d & 15) != 0;
  constexpr int kChunkSteps = kDC / 16;
  // chunks of PF steps start at the first step of each round of the ring, so
  // that step's products can start from zero (no accumulator clearing) and
  // the last step of the round ends the chunk
  constexpr bool kFreshStart = CSUM && kChunkSteps == PF;
  auto step = [&](const Step<NB>& q, int s, auto pos_c) {
    constexpr int POS = decltype(pos_c)::value;  // position in the round of the ring
    constexpr bool F = kFreshStart && POS == 0;
    const int o0 = 16 * s + 8 * half;
    float x[NB][8];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
#pragma unroll
      for (int e = 0; e < 8; ++e) x[b][e] = q.x[b][e];
    }
    if (ragged && s == nsteps - 1) {
#pragma unroll
      for (int b = 0; b < NB; ++b) {
#pragma unroll
        for (int e = 0; e < 8; ++e) x[b][e] = o0 + e < d ? x[b][e] : 0.f;
      }
    }
    const float4 p0 = *(const float4*)(xs + o0);
    const float4 p1 = *(const float4*)(xs + o0 + 4);
    v8h hi[NB], lo[NB];
    split8(x[0], p0, p1, scf, hi[0], lo[0]);
    gram3<F>(cur[blk(0, 0)], hi[0], lo[0], hi[0], lo[0]);
    if (nbu > 1) {
      split8(x[1], p0, p1, scf, hi[1], lo[1]);
      gram3<F>(cur[blk(0, 1)], hi[0], lo[0], hi[1], lo[1]);
      gram3<F>(cur[blk(1, 1)], hi[1], lo[1], hi[1], lo[1]);
    }
    if constexpr (NB > 2) {
      if (nbu > 2) {
        split8(x[2], p0, p1, scf, hi[2], lo[2]);
        gram3<F>(cur[blk(0, 2)], hi[0], lo[0], hi[2], lo[2]);
        gram3<F>(cur[blk(1, 2)], hi[1], lo[1], hi[2], lo[2]);
        gram3<F>(cur[blk(2, 2)], hi[2], lo[2], hi[2], lo[2]);
      }
    }
    if constexpr (NB > 3) {
      if (nbu > 3) {
        split8(x[3], p0, p1, scf, hi[3], lo[3]);
        gram3<F>(cur[blk(0, 3)], hi[0], lo[0], hi[3], lo[3]);
        gram3<F>(cur[blk(1, 3)], hi[1], lo[1], hi[3], lo[3]);
        gram3<F>(cur[blk(2, 3)], hi[2], lo[2], hi[3], lo[3]);
        gram3<F>(cur[blk(3, 3)], hi[3], lo[3], hi[3], lo[3]);
      }
    }
    // a fresh accumulator every kDC dimensions
    const bool chunk_end = kFreshStart ? POS == PF - 1 : (s % kChunkSteps) == kChunkSteps - 1;
    if (CSUM && (chunk_end || s == nsteps - 1))
      chunk_flush<NB, !kFreshStart>(cur, acc, lane, nbu);
    if (PROW) {
      sp[0] = row_step(sp[0], x[0], x[1], xq + 16 * s);
      if constexpr (NB > 2) {
        if (nbu > 2) sp[1] = row_step(sp[1], x[2], x[NB > 3 ? 3 : 2], xq + 16 * s);
      }
    }
  };
  // PF buffers in rotation, held as values (the slices of step s + PF are
  // requested before step s is used)
  Step<NB>& qa = ring.a;
  Step<NB>& qb = ring.b;
  Step<NB>& qc = ring.c;
  Step<NB>& qd = ring.d;
  for (int s = 0; s < nsteps; s += PF) {
    {
      const Step<NB> c = qa;
      if (s + PF < nsteps) qa = fetch_step<NB, VEC>(rows, d, s + PF, half);
      step(c, s, std::integral_constant<int, 0>{});
    }
    if (s + 1 < nsteps) {
      const Step<NB> c = qb;
      if (s + 1 + PF < nsteps) qb = fetch_step<NB, VEC>(rows, d, s + 1 + PF, half);
      step(c, s + 1, std::integral_constant<int, 1>{});
    }
    if (PF > 2 && s + 2 < nsteps) {
      const Step<NB> c = qc;
      if (s + 2 + PF < nsteps) qc = fetch_step<NB, VEC>(rows, d, s + 2 + PF, half);
      step(c, s + 2, std::integral_constant<int, 2>{});
    }
    if (PF > 3 && s + 3 < nsteps) {
      const Step<NB> c = qd;
      if (s + 3 + PF < nsteps) qd = fetch_step<NB, VEC>(rows, d, s + 3 + PF, half);
      step(c, s + 3, std::integral_constant<int, 3>{});
    }
  }
}

// S~ of one 32 x 32 block (rows of block BI, columns of block BJ) into the
// tile.  Accumulator layout: lane l holds column l % 32 of rows
// 8 (v / 4) + 4 (l / 32) + v % 4 in register v.
template <int BI, int BJ>
__device__ __forceinline__ void store_block(float* St, const float* sr, const v16f& acc, int l32,
                                            int half) {
  const float scol = sr[32 * BJ + l32];
  float4 nrow[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) nrow[q] = *(const float4*)(sr + 32 * BI + 8 * q + 4 * half);
  float* base = St + cb_base(BJ) + 1024 * BI + 128 * half + l32;
  const int below = l32 - 4 * half;  // column after row  <=>  below > 8 q + j
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int rr = 8 * (v >> 2) + (v & 3);
    const float4 nq = nrow[v >> 2];
    const float srow = (v & 3) == 0 ? nq.x : (v & 3) == 1 ? nq.y : (v & 3) == 2 ? nq.z : nq.w;
    const float val = __builtin_fmaf(-2.f, acc[v], srow + scol);  // 2 acc is exact
    base[32 * rr] = (BI != BJ || below > rr) ? val : __builtin_inff();
  }
}

// Minimum over the 32 columns of block cb of tile row i of S~(i, j) / S(p, j)
// (reciprocals by rank in invt; NaN for empty ranks, which fminf ignores).
__device__ __forceinline__ float row_zmin(const float* St, const float* invt, int cb, int i,
                                          float z) {
  const float* row = St + cb_base(cb) + 32 * i;
#pragma unroll
  for (int c0 = 0; c0 < 32; c0 += 4) {
    const float4 v = *(const float4*)(row + c0);
    const float4 iv = *(const float4*)(invt + 32 * cb + c0);
    z = fminf(z, fminf(fminf(v.x * iv.x, v.y * iv.y), fminf(v.z * iv.z, v.w * iv.w)));
  }
  return z;
}

// DIAG: measure instead of prune -- for the listed vertices, every candidate
// pair's S~ is compared with the canonical FP64 S(i, j) (relative error, and
// error over the proven band), and nothing is written.
// Workgroups of up to 8 wavefronts for 64 candidates, 4 for 96 (whose
// registers take a whole SIMD lane file); one vertex per wavefront.
template <int NA, int NB, bool CSUM, bool VEC, int PF, bool CAP, bool DIAG>
__global__ __launch_bounds__(NB >= 3 ? 256 : 512) void prune_f32_kernel(GraphView g, SweepArgs a, F32Args fa,
                                                        DevCounters* ctr, int32_t wave_lds) {
  using SH = Shape<NB>;
  constexpr int NW = SH::NW;
  constexpr int NP = SH::NP;
  constexpr int SB = NW == 2 ? 7 : 6;  // slot bits of a sort key
  extern __shared__ __align__(16) uint8_t lds_all[];
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // uniform: scalar vertex index
  int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (DIAG) {
    if (p >= fa.n_nodes) return;
    p = fa.nodes[p];
  }
  if (p >= g.n) return;
  uint8_t* lds = lds_all + (size_t)wave * wave_lds;
  float* St = (float*)lds;          // S~ tile
  double* xq = (double*)(St + SH::TILE);  // x_p in FP64, zero padded
  float* xs = (float*)(xq + xp_floats(g.d));  // x_p 2^e while the rows stream,
  float* sr = xs;                              // then S(p, .) 2^2e by rank,
  float* invt = xs;                            // then its reciprocal
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int d = g.d;
  const float* X = (const float*)g.X;
  const int xpf = xp_floats(d);

  // ---- a1: the list of vertex q (ids by slot, degree) -----------------------
  auto load_list = [&](int64_t q, int (&raw)[NW], int& mq) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int s = lane + 64 * w;
      raw[w] = s < g.r_max && s < SH::MS ? g.nbr[q * g.r_max + s] : -1;
    }
    mq = g.deg[q];
  };
  // usable ids by slot; the rows of the first NL row blocks of this lane
  int idw[NW];
  int fe = 0;
  float4 xv;
  auto usable_ids = [&](int64_t q, const int (&raw)[NW], int mq) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int s = lane + 64 * w;
      idw[w] = (s < mq && raw[w] != (int)q) ? raw[w] : -1;
    }
  };
  auto rows_of = [&](const int (&ids)[NW], auto& rows) {
    constexpr int NL = sizeof(rows) / sizeof(rows[0]);
#pragma unroll
    for (int b = 0; b < NL; ++b) {
      const int id = __shfl(ids[b >> 1], 32 * (b & 1) + l32, 64);
      rows[b] = X + (int64_t)(id >= 0 ? id : (int)p) * d;
    }
  };
  // loads that do not wait for the list: x_p and the vertex's frame exponent
  // (computed with the graph from its list and the per-point max |x_k|)
  auto early = [&](int64_t q) {
    fe = g.frame_e[q];
    const float* xrow = X + q * d;
    xv = make_float4(0.f, 0.f, 0.f, 0.f);
    if (VEC) {
      if (4 * lane < d) xv = *(const float4*)(xrow + 4 * lane);
    } else {
      const int c = 4 * lane;
      xv.x = c < d ? xrow[c] : 0.f;
      xv.y = c + 1 < d ? xrow[c + 1] : 0.f;
      xv.z = c + 2 < d ? xrow[c + 2] : 0.f;
      xv.w = c + 3 < d ? xrow[c + 3] : 0.f;
    }
  };

  int m, raw[NW];
  load_list(p, raw, m);
  early(p);
  usable_ids(p, raw, m);
  unsigned long long rechecks = 0;
  double dg_max_rel = 0.0, dg_sum_rel = 0.0, dg_max_band = 0.0;
  unsigned long long dg_pairs = 0;
  const int nbu = max(1, min(NB, (m + 31) >> 5));  // uniform: blocks holding listed slots

  const int e = fe;
  const float scf = ldexpf(1.f, e);
  const double sc = ldexp(1.0, e);
  const double sc2 = sc * sc;
  // x_p and x_p 2^e (a power-of-two scale: exact unless it leaves the
  // normal range, where the error stays far below the subnormal term)
  auto stage = [&](int c, float4 v) {
    *(double2*)(xq + c) = make_double2((double)v.x, (double)v.y);
    *(double2*)(xq + c + 2) = make_double2((double)v.z, (double)v.w);
    *(float4*)(xs + c) = make_float4(v.x * scf, v.y * scf, v.z * scf, v.w * scf);
  };
  {
    if (4 * lane < xpf) stage(4 * lane, xv);
    for (int c = 4 * lane + 256; c < xpf; c += 256) {  // long rows
      const float* xrow = X + p * d;
      float4 v;
      v.x = c < d ? xrow[c] : 0.f;
      v.y = c + 1 < d ? xrow[c + 1] : 0.f;
      v.z = c + 2 < d ? xrow[c + 2] : 0.f;
      v.w = c + 3 < d ? xrow[c + 3] : 0.f;
      stage(c, v);
    }
  }
  wave_sync();

  // ---- a2 + a3 + a5: one pass over the rows in slot order ----------------
  v16f cur[NP];
#pragma unroll
  for (int c = 0; c < NP; ++c) {
#pragma unroll
    for (int v = 0; v < 16; ++v) cur[c][v] = 0.f;
  }
  double sp[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) sp[w] = 0.0;
  // one pass over the rows of `ids` (the tile region holds the chunk sums
  // for now)
  auto pass = [&](const int (&ids)[NW], auto prow_c) {
    constexpr bool PROW = decltype(prow_c)::value;
    const float* rows[NB];
    rows_of(ids, rows);
    Ring<NB> ring;
    ring_fill<NB, VEC, PF>(ring, rows, d, half);
    if (CSUM) chunk_zero<NB>(St, lane);
    gram_pass<NB, CSUM, PROW, VEC, PF>(ring, rows, d, nbu, xq, xs, scf, half, cur, St, lane, sp);
  };
  pass(idw, std::true_type{});

  // ---- a4: sort by (S(p, j), id); drop repeated ids -------------------------
  uint64_t kh[NW];
  uint32_t kl[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    kh[w] = ~0ull;
    kl[w] = ~0u;
    if (idw[w] >= 0) {
      kh[w] = (uint64_t)__double_as_longlong(sp[w]);
      kl[w] = ((uint32_t)idw[w] << SB) | (uint32_t)(lane + 64 * w);
    }
  }
  {
    bool unsorted = false;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint64_t ph = shfl_u64(kh[w], lane > 0 ? lane - 1 : 0);
      const uint32_t pl = (uint32_t)__shfl((int)kl[w], lane > 0 ? lane - 1 : 0, 64);
      unsorted = unsorted || (lane > 0 && key_less(kh[w], kl[w], ph, pl));
    }
    if (NW == 2) {
      const uint64_t lh = shfl_u64(kh[0], 63);
      const uint32_t ll = (uint32_t)__shfl((int)kl[0], 63, 64);
      unsorted = unsorted || (lane == 0 && key_less(kh[NW - 1], kl[NW - 1], lh, ll));
    }
    // out of rank order: sort the keys, stream the rows again by rank
    bool again = false;
    int idk[NW];
    if (!a.unsorted && __ballot(unsorted) != 0) {
      if constexpr (NW == 2) wave_sort128(kh[0], kl[0], kh[1], kl[1], lane);
      else wave_sort2(kh[0], kl[0], lane);
#pragma unroll
      for (int w = 0; w < NW; ++w) idk[w] = kh[w] != ~0ull ? (int)(kl[w] >> SB) : -1;
      again = true;
    }
    if (again) {
#pragma unroll
      for (int c = 0; c < NP; ++c) {
#pragma unroll
        for (int v = 0; v < 16; ++v) cur[c][v] = 0.f;
      }
      pass(idk, std::false_type{});
    }
  }
  wave_sync();  // the x_p 2^e reads are done before the region takes S(p, .)
  bool valid[NW];
  uint64_t vm[NW];
  int id_rank[NW];
  double sw[NW], s2[NW];
  // UnsortedRobustPrune (Section 3): the ranks are the list order, and a
  // repeated id counts at its first slot
  bool later[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) later[w] = false;
  if (a.unsorted) {
#pragma unroll 1
    for (int t = 0; t < 64; ++t) {
      const int v = __builtin_amdgcn_readlane(idw[0], t);
#pragma unroll
      for (int w = 0; w < NW; ++w)
        later[w] = later[w] || (t < lane + 64 * w && v >= 0 && v == idw[w]);
    }
    if constexpr (NW == 2) {
#pragma unroll 1
      for (int t = 0; t < 32; ++t) {
        const int v = __builtin_amdgcn_readlane(idw[1], t);
        later[1] = later[1] || (t < lane && v >= 0 && v == idw[1]);
      }
    }
  }
  {
    const uint64_t last0h = shfl_u64(kh[0], 63);
    const uint32_t last0l = (uint32_t)__shfl((int)kl[0], 63, 64);
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      // previous rank: lane - 1 of this word, or rank 63 for lane 0 of word 1
      uint64_t ph = shfl_u64(kh[w], lane > 0 ? lane - 1 : 0);
      uint32_t pl = (uint32_t)__shfl((int)kl[w], lane > 0 ? lane - 1 : 0, 64);
      if (lane == 0) {
        ph = w == 0 ? ~0ull - 1 : last0h;
        pl = w == 0 ? 0u : last0l;
      }
      valid[w] = kh[w] != ~0ull &&
                 (a.unsorted ? !later[w] : !(kh[w] == ph && (kl[w] >> SB) == (pl >> SB)));
      vm[w] = __ballot(valid[w]);
      id_rank[w] = valid[w] ? (int)(kl[w] >> SB) : -1;
      sw[w] = valid[w] ? __longlong_as_double((long long)kh[w]) : 0.0;
      s2[w] = sw[w] * sc2;
      sr[lane + 64 * w] = valid[w] ? (float)s2[w] : 0.f;
    }
  }
  wave_sync();

  // ---- a5: S~ tile by rank ----------------------------------------------------
  if (CSUM) {
    chunk_load<NB>(cur, St, lane);  // every chunk has been flushed
    wave_sync();                    // all read before the tile is written
  }
  auto acc_of = [&](int c) -> const v16f& { return cur[c]; };
  store_block<0, 0>(St, sr, acc_of(blk(0, 0)), l32, half);
  if (nbu > 1) {
    store_block<0, 1>(St, sr, acc_of(blk(0, 1)), l32, half);
    store_block<1, 1>(St, sr, acc_of(blk(1, 1)), l32, half);
  }
  if constexpr (NB > 2) {
    if (nbu > 2) {
      store_block<0, 2>(St, sr, acc_of(blk(0, 2)), l32, half);
      store_block<1, 2>(St, sr, acc_of(blk(1, 2)), l32, half);
      store_block<2, 2>(St, sr, acc_of(blk(2, 2)), l32, half);
    }
  }
  if constexpr (NB > 3) {
    if (nbu > 3) {
      store_block<0, 3>(St, sr, acc_of(blk(0, 3)), l32, half);
      store_block<1, 3>(St, sr, acc_of(blk(1, 3)), l32, half);
      store_block<2, 3>(St, sr, acc_of(blk(2, 3)), l32, half);
      store_block<3, 3>(St, sr, acc_of(blk(3, 3)), l32, half);
    }
  }
  // tile entry (i, rank of word w of this lane) = St[32 i + lbase[w]] for the
  // rows i the column block holds (i < 32 (cb + 1)); with three blocks the
  // second word's lanes 32..63 (ranks past 95, never alive) read in bounds
  int lbase[NW];
  lbase[0] = l32 + 1024 * half;
  if (NW == 2) lbase[NW - 1] = (NB > 3 && half ? cb_base(3) : cb_base(2)) + l32;

  if constexpr (DIAG) {
    wave_sync();
    double& max_rel = dg_max_rel;
    double& sum_rel = dg_sum_rel;
    double& max_band = dg_max_band;
    unsigned long long& pairs = dg_pairs;
    for (int i = 0; i < SH::MS; ++i) {
      const uint64_t vi = i < 64 ? vm[0] : vm[NW - 1];
      if (((vi >> (i & 63)) & 1ull) == 0) continue;  // uniform
      const int idi = __builtin_amdgcn_readlane(i < 64 ? id_rank[0] : id_rank[NW - 1], i & 63);
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int j = lane + 64 * w;
        if (j > i && valid[w]) {
          const double ex =
              canon_rows<VEC>(X + (int64_t)idi * d, X + (int64_t)id_rank[w] * d, d);
          const double ap = (double)St[32 * i + lbase[w]];
          const double err = fabs(ap - ex * sc2);
          if (ex > 0.0) {
            const double rel = err / (ex * sc2);
            max_rel = fmax(max_rel, rel);
            sum_rel += rel;
          }
          const double sm = fmax((double)sr[i], (double)sr[j]) * (1.0 + 0x1p-20);
          const double E = fa.c1 * sm + fa.c2 * sqrt(sm) + fa.c3;
          max_band = fmax(max_band, err / E);
          ++pairs;
        }
      }
    }
  } else {

  // ---- a6: decision thresholds of this lane's ranks ----------------------------
  // P and K in FP32 from one fused multiply-add each.  With s = S(p, j) 2^2e
  // (exact), ts = fl32(s), rd <= ratio (1 - 2^-22) and ru >= ratio (1 + 2^-22)
  // for the exact ratio den^2 / num^2 (host-rounded floats), and
  // eu >= E (1 + 2^-22):
  //   P = fl(ts rd - eu) <= s ratio (1 - 2^-23) - E   (ts <= s (1 + 2^-24),
  //       one rounding of 2^-24 either side; eu covers the negative case),
  //   K = fl(ts ru + eu) >= s ratio (1 + 2^-23) + E   (ts >= s (1 - 2^-24)).
  // S~ <= P gives S(i, j) <= T (1 - 2^-50) with T = S(p, j) den^2 / num^2,
  // hence fl(num^2 S(i, j)) <= fl(den^2 S(p, j)); S~ > K gives
  // S(i, j) > T (1 + 2^-50), hence the opposite (FP64 roundings of 2^-53).
  // A subnormal ts adds at most 2^-149, far below E 2^-22 (E > c3).
  float P[NW][NA], K[NW][NA];
  double Ew[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const double E = fa.c1 * s2[w] + fa.c2 * sqrt(s2[w]) + fa.c3;
    Ew[w] = E;
    const float ts = (float)s2[w];
    const float eu = f32_up(E * (1.0 + 0x1p-22));
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      P[w][ai] = __builtin_fmaf(ts, a.ratio_dn[ai], -eu);
      K[w][ai] = __builtin_fmaf(ts, a.ratio_up[ai], eu);
    }
  }

  // Rows that can prune: row i can remove some j > i at alpha_k only if
  // S~(i, j) <= K_k(j), which implies fl(S~(i, j) fl(1 / s_j)) <=
  // fl(K_k(j) fl(1 / s_j)) (the same reciprocal, monotone rounding).  The
  // right side is at most (ratio_k + E_j / s_j)(1 + 2^-20.5): K_k(j) =
  // fl(ts ru + eu) with ru <= ratio_k (1 + 2^-22)(1 + 2^-23), eu <=
  // E_j (1 + 2^-22)(1 + 2^-23)(1 + 2^-53), and FP32 roundings of 2^-24 in ts,
  // K, the reciprocal and the product (K is a normal float: it exceeds c3).
  // So with eps >= max_j E_j / s_j,
  // kappa_k = (ratio_k (1 + 2^-48) + eps)(1 + 2^-19) rounded up bounds every
  // such product, and zmin_i = min_j fl(S~(i, j) fl(1 / s_j)) <= kappa_k
  // holds for every row that can prune (one reduction serves all alphas; a
  // looser bound only adds rows to visit).  Empty ranks have a NaN
  // reciprocal, which fminf ignores; S(p, j) = 0 gives 0, which keeps the
  // row visited.  A survivor whose row cannot prune is kept with nothing
  // removed.
  uint64_t vis[NA][NW];
  {
    float inv[NW];
    wave_sync();  // the tile's reads of S(p, .) are done before the region is reused
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      inv[w] = valid[w] ? (s2[w] > 0.0 ? (float)(1.0 / s2[w]) : 0.f) : __builtin_nanf("");
      invt[lane + 64 * w] = inv[w];
    }
    wave_sync();
    float zmin[NW];
    // row = rank lane: column blocks 0 (rows 0..31 only), 1, 2 and 3; row =
    // rank 64 + lane: column block 2 (rows 64..95 only) and 3; entries on and
    // below the diagonal hold +inf
    zmin[0] = __builtin_inff();
    if (lane < 32) zmin[0] = row_zmin(St, invt, 0, lane, zmin[0]);
    if (nbu > 1) zmin[0] = row_zmin(St, invt, 1, lane, zmin[0]);
    if constexpr (NW == 2) {
      zmin[1] = __builtin_inff();
      if (nbu > 2) {
        zmin[0] = row_zmin(St, invt, 2, lane, zmin[0]);
        if (lane < 32) zmin[1] = row_zmin(St, invt, 2, 64 + lane, zmin[1]);
      }
      if constexpr (NB > 3) {
        if (nbu > 3) {
          zmin[0] = row_zmin(St, invt, 3, lane, zmin[0]);
          zmin[1] = row_zmin(St, invt, 3, 64 + lane, zmin[1]);
        }
      }
    }
    float eps = 0.f;
#pragma unroll
    for (int w = 0; w < NW; ++w)
      if (valid[w] && s2[w] > 0.0) eps = fmaxf(eps, f32_up(Ew[w] / s2[w] * (1.0 + 0x1p-50)));
    for (int off = 32; off > 0; off >>= 1) eps = fmaxf(eps, __shfl_xor(eps, off, 64));
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      const float kappa = f32_up((a.ratio[ai] * (1.0 + 0x1p-48) + (double)eps) * (1.0 + 0x1p-19));
#pragma unroll
      for (int w = 0; w < NW; ++w) vis[ai][w] = __ballot(valid[w] && zmin[w] <= kappa);
    }
  }

  // ---- a7: greedy, all alphas ---------------------------------------------------
  // The ranks of mask am (one word; lane l holds rank l's id and S(p, .)) that
  // row pid prunes at alpha ai, from canonical FP64 distances: a few pairs by
  // the whole wavefront each (the x_p region of LDS is free after the pass),
  // more one per lane.
  auto recheck = [&](uint64_t am, int pid, int idl, double swl,
                     int ai) __attribute__((always_inline)) -> uint64_t {
    const float* xr = X + (int64_t)pid * d;
    if (__popcll(am) <= kWaveRechecks) {
      uint64_t pm = 0;
      for (uint64_t m = am; m != 0; m &= m - 1) {
        const int j = __builtin_ctzll(m);
        const int idj = __builtin_amdgcn_readlane(idl, j);
        const double sx = canon_rows_wave<VEC>(xr, X + (int64_t)idj * d, d, xq, lane);
        if (alpha_test_f64(a.num2[ai], a.den2[ai], sx, readlane_f64(swl, j))) pm |= 1ull << j;
      }
      return pm;
    }
    bool prune = false;
    if ((am >> lane) & 1ull)
      prune = alpha_test_f64(a.num2[ai], a.den2[ai], canon_rows<VEC>(xr, X + (int64_t)idl * d, d),
                             swl);
    return __ballot(prune);
  };
  // CAP: some output bounds R below r_max, so a chain can reach its largest R
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    rmax[ai] = 64 * NW;
    if (CAP) {
      rmax[ai] = 0;
      for (int ir = 0; ir < fa.nr; ++ir) rmax[ai] = max(rmax[ai], a.out[ai * fa.nr + ir].R);
    }
  }
  uint64_t alive[NA][NW], kept[NA][NW];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      alive[ai][w] = vm[w];
      kept[ai][w] = 0;
    }
  }
  // Chain k: the survivors before the first survivor i whose row can prune
  // at alpha_k are kept in turn (none removes anything), then i is kept and
  // row i removes what it prunes; the chain stops at its largest R (trimmed
  // below).
  if constexpr (NW == 1) {
    // Alphas arrive in descending order, so chains visit ever more rows:
    // phase s0 advances chains s0..end of its group while chain s0 has
    // survivors (a finished chain repeats harmless empty steps).  Groups of
    // four chains run one after the other, so a group's masks stay in scalar
    // registers.
    // alive[k][0] holds chain k's ranks not pruned so far and cand[k] its
    // survivors after the last visited row whose rows can prune; every rank
    // up to the visited row is decided and a survivor after the last
    // candidate prunes nothing, so the chain ends when cand is empty and
    // keeps what is left.
    uint64_t cand[NA];
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) cand[ai] = vis[ai][0] & alive[ai][0];
    constexpr int GS = 4;
#pragma unroll
    for (int g0 = 0; g0 < NA; g0 += GS) {
      const int g1 = g0 + GS < NA ? g0 + GS : NA;
#pragma unroll
      for (int s0 = g0; s0 < g1; ++s0) {
        // tested at the bottom, so the masks stay in place across steps
        if (uniform_u64(cand[s0]) == 0) continue;
        do {
          float row[NA];
          int istar[NA];
          uint64_t above[NA];
#pragma unroll
          for (int ai = s0; ai < g1; ++ai) {
            const int i = ff1_u64(uniform_u64(cand[ai]));
            // ranks after i; with no candidate (i = -1, shift 63) none
            above[ai] = 0xFFFFFFFFFFFFFFFEull << (i & 63);
            istar[ai] = i & 63;
            row[ai] = St[(i & 63) * 32 + lbase[0]];
          }
          uint64_t amb[NA];
          uint64_t any_amb = 0;
#pragma unroll
          for (int ai = s0; ai < g1; ++ai) {
            uint64_t ab = above[ai];
            uint64_t r = uniform_u64(alive[ai][0]);
            if (CAP && __popcll(r & ~ab) >= rmax[ai]) {  // R kept up to i: stop
              r &= ~ab;
              ab = 0;
            }
            const uint64_t pm = __ballot(row[ai] <= P[0][ai]);
            amb[ai] = __ballot(row[ai] <= K[0][ai]) & ~pm & r & ab;
            alive[ai][0] = r & ~(pm & ab);
            above[ai] = ab;
            any_amb |= amb[ai];
          }
          if (uniform_u64(any_amb) != 0) {
#pragma unroll
            for (int ai = s0; ai < g1; ++ai) {
              const uint64_t am = uniform_u64(amb[ai]);
              if (am) {
                const int pid = __builtin_amdgcn_readlane(id_rank[0], istar[ai]);
                alive[ai][0] &= ~recheck(am, pid, id_rank[0], sw[0], ai);
                rechecks += __popcll(am);
              }
            }
          }
#pragma unroll
          for (int ai = s0; ai < g1; ++ai) cand[ai] = alive[ai][0] & above[ai] & vis[ai][0];
        } while (uniform_u64(cand[s0]) != 0);
      }
    }
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) kept[ai][0] = alive[ai][0];
  } else {
  // Two mask words: each step advances every chain that still has survivors.
  for (;;) {
    bool live[NA];
    uint64_t any = 0;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      uint64_t al = alive[ai][0];
      if (NW == 2) al |= alive[ai][NW - 1];
      al = uniform_u64(al);
      live[ai] = al != 0;
      any |= al;
    }
    if (any == 0) break;
    float row[NA][NW];
    int istar[NA];
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      if (!live[ai]) continue;  // uniform
      // ranks after the chosen survivor i (none if no survivor can prune:
      // then every survivor is kept and the chain ends; shift 63 of the
      // constant clears it)
      const uint64_t al0 = uniform_u64(alive[ai][0]);
      const int i0 = ff1_u64(al0 & vis[ai][0]);
      const uint64_t above0 = 0xFFFFFFFFFFFFFFFEull << (i0 & 63);
      int i = i0 & 63;
      const uint64_t k0 = uniform_u64(kept[ai][0]) | (al0 & ~above0);
      int cnt = __popcll(k0);
      if constexpr (NW == 2) {
        const uint64_t al1 = uniform_u64(alive[ai][1]);
        const int i1 = ff1_u64(al1 & vis[ai][1]);
        const bool in0 = i0 >= 0;
        const uint64_t above1 = in0 ? ~0ull : 0xFFFFFFFFFFFFFFFEull << (i1 & 63);
        i = in0 ? i0 : (i1 >= 0 ? 64 + i1 : 0);
        const uint64_t k1 = uniform_u64(kept[ai][1]) | (al1 & ~above1);
        kept[ai][1] = k1;
        cnt += __popcll(k1);
        alive[ai][1] = (CAP && cnt >= rmax[ai]) ? 0ull : al1 & above1;
      }
      kept[ai][0] = k0;
      alive[ai][0] = (CAP && cnt >= rmax[ai]) ? 0ull : al0 & above0;
      istar[ai] = i;
#pragma unroll
      for (int w = 0; w < NW; ++w) row[ai][w] = St[32 * i + lbase[w]];
    }
    uint64_t amb[NA][NW];
    uint64_t any_amb = 0;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      if (!live[ai]) continue;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint64_t pm = __ballot(row[ai][w] <= P[w][ai]);
        amb[ai][w] = __ballot(row[ai][w] <= K[w][ai]) & ~pm & alive[ai][w];
        alive[ai][w] &= ~pm;
        any_amb |= amb[ai][w];
      }
    }
    if (uniform_u64(any_amb) != 0) {
#pragma unroll
      for (int ai = 0; ai < NA; ++ai) {
        if (!live[ai]) continue;
        const int is = istar[ai];
        const int pid = __builtin_amdgcn_readlane(is < 64 ? id_rank[0] : id_rank[NW - 1], is & 63);
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint64_t am = uniform_u64(amb[ai][w]);
          if (am) {
            alive[ai][w] &= ~recheck(am, pid, id_rank[w], sw[w], ai);
            rechecks += __popcll(am);
          }
        }
      }
    }
  }
  }
  // a chain that reached its R keeps its first R ranks
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    if (!CAP) break;
    int before_w = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint64_t k = kept[ai][w];
      const int before = before_w + (int)__builtin_amdgcn_mbcnt_hi(
                                        (uint32_t)(k >> 32),
                                        __builtin_amdgcn_mbcnt_lo((uint32_t)k, 0u));
      before_w += __popcll(k);
      kept[ai][w] = __ballot(((k >> lane) & 1ull) && before < rmax[ai]);
    }
  }

  // ---- a8: write every output ---------------------------------------------------
  auto write_out = [&](const SweepOut& out, int ai) {
    if constexpr (NW == 1) {
      // one store per output row: a kept rank goes to its position, every
      // other lane, in lane order, to the next -1 slot after the kept ones
      const uint64_t km = kept[ai][0];
      const int tot = __popcll(km);
      const bool mine = (km >> lane) & 1ull;
      const int before = (int)__builtin_amdgcn_mbcnt_hi(
          (uint32_t)(km >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)km, 0u));
      const int R = out.R;
      const int cntR = tot < R ? tot : R;
      int32_t* orow = out.nbr + p * R;
      const int pos = mine ? before : cntR + (lane - before);
      if (pos < R) orow[pos] = mine ? id_rank[0] : -1;
      if (R > 64) {
        for (int t = 64 + lane; t < R; t += 64) orow[t] = -1;
      }
      if (lane == 0) out.deg[p] = cntR;
      return;
    }
    int tot_k = 0, before_w[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      before_w[w] = tot_k;
      tot_k += __popcll(kept[ai][w]);
    }
    const int R = out.R;
    const int cntR = tot_k < R ? tot_k : R;
    int32_t* orow = out.nbr + p * R;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const uint64_t km = kept[ai][w];
      const int pos = before_w[w] + __popcll(km & ((1ull << lane) - 1ull));
      if (((km >> lane) & 1ull) && pos < R) orow[pos] = id_rank[w];
    }
    for (int t = cntR + lane; t < R; t += 64) orow[t] = -1;
    if (lane == 0) out.deg[p] = cntR;
  };
  if (fa.nr == 1) {  // one bound per alpha: fixed argument offsets, loaded together
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) write_out(a.out[ai], ai);
  } else {
#pragma unroll
    for (int ai = 0; ai < NA; ++ai)
      for (int ir = 0; ir < fa.nr; ++ir) write_out(a.out[ai * fa.nr + ir], ai);
  }
  }  // not DIAG


  if constexpr (DIAG) {
    for (int off = 32; off > 0; off >>= 1) {
      dg_max_rel = fmax(dg_max_rel, __shfl_xor(dg_max_rel, off, 64));
      dg_max_band = fmax(dg_max_band, __shfl_xor(dg_max_band, off, 64));
      dg_sum_rel += __shfl_xor(dg_sum_rel, off, 64);
      dg_pairs += __shfl_xor(dg_pairs, off, 64);
    }
    if (lane == 0) {
      atomicMax((unsigned long long*)&fa.stats->max_rel,
                (unsigned long long)__double_as_longlong(dg_max_rel));
      atomicMax((unsigned long long*)&fa.stats->max_band,
                (unsigned long long)__double_as_longlong(dg_max_band));
      atomicAdd(&fa.stats->sum_rel, dg_sum_rel);
      atomicAdd(&fa.stats->pairs, dg_pairs);
    }
  }
  if (lane == 0 && rechecks) atomicAdd(&ctr->rechecks, rechecks);
}

// Bound of |S~ - S(i, j) 2^2e| for every rank i before j (S(p, i) <= S(p, j)),
// s = S(p, j) 2^2e, U = (x - x_p) 2^e exact:
//   e1 = 2^-22 + 2^-23  relative error of hi + lo against U (the one FP32
//                       rounding of the scaled difference 2^-24, rounding of
//                       lo 2^-22);
//   ea = 2^-14          absolute error of one element whose hi or lo is an
//                       FP16 subnormal, even if the matrix unit flushes it;
//   dropped lo lo'      <= 2^-22 (1 + 2^-9) s;
//   FP32 accumulation   gamma over the additions into one accumulator, with
//                       unit 2^-23 (covers truncating hardware), plus the
//                       gamma of the chunk sums (unit 2^-23 as well);
//   |G~ - G| <= (2 e1 + e1^2 + lo lo' + acc) s + 2 ea sqrt(d) (1 + e1)(1 + acc) sqrt(s)
//               + d ea^2 (1 + acc);
//   S~ = (S(p,i) + S(p,j)) 2^2e - 2 G~ in FP32 adds 8 * 2^-24 s, and the
//   canonical FP64 values differ from the exact ones by at most 12 d 2^-53 s.
// Every coefficient is doubled; the FP64 threshold's own rounding is covered
// by the (1 -/+ 2^-50) factors.  csum: the accumulator restarts every kDC
// dimensions and the chunk results are summed in FP32.
void f32_bound_constants(int d, bool csum, double* c1, double* c2, double* c3) {
  auto gam = [](double n, double u) { return n * u / (1.0 - n * u); };
  const double u24 = 0x1p-24;
  const double e1 = 0x1p-22 + 0x1p-23;
  const double ea = 0x1p-14;
  const double nadd = csum ? 3.0 * kDC + 1.0 : 3.0 * d + 1.0;
  const double g1 = gam(nadd, 0x1p-23);
  // chunk sums: FP32 adds, taken with the unit of truncation as well
  const double g2 = csum ? gam((double)((d + kDC - 1) / kDC), 0x1p-23) : 0.0;
  const double acc = (g1 + g2 + g1 * g2) * (1.0 + 0x1p-9);
  const double lolo = 0x1p-22 * (1.0 + 0x1p-9);
  const double sd = sqrt((double)d);
  *c1 = 2.0 * (2.0 * (2.0 * e1 + e1 * e1 + lolo + acc) + 8.0 * u24 + 12.0 * d * 0x1p-53);
  *c2 = 2.0 * (2.0 * 2.0 * ea * sd * (1.0 + e1) * (1.0 + acc));
  *c3 = 2.0 * (2.0 * d * ea * ea * (1.0 + acc));
}

// Launch shape per graph: NB row blocks, restarted accumulators for long rows,
// 16-byte row slices when d % 4 == 0 and the point array is 16-byte aligned.
struct Plan {
  int nb;
  bool csum, vec;
  int wave_lds;
};

Plan plan_of(const GraphView& g) {
  Plan pl;
  pl.nb = g.r_max > 96 ? 4 : g.r_max > 64 ? 3 : 2;
  pl.csum = g.d > 128;
  pl.vec = (g.d % 4) == 0 && (((uintptr_t)g.X) & 15) == 0;
  pl.wave_lds = pl.nb == 4   ? wave_lds_bytes<4>(g.d)
                 : pl.nb == 3 ? wave_lds_bytes<3>(g.d)
                              : wave_lds_bytes<2>(g.d);
  return pl;
}

// Steps in flight: two for 64 candidates (three wavefronts per SIMD fit),
// four for 96 (one wavefront per SIMD), two for 128 (whose ten accumulator
// blocks take most of a wavefront's registers).
template <int NB>
constexpr int prefetch_steps() {
  return NB == 3 ? 4 : 2;
}

template <int NB, bool CSUM, bool VEC>
hipError_t launch_shape(const GraphView& g, const SweepArgs& a, const F32Args& fa,
                        DevCounters* ctr, hipStream_t s, int wave_lds) {
  constexpr int PF = prefetch_steps<NB>();
  const int waves =
      min(waves_for(TuneKey{kKernelF32, g.dtype, g.d, g.r_max, a.n_alpha, a.n_out}, wave_lds),
          NB >= 3 ? 4 : 8);  // within the launch bounds
  const dim3 grid((unsigned)((g.n + waves - 1) / waves)), block(64 * waves);
  const size_t shmem = (size_t)wave_lds * waves;
  // a bound below r_max needs the chains' keep counts (always kept for the
  // rarer shapes: 96 candidates, unaligned rows)
  bool cap = NB >= 3 || !VEC;
  for (int o = 0; o < a.n_out; ++o) cap = cap || a.out[o].R < g.r_max;
#define RP_LAUNCH_F32(NA_)                                                                 \
  case NA_:                                                                                \
    if (cap) {                                                                             \
      auto k = prune_f32_kernel<NA_, NB, CSUM, VEC, PF, true, false>;                      \
      hipLaunchKernelGGL(k, grid, block, shmem, s, g, a, fa, ctr, wave_lds);              \
    } else if constexpr (NB == 2 && VEC) {                                                 \
      auto k = prune_f32_kernel<NA_, NB, CSUM, VEC, PF, false, false>;                     \
      hipLaunchKernelGGL(k, grid, block, shmem, s, g, a, fa, ctr, wave_lds);              \
    }                                                                                      \
    break;
  switch (a.n_alpha) {
    RP_LAUNCH_F32(1)
    RP_LAUNCH_F32(2)
    RP_LAUNCH_F32(3)
    RP_LAUNCH_F32(4)
    RP_LAUNCH_F32(5)
    RP_LAUNCH_F32(6)
    RP_LAUNCH_F32(7)
    RP_LAUNCH_F32(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RP_LAUNCH_F32
  return hipGetLastError();
}

template <int NB, bool CSUM, bool VEC>
hipError_t launch_diag(const GraphView& g, const SweepArgs& a, const F32Args& fa,
                       DevCounters* ctr, hipStream_t s, int wave_lds) {
  constexpr int PF = prefetch_steps<NB>();
  auto k = prune_f32_kernel<1, NB, CSUM, VEC, PF, false, true>;
  hipLaunchKernelGGL(k, dim3((unsigned)fa.n_nodes), dim3(64), (size_t)wave_lds, s, g, a, fa, ctr,
                     wave_lds);
  return hipGetLastError();
}

// Runs L<NB, CSUM, VEC> for the graph's plan.
template <template <int, bool, bool> class L>
hipError_t dispatch(const Plan& pl, const GraphView& g, const SweepArgs& a, const F32Args& fa,
                    DevCounters* ctr, hipStream_t s) {
  if (pl.nb == 4) {  // 16-byte row slices only (prune_f32_shape_ok)
    return pl.csum ? L<4, true, true>::run(g, a, fa, ctr, s, pl.wave_lds)
                   : L<4, false, true>::run(g, a, fa, ctr, s, pl.wave_lds);
  }
  if (pl.nb == 3) {
    if (pl.csum)
      return pl.vec ? L<3, true, true>::run(g, a, fa, ctr, s, pl.wave_lds)
                    : L<3, true, false>::run(g, a, fa, ctr, s, pl.wave_lds);
    return pl.vec ? L<3, false, true>::run(g, a, fa, ctr, s, pl.wave_lds)
                  : L<3, false, false>::run(g, a, fa, ctr, s, pl.wave_lds);
  }
  if (pl.csum)
    return pl.vec ? L<2, true, true>::run(g, a, fa, ctr, s, pl.wave_lds)
                  : L<2, true, false>::run(g, a, fa, ctr, s, pl.wave_lds);
  return pl.vec ? L<2, false, true>::run(g, a, fa, ctr, s, pl.wave_lds)
                : L<2, false, false>::run(g, a, fa, ctr, s, pl.wave_lds);
}

template <int NB, bool CSUM, bool VEC>
struct SweepLaunch {
  static hipError_t run(const GraphView& g, const SweepArgs& a, const F32Args& fa,
                        DevCounters* ctr, hipStream_t s, int wave_lds) {
    return launch_shape<NB, CSUM, VEC>(g, a, fa, ctr, s, wave_lds);
  }
};

template <int NB, bool CSUM, bool VEC>
struct DiagLaunch {
  static hipError_t run(const GraphView& g, const SweepArgs& a, const F32Args& fa,
                        DevCounters* ctr, hipStream_t s, int wave_lds) {
    return launch_diag<NB, CSUM, VEC>(g, a, fa, ctr, s, wave_lds);
  }
};

// FP32 value <= x and >= x (host).
float host_f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = std::nextafter(f, -HUGE_VALF);
  return f;
}

float host_f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = std::nextafter(f, HUGE_VALF);
  return f;
}

// Sorts the alphas of a sweep in descending order (num_a^2 den_b^2 against
// num_b^2 den_a^2) and moves every output with its alpha (outputs are
// alpha-major: o = alpha * nr + iR).
SweepArgs alphas_descending(const SweepArgs& a_in, int nr) {
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

}  // namespace

int prune_f32_wave_lds(const GraphView& g) { return plan_of(g).wave_lds; }

// The band of a float32 graph of dimension d as its sweeps use it (chunked
// accumulators above d = 128), and the dimensions per accumulator chunk.
void f32_band(int d, double* c) {
  const bool csum = d > 128;
  f32_bound_constants(d, csum, &c[0], &c[1], &c[2]);
  c[3] = csum ? kDC : d;
}

// Lists of at most 128 ids whose LDS fits a workgroup of the device (on
// gfx950, 160 KiB: every d up to 4096; with 64 KiB, 96 candidates up to
// d = 3408 and 128 up to d = 2048); lists of 97..128 ids need 16-byte row
// slices.  Other graphs take the plain kernel.
bool prune_f32_shape_ok(const GraphView& g) {
  if (g.dtype != RP_F32 || g.r_max > 128 || g.d > kMaxDimF32 || g.n > (1ll << 25) ||
      g.maxabs == nullptr)
    return false;
  const Plan pl = plan_of(g);
  return pl.wave_lds <= max_lds_per_group() && (pl.nb < 4 || pl.vec);
}

bool prune_f32_supported(const GraphView& g) {
  return prune_f32_shape_ok(g) && g.frame_e != nullptr;
}

hipError_t launch_gram_error_f32(const GraphView& g, const int32_t* nodes, int64_t n_nodes,
                                 GramErrorStats* stats, DevCounters* ctr, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  if (g.frame_e == nullptr) return hipErrorInvalidValue;  // set by graph load / derive
  SweepArgs a = {};
  a.n_alpha = 1;
  a.n_out = 0;
  a.num2[0] = a.den2[0] = 1;
  a.ratio[0] = 1.0;
  F32Args fa = {};
  fa.nr = 0;
  fa.nodes = nodes;
  fa.n_nodes = n_nodes;
  fa.stats = stats;
  const Plan pl = plan_of(g);
  f32_bound_constants(g.d, pl.csum, &fa.c1, &fa.c2, &fa.c3);
  return dispatch<DiagLaunch>(pl, g, a, fa, ctr, s);
}

hipError_t launch_prune_f32(const GraphView& g, const SweepArgs& a_in, DevCounters* ctr,
                            hipStream_t s) {
  if (a_in.n_alpha < 1 || a_in.n_out % a_in.n_alpha != 0) return hipErrorInvalidValue;
  if (g.frame_e == nullptr) return hipErrorInvalidValue;  // set by graph load / derive
  F32Args fa = {};
  fa.nr = a_in.n_out / a_in.n_alpha;
  // the kernel takes the alphas in descending order, with FP32 bounds of
  // each ratio den^2 / num^2 (within (1 -/+ 2^-22))
  SweepArgs a = alphas_descending(a_in, fa.nr);
  for (int k = 0; k < a.n_alpha; ++k) {
    const double x = (double)a.den2[k] / (double)a.num2[k];  // within 2^-53 of the ratio
    a.ratio_dn[k] = host_f32_down(x * (1.0 - 0x1p-22) * (1.0 - 0x1p-50));
    a.ratio_up[k] = host_f32_up(x * (1.0 + 0x1p-22) * (1.0 + 0x1p-50));
  }
  const Plan pl = plan_of(g);
  f32_bound_constants(g.d, pl.csum, &fa.c1, &fa.c2, &fa.c3);
  return dispatch<SweepLaunch>(pl, g, a, fa, ctr, s);
}

}  // namespace rp
