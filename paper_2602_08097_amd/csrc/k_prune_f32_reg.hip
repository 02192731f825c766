// k_prune_f32_reg.hip -- batched RP-Tuning for float32 points, rows streamed
// straight into matrix-unit registers (out-lists of at most 64 ids).
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep, reading each candidate row once:
//
//  a1  read:   lane t holds the t-th listed id (its slot); p itself and -1
//              padding are empty slots.
//  a2  gather: 16 dimensions per step, straight from global memory into the
//              operand layout of the matrix instruction: for row block b
//              (slots 32 b .. 32 b + 31) lane l holds dimensions
//              16 s + 8 (l / 32) .. + 7 of row 32 b + l % 32 (two 16-byte
//              loads per block), several steps in flight.  x_p sits in LDS.
//  a3  p-row:  one lane swap (lanes 32..63 of block 0 with lanes 0..31 of
//              block 1) gives lane t all 16 dimensions of slot t's row, and
//              lane t accumulates the canonical FP64 S(p, t)
//              (t = (double)a - (double)b, fused multiply-add, k ascending).
//  a4  sort:   (S(p, j), id) ascending -- the order in which the repeated
//              argmin of Algorithm 1 visits the candidates.  A list already in
//              that order (every RobustPrune output is) is used as read;
//              otherwise the keys are sorted and the rows are streamed a
//              second time in rank order.  Repeated ids are dropped.
//  a5  Gram:   in the frame centred on p and scaled by 2^e, each FP32
//              difference is split as hi + lo (two FP16 values) and
//              G~ = sum hi hi' + hi lo' + lo hi' runs on
//              v_mfma_f32_32x32x16_f16; S~(i, j) = (S(p, i) + S(p, j)) 2^2e
//              - 2 G~(i, j) goes to a 12 KiB FP32 tile of the blocks on and
//              above the diagonal, by rank (entries with j <= i hold +inf).
//  a6  test:   fl(num^2 S(i, j)) <= fl(den^2 S(p, j)) is decided from S~
//              outside the proven band [P_j, K_j]; pairs inside it are
//              recomputed in canonical FP64 from the rows.
//  a7  greedy: per alpha a 64-bit survivor mask.  A row-minimum scan marks the
//              rows that can prune at each alpha; survivors whose row cannot
//              are kept in runs (one shift mask per step), each survivor whose
//              row can prune is kept and one ballot over its tile row removes
//              what it prunes.  A chain stops at its largest R.
//  a8  write:  kept ranks are scattered to their positions, -1 padded.
#include "f32_common.h"

namespace rp {

namespace {

constexpr int kTileEntries = 3072;  // S~ blocks (0,0), (0,1), (1,1) by rank
constexpr int kMaxDimReg = 4096;

__host__ __device__ inline int xp_floats(int d) { return (d + 15) & ~15; }

// LDS of one wavefront: S~ tile, S(p, .) 2^2e and its reciprocal by rank,
// x_p zero padded to a multiple of 16 floats.
inline int reg_wave_lds(int d) { return kTileEntries * 4 + 64 * 4 + 64 * 4 + xp_floats(d) * 4; }

struct Step {
  float4 a0, a1;  // block 0: dimensions 16 s + 8 half + 0..3, + 4..7
  float4 b0, b1;  // block 1
};

// component-wise, so the selects stay in registers
__device__ __forceinline__ void keep_or_zero(float4& v, bool keep) {
  v.x = keep ? v.x : 0.f;
  v.y = keep ? v.y : 0.f;
  v.z = keep ? v.z : 0.f;
  v.w = keep ? v.w : 0.f;
}

__device__ __forceinline__ void split8(const float4& x0, const float4& x1, const float4& p0,
                                       const float4& p1, float scf, v8h& hi, v8h& lo) {
  float u[8];
  u[0] = (x0.x - p0.x) * scf;
  u[1] = (x0.y - p0.y) * scf;
  u[2] = (x0.z - p0.z) * scf;
  u[3] = (x0.w - p0.w) * scf;
  u[4] = (x1.x - p1.x) * scf;
  u[5] = (x1.y - p1.y) * scf;
  u[6] = (x1.z - p1.z) * scf;
  u[7] = (x1.w - p1.w) * scf;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const _Float16 h = (_Float16)u[i];
    hi[i] = h;
    lo[i] = (_Float16)(u[i] - (float)h);
  }
}

// Lanes 32..63 of a and lanes 0..31 of b trade places: afterwards `lo` holds
// the first and `hi` the second half of the 16 dimensions of one row -- block
// 0's row l for lanes l < 32, block 1's row l - 32 for lanes l >= 32.
__device__ __forceinline__ void swap_halves(float a, float b, float& lo, float& hi) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(a), __float_as_uint(b), false,
                                                  false);
  lo = __uint_as_float(r[0]);
  hi = __uint_as_float(r[1]);
}

__device__ __forceinline__ double acc_sq(double acc, float a, float b) {
  const double t = (double)a - (double)b;
  return __fma_rn(t, t, acc);
}

// One pass over the rows r0 (block 0) and r1 (block 1) of this lane: the Gram
// blocks into cur / tot and, with PROW, the canonical S(p, lane's slot) into sp.
template <bool CSUM, bool PROW, int PF>  // PF: 2 or 3 steps in flight
__device__ __forceinline__ void gram_pass(const float* __restrict__ r0,
                                          const float* __restrict__ r1, int d, bool two,
                                          const float* __restrict__ xq, float scf, int half,
                                          v16f (&cur)[3], v16f (&tot)[3], double& sp) {
  const int nsteps = (d + 15) >> 4;
  const bool ragged = (d & 15) != 0;
  // every load reads valid memory: slices past d read the row's first
  // 16 bytes and are zeroed before use
  auto fetch = [&](int s) {
    const int o0 = 16 * s + 8 * half;
    const int c0 = o0 < d ? o0 : 0;
    const int c1 = o0 + 4 < d ? o0 + 4 : 0;
    Step q;
    q.a0 = *(const float4*)(r0 + c0);
    q.a1 = *(const float4*)(r0 + c1);
    q.b0 = *(const float4*)(r1 + c0);
    q.b1 = *(const float4*)(r1 + c1);
    return q;
  };
  // step s of the pass from its fetched slices
  auto step = [&](const Step q, int s) {
    const int o0 = 16 * s + 8 * half;
    float4 a0 = q.a0, a1 = q.a1, b0 = q.b0, b1 = q.b1;
    if (ragged && s == nsteps - 1) {
      const bool in0 = o0 < d, in1 = o0 + 4 < d;
      keep_or_zero(a0, in0);
      keep_or_zero(b0, in0);
      keep_or_zero(a1, in1);
      keep_or_zero(b1, in1);
    }
    const float4 p0 = *(const float4*)(xq + o0);
    const float4 p1 = *(const float4*)(xq + o0 + 4);
    v8h ha, la;
    split8(a0, a1, p0, p1, scf, ha, la);
    cur[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ha, ha, cur[0], 0, 0, 0);
    cur[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ha, la, cur[0], 0, 0, 0);
    cur[0] = __builtin_amdgcn_mfma_f32_32x32x16_f16(la, ha, cur[0], 0, 0, 0);
    if (two) {
      v8h hb, lb;
      split8(b0, b1, p0, p1, scf, hb, lb);
      cur[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ha, hb, cur[1], 0, 0, 0);
      cur[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(ha, lb, cur[1], 0, 0, 0);
      cur[1] = __builtin_amdgcn_mfma_f32_32x32x16_f16(la, hb, cur[1], 0, 0, 0);
      cur[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hb, hb, cur[2], 0, 0, 0);
      cur[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hb, lb, cur[2], 0, 0, 0);
      cur[2] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lb, hb, cur[2], 0, 0, 0);
    }
    if (CSUM && ((s & 1) || s == nsteps - 1)) {  // a fresh accumulator every 32 dimensions
#pragma unroll
      for (int q3 = 0; q3 < 3; ++q3) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          tot[q3][v] += cur[q3][v];
          cur[q3][v] = 0.f;
        }
      }
    }
    if (PROW) {
      float lo[8], hi[8];
      swap_halves(a0.x, b0.x, lo[0], hi[0]);
      swap_halves(a0.y, b0.y, lo[1], hi[1]);
      swap_halves(a0.z, b0.z, lo[2], hi[2]);
      swap_halves(a0.w, b0.w, lo[3], hi[3]);
      swap_halves(a1.x, b1.x, lo[4], hi[4]);
      swap_halves(a1.y, b1.y, lo[5], hi[5]);
      swap_halves(a1.z, b1.z, lo[6], hi[6]);
      swap_halves(a1.w, b1.w, lo[7], hi[7]);
      const float4 q0 = *(const float4*)(xq + 16 * s);
      const float4 q1 = *(const float4*)(xq + 16 * s + 4);
      const float4 q2 = *(const float4*)(xq + 16 * s + 8);
      const float4 q3 = *(const float4*)(xq + 16 * s + 12);
      double acc = sp;
      acc = acc_sq(acc, lo[0], q0.x);
      acc = acc_sq(acc, lo[1], q0.y);
      acc = acc_sq(acc, lo[2], q0.z);
      acc = acc_sq(acc, lo[3], q0.w);
      acc = acc_sq(acc, lo[4], q1.x);
      acc = acc_sq(acc, lo[5], q1.y);
      acc = acc_sq(acc, lo[6], q1.z);
      acc = acc_sq(acc, lo[7], q1.w);
      acc = acc_sq(acc, hi[0], q2.x);
      acc = acc_sq(acc, hi[1], q2.y);
      acc = acc_sq(acc, hi[2], q2.z);
      acc = acc_sq(acc, hi[3], q2.w);
      acc = acc_sq(acc, hi[4], q3.x);
      acc = acc_sq(acc, hi[5], q3.y);
      acc = acc_sq(acc, hi[6], q3.z);
      acc = acc_sq(acc, hi[7], q3.w);
      sp = acc;
    }
  };
  // PF buffers in rotation, held as values (the slices of step s + PF are
  // requested before step s is used); fetches past the last step are clamped
  Step qa = fetch(0), qb = fetch(1), qc;
  if (PF > 2) qc = fetch(2);
  for (int s = 0; s < nsteps; s += PF) {
    {
      const Step c = qa;
      if (s + PF < nsteps) qa = fetch(s + PF);
      step(c, s);
    }
    if (s + 1 < nsteps) {
      const Step c = qb;
      if (s + 1 + PF < nsteps) qb = fetch(s + 1 + PF);
      step(c, s + 1);
    }
    if (PF > 2 && s + 2 < nsteps) {
      const Step c = qc;
      if (s + 2 + PF < nsteps) qc = fetch(s + 2 + PF);
      step(c, s + 2);
    }
  }
}

// S~ of one 32 x 32 block (rows of block BI, columns of block BJ) into the
// tile.  Layout: columns 0..31 of rows 0..31 at 32 i + c; columns 32..63 of
// rows 0..63 at 1024 + 32 i + (c - 32).  Accumulator layout: lane l holds
// column l % 32 of rows 8 (v / 4) + 4 (l / 32) + v % 4 in register v.
template <int BI, int BJ>
__device__ __forceinline__ void store_block(float* St, const float* sr, const v16f& acc, int l32,
                                            int half) {
  const float scol = sr[32 * BJ + l32];
  float4 nrow[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) nrow[q] = *(const float4*)(sr + 32 * BI + 8 * q + 4 * half);
  float* base = St + (BJ == 0 ? 0 : 1024 + 32 * 32 * BI) + 128 * half + l32;
  const int below = l32 - 4 * half;  // column after row  <=>  below > 8 q + j
#pragma unroll
  for (int v = 0; v < 16; ++v) {
    const int rr = 8 * (v >> 2) + (v & 3);
    const float4 nq = nrow[v >> 2];
    const float srow = (v & 3) == 0 ? nq.x : (v & 3) == 1 ? nq.y : (v & 3) == 2 ? nq.z : nq.w;
    const float val = (srow + scol) - 2.f * acc[v];
    base[32 * rr] = (BI != BJ || below > rr) ? val : __builtin_inff();
  }
}

// DIAG: measure instead of prune -- for the listed vertices, every candidate
// pair's S~ is compared with the canonical FP64 S(i, j) (relative error, and
// error over the proven band), and nothing is written.
template <int NA, bool CSUM, bool CAP, int PF, bool DIAG>
__global__ __launch_bounds__(512) void prune_f32r_kernel(GraphView g, SweepArgs a, F32Args fa,
                                                         DevCounters* ctr, int32_t wave_lds) {
  extern __shared__ __align__(16) uint8_t lds_all[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (DIAG) {
    if (p >= fa.n_nodes) return;
    p = fa.nodes[p];
  }
  if (p >= g.n) return;
  uint8_t* lds = lds_all + (size_t)wave * wave_lds;
  float* St = (float*)lds;          // S~ tile
  float* sr = St + kTileEntries;    // S(p, .) 2^2e by rank (FP32)
  float* invt = sr + 64;            // 1 / S(p, .) 2^2e by rank
  float* xq = invt + 64;            // x_p, zero padded
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int d = g.d;
  const float* X = (const float*)g.X;

  // ---- a1 ------------------------------------------------------------------
  const int raw = lane < g.r_max ? g.nbr[p * g.r_max + lane] : -1;
  const int m = g.deg[p];
  const int id = (lane < m && raw != (int)p) ? raw : -1;
  const bool two = m > 32;  // uniform: block 1 holds listed slots
  const int id0 = __shfl(id, l32, 64);
  const int id1 = __shfl(id, 32 + l32, 64);

  // loads in the order they are needed: scale inputs, x_p, then the rows
  const float mj0 = id >= 0 ? g.maxabs[id] : 0.f;
  const float mp = g.maxabs[p];
  const float* xrow = X + p * d;
  const int xpf = xp_floats(d);
  float4 xv = make_float4(0.f, 0.f, 0.f, 0.f);
  if (4 * lane < d) xv = *(const float4*)(xrow + 4 * lane);

  // ---- a2 + a3 + a5: one pass over the rows in slot order ----------------
  const float* r0 = X + (int64_t)(id0 >= 0 ? id0 : (int)p) * d;
  const float* r1 = X + (int64_t)(id1 >= 0 ? id1 : (int)p) * d;

  float mj = mj0;
  for (int off = 32; off > 0; off >>= 1) mj = fmaxf(mj, __shfl_xor(mj, off, 64));
  const int e = frame_exponent(mj + mp);
  const float scf = ldexpf(1.f, e);
  const double sc = ldexp(1.0, e);
  const double sc2 = sc * sc;
  if (4 * lane < xpf) *(float4*)(xq + 4 * lane) = xv;
  for (int c = 4 * lane + 256; c < xpf; c += 256) {  // long rows
    const float4 v = c < d ? *(const float4*)(xrow + c) : make_float4(0.f, 0.f, 0.f, 0.f);
    *(float4*)(xq + c) = v;
  }
  wave_sync();

  v16f cur[3], tot[3];
#pragma unroll
  for (int q = 0; q < 3; ++q) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      cur[q][v] = 0.f;
      tot[q][v] = 0.f;
    }
  }
  double sp = 0.0;
  gram_pass<CSUM, true, PF>(r0, r1, d, two, xq, scf, half, cur, tot, sp);

  // ---- a4: sort by (S(p, j), id); drop repeated ids -------------------------
  uint64_t kh = ~0ull;
  uint32_t kl = ~0u;
  if (id >= 0) {
    kh = (uint64_t)__double_as_longlong(sp);
    kl = ((uint32_t)id << 6) | (uint32_t)lane;
  }
  {
    const uint64_t ph = shfl_u64(kh, lane > 0 ? lane - 1 : 0);
    const uint32_t pl = (uint32_t)__shfl((int)kl, lane > 0 ? lane - 1 : 0, 64);
    if (__ballot(lane > 0 && key_less(kh, kl, ph, pl)) != 0) {
      // out of rank order: sort the keys, stream the rows again by rank
      wave_sort2(kh, kl, lane);
      const int idk = kh != ~0ull ? (int)(kl >> 6) : -1;
      const int k0 = __shfl(idk, l32, 64);
      const int k1 = __shfl(idk, 32 + l32, 64);
      const float* q0 = X + (int64_t)(k0 >= 0 ? k0 : (int)p) * d;
      const float* q1 = X + (int64_t)(k1 >= 0 ? k1 : (int)p) * d;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          cur[q][v] = 0.f;
          tot[q][v] = 0.f;
        }
      }
      double unused = 0.0;
      gram_pass<CSUM, false, PF>(q0, q1, d, two, xq, scf, half, cur, tot, unused);
    }
  }
  bool valid;
  {
    uint64_t ph = shfl_u64(kh, lane > 0 ? lane - 1 : 0);
    uint32_t pl = (uint32_t)__shfl((int)kl, lane > 0 ? lane - 1 : 0, 64);
    if (lane == 0) {
      ph = ~0ull - 1;
      pl = 0u;
    }
    valid = kh != ~0ull && !(kh == ph && (kl >> 6) == (pl >> 6));
  }
  const uint64_t vm = __ballot(valid);
  const int id_rank = valid ? (int)(kl >> 6) : -1;
  const double sw = valid ? __longlong_as_double((long long)kh) : 0.0;
  const double s2 = sw * sc2;
  sr[lane] = valid ? (float)s2 : 0.f;
  wave_sync();

  // ---- a5: S~ tile by rank ----------------------------------------------------
  store_block<0, 0>(St, sr, CSUM ? tot[0] : cur[0], l32, half);
  if (two) {
    store_block<0, 1>(St, sr, CSUM ? tot[1] : cur[1], l32, half);
    store_block<1, 1>(St, sr, CSUM ? tot[2] : cur[2], l32, half);
  }
  const int lbase = l32 + 1024 * half;  // tile entry (i, lane) = St[32 i + lbase]

  if constexpr (DIAG) {
    wave_sync();
    double max_rel = 0.0, sum_rel = 0.0, max_band = 0.0;
    unsigned long long pairs = 0;
    for (int i = 0; i < 64; ++i) {
      if (((vm >> i) & 1ull) == 0) continue;  // uniform
      const int idi = __builtin_amdgcn_readlane(id_rank, i);
      if (lane > i && valid) {
        const double ex =
            canon_rows<true>(X + (int64_t)idi * d, X + (int64_t)id_rank * d, d);
        const double ap = (double)St[32 * i + lbase];
        const double err = fabs(ap - ex * sc2);
        if (ex > 0.0) {
          const double rel = err / (ex * sc2);
          max_rel = fmax(max_rel, rel);
          sum_rel += rel;
        }
        const double sm = fmax((double)sr[i], (double)sr[lane]) * (1.0 + 0x1p-20);
        const double E = fa.c1 * sm + fa.c2 * sqrt(sm) + fa.c3;
        max_band = fmax(max_band, err / E);
        ++pairs;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      max_rel = fmax(max_rel, __shfl_xor(max_rel, off, 64));
      max_band = fmax(max_band, __shfl_xor(max_band, off, 64));
      sum_rel += __shfl_xor(sum_rel, off, 64);
      pairs += __shfl_xor(pairs, off, 64);
    }
    if (lane == 0) {
      atomicMax((unsigned long long*)&fa.stats->max_rel,
                (unsigned long long)__double_as_longlong(max_rel));
      atomicMax((unsigned long long*)&fa.stats->max_band,
                (unsigned long long)__double_as_longlong(max_band));
      atomicAdd(&fa.stats->sum_rel, sum_rel);
      atomicAdd(&fa.stats->pairs, pairs);
    }
    return;
  }

  // ---- a6: decision thresholds of this lane's rank ----------------------------
  float P[NA], K[NA];
  {
    const double E = fa.c1 * s2 + fa.c2 * sqrt(s2) + fa.c3;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      // t = fl(S(p, j) fl(den^2 / num^2)) is within 2^-51.4 of den^2 S(p, j) / num^2,
      // so S(i, j) <= t (1 - 2^-50) implies fl(num^2 S(i, j)) <= fl(den^2 S(p, j)),
      // and S(i, j) > t (1 + 2^-49) implies the opposite.
      const double t = sw * a.ratio[ai];
      P[ai] = f32_down(t * (1.0 - 0x1p-50) * sc2 - E);
      K[ai] = f32_up(t * (1.0 + 0x1p-49) * sc2 + E);
    }
  }

  // Rows that can prune: row i can remove some j > i at alpha_k only if
  // S~(i, j) <= K_k(j), which implies fl(S~(i, j) / s_j) <= kappa_k :=
  // max_j fl(K_k(j) / s_j) (FP32 products with the same reciprocal, so the
  // implication survives rounding; empty ranks have a NaN reciprocal and drop
  // out of both).  A survivor whose row cannot prune is kept with nothing
  // removed.
  uint64_t vis[NA];
  {
    const float inv = valid ? (s2 > 0.0 ? (float)(1.0 / s2) : 0.f) : __builtin_nanf("");
    invt[lane] = inv;
    wave_sync();
    float zmin = __builtin_inff();
    const float* rowB = St + 1024 + 32 * lane;  // columns 32..63
#pragma unroll
    for (int c0 = 0; c0 < 32; c0 += 4) {
      const float4 v = *(const float4*)(rowB + c0);
      const float4 iv = *(const float4*)(invt + 32 + c0);
      zmin = fminf(zmin, fminf(fminf(v.x * iv.x, v.y * iv.y), fminf(v.z * iv.z, v.w * iv.w)));
    }
    if (lane < 32) {  // columns 0..31 (entries on and below the diagonal hold +inf)
      const float* rowA = St + 32 * lane;
#pragma unroll
      for (int c0 = 0; c0 < 32; c0 += 4) {
        const float4 v = *(const float4*)(rowA + c0);
        const float4 iv = *(const float4*)(invt + c0);
        zmin =
            fminf(zmin, fminf(fminf(v.x * iv.x, v.y * iv.y), fminf(v.z * iv.z, v.w * iv.w)));
      }
    }
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      float q = valid ? K[ai] * inv : -__builtin_inff();
      for (int off = 32; off > 0; off >>= 1) q = fmaxf(q, __shfl_xor(q, off, 64));
      vis[ai] = __ballot(valid && zmin <= q);
    }
  }

  // ---- a7: greedy, all alphas ---------------------------------------------------
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    rmax[ai] = 64;
    if (CAP) {
      rmax[ai] = 0;
      for (int ir = 0; ir < fa.nr; ++ir) rmax[ai] = max(rmax[ai], a.out[ai * fa.nr + ir].R);
    }
  }
  uint64_t alive[NA], kept[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    alive[ai] = vm;
    kept[ai] = 0;
  }
  unsigned long long rechecks = 0;
  // Chain k: the survivors before the first survivor i whose row can prune
  // at alpha_k are kept in turn (none removes anything), then i is kept and
  // row i removes what it prunes; the chain stops at its largest R (trimmed
  // below).  Alphas arrive in descending order, so chains visit ever more
  // rows: phase s0 advances chains s0..NA-1 while chain s0 has survivors (a
  // finished chain repeats harmless empty steps).
#pragma unroll
  for (int s0 = 0; s0 < NA; ++s0) {
    while (uniform_u64(alive[s0]) != 0) {
      float row[NA];
      int istar[NA];
#pragma unroll
      for (int ai = s0; ai < NA; ++ai) {
        const uint64_t al = uniform_u64(alive[ai]);
        const int i = ff1_u64(al & vis[ai]);
        // ranks above i; with no candidate (i = -1, shift 63) none, so every
        // survivor is kept and the chain ends
        const uint64_t above = 0xFFFFFFFFFFFFFFFEull << (i & 63);
        const uint64_t k = uniform_u64(kept[ai]) | (al & ~above);
        kept[ai] = k;
        alive[ai] = (CAP && __popcll(k) >= rmax[ai]) ? 0ull : al & above;
        istar[ai] = i & 63;
        row[ai] = St[(i & 63) * 32 + lbase];
      }
      uint64_t amb[NA];
      uint64_t any_amb = 0;
#pragma unroll
      for (int ai = s0; ai < NA; ++ai) {
        const uint64_t pm = __ballot(row[ai] <= P[ai]);
        amb[ai] = __ballot(row[ai] <= K[ai]) & ~pm & alive[ai];
        alive[ai] &= ~pm;
        any_amb |= amb[ai];
      }
      if (uniform_u64(any_amb) != 0) {
#pragma unroll
        for (int ai = s0; ai < NA; ++ai) {
          const uint64_t am = uniform_u64(amb[ai]);
          if (am) {
            const int pid = __builtin_amdgcn_readlane(id_rank, istar[ai]);
            bool prune = false;
            if ((am >> lane) & 1ull) {
              const double sx =
                  canon_rows<true>(X + (int64_t)pid * d, X + (int64_t)id_rank * d, d);
              prune = alpha_test_f64(a.num2[ai], a.den2[ai], sx, sw);
            }
            alive[ai] &= ~(uint64_t)__ballot(prune);
            rechecks += __popcll(am);
          }
        }
      }
    }
  }
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

  // ---- a8: write every output ---------------------------------------------------
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    const uint64_t km = kept[ai];
    const int tot_k = __popcll(km);
    const bool mine = (km >> lane) & 1ull;
    const int pos = __popcll(km & ((1ull << lane) - 1ull));
    for (int ir = 0; ir < fa.nr; ++ir) {
      const SweepOut& out = a.out[ai * fa.nr + ir];
      const int R = out.R;
      const int cntR = tot_k < R ? tot_k : R;
      int32_t* orow = out.nbr + p * R;
      if (mine && pos < R) orow[pos] = id_rank;
      for (int t = cntR + lane; t < R; t += 64) orow[t] = -1;
      if (lane == 0) out.deg[p] = cntR;
    }
  }
  if (lane == 0 && rechecks) atomicAdd(&ctr->rechecks, rechecks);
}

template <bool CSUM, int PF>
hipError_t launch_na(const GraphView& g, const SweepArgs& a, const F32Args& fa, DevCounters* ctr,
                     hipStream_t s, int wave_lds, int waves) {
  bool cap = false;
  for (int o = 0; o < a.n_out; ++o) cap = cap || a.out[o].R < g.r_max;
  const dim3 grid((unsigned)((g.n + waves - 1) / waves)), block(64 * waves);
  const size_t shmem = (size_t)wave_lds * waves;
#define RP_LAUNCH_F32R(NA_)                                                                    \
  case NA_:                                                                                    \
    if (cap)                                                                                   \
      hipLaunchKernelGGL((prune_f32r_kernel<NA_, CSUM, true, PF, false>), grid, block, shmem,  \
                         s, g, a, fa, ctr, wave_lds);                                          \
    else                                                                                       \
      hipLaunchKernelGGL((prune_f32r_kernel<NA_, CSUM, false, PF, false>), grid, block, shmem, \
                         s, g, a, fa, ctr, wave_lds);                                          \
    break;
  switch (a.n_alpha) {
    RP_LAUNCH_F32R(1)
    RP_LAUNCH_F32R(2)
    RP_LAUNCH_F32R(3)
    RP_LAUNCH_F32R(4)
    RP_LAUNCH_F32R(5)
    RP_LAUNCH_F32R(6)
    RP_LAUNCH_F32R(7)
    RP_LAUNCH_F32R(8)
    default:
      return hipErrorInvalidValue;
  }
#undef RP_LAUNCH_F32R
  return hipGetLastError();
}

}  // namespace

int prune_f32r_wave_lds(const GraphView& g) { return reg_wave_lds(g.d); }

// 16-byte row slices need d % 4 == 0 and a 16-byte aligned point array.
bool prune_f32r_supported(const GraphView& g) {
  return g.dtype == RP_F32 && g.r_max <= 64 && (g.d % 4) == 0 && g.d <= kMaxDimReg &&
         (((uintptr_t)g.X) & 15) == 0 && g.n <= (1ll << 25) && g.maxabs != nullptr;
}

// Alphas in descending order (alphas_descending), fa.nr outputs per alpha.
hipError_t launch_prune_f32r(const GraphView& g, const SweepArgs& a, F32Args fa,
                             DevCounters* ctr, hipStream_t s) {
  const int wave_lds = reg_wave_lds(g.d);
  const int waves =
      waves_for(TuneKey{kKernelF32, g.dtype, g.d, g.r_max, a.n_alpha, a.n_out}, wave_lds);
  const bool csum = g.d > 128;
  f32_bound_constants(g.d, csum, &fa.c1, &fa.c2, &fa.c3);
  return csum ? launch_na<true, 2>(g, a, fa, ctr, s, wave_lds, waves)
              : launch_na<false, 2>(g, a, fa, ctr, s, wave_lds, waves);
}

hipError_t launch_gram_error_f32r(const GraphView& g, const SweepArgs& a, F32Args fa,
                                  DevCounters* ctr, hipStream_t s) {
  const int wave_lds = reg_wave_lds(g.d);
  const bool csum = g.d > 128;
  f32_bound_constants(g.d, csum, &fa.c1, &fa.c2, &fa.c3);
  const dim3 grid((unsigned)fa.n_nodes), block(64);
  if (csum)
    hipLaunchKernelGGL((prune_f32r_kernel<1, true, false, 2, true>), grid, block, wave_lds, s, g,
                       a, fa, ctr, wave_lds);
  else
    hipLaunchKernelGGL((prune_f32r_kernel<1, false, false, 2, true>), grid, block, wave_lds, s,
                       g, a, fa, ctr, wave_lds);
  return hipGetLastError();
}

}  // namespace rp
