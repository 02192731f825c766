// k_prune_f32.hip -- batched RP-Tuning for float32 points: split-FP16 MFMA
// Gram tile with a rigorous rounding band and a canonical FP64 recheck.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep, for out-lists of at most 96 ids and any
// d.  The candidate rows are streamed once, 32 dimensions at a time:
//
//  a1  read:   the listed ids by slot (p itself and -1 padding are empty).
//  a2  gather: per chunk, coalesced 16-byte loads of the slot rows and of x_p
//              into an FP32 LDS tile; the next chunk's loads are in flight
//              while the current one is used.
//  a3  p-row:  lane j accumulates the canonical FP64 S(p, j) of its slot
//              (t = (double)a - (double)b, fused multiply-add in ascending k)
//              across the chunks -- the exact sort key and test operand.
//  a5  Gram:   in the frame centred on p and scaled by 2^e (so that every
//              |x_jk - x_pk| 2^e < 2^14; e from per-point max |x_k|), each
//              FP32 difference v is split as hi + lo, two FP16 values, and
//              G~ = sum hi hi' + hi lo' + lo hi' runs on
//              v_mfma_f32_32x32x16_f16; for long rows every chunk starts a
//              fresh accumulator that is then added to the total, which keeps
//              the FP32 accumulation error near gamma_{3 * 32} instead of
//              gamma_{3 d}.  S~(i, j) = (S(p, i) + S(p, j)) 2^2e - 2 G~(i, j)
//              goes to an FP32 LDS tile in slot order.
//  a4  sort:   (S(p, j), id) ascending -- the order in which the repeated
//              argmin of Algorithm 1 visits the candidates (a list already in
//              that order skips the network); repeated ids are dropped.
//  a6  test:   fl(num^2 S(i, j)) <= fl(den^2 S(p, j)), the condition on
//              canonical values, is decided from S~ when S~ lies outside
//              [P_j, K_j]: thresholds that carry the proven bound
//              |S~ - S(i, j) 2^2e| <= c1 s + c2 sqrt(s) + c3 (s = S(p, j) 2^2e)
//              and the FP64 rounding of both products.  Pairs inside the band
//              are recomputed in canonical FP64 from the float32 rows.
//  a7  greedy: per alpha a rank mask of survivors; the lowest survivor i is
//              kept, row i of S~ is compared with each lane's thresholds;
//              the chains of all alphas advance in lockstep.
//  a8  write:  kept ranks are scattered to their positions, -1 padded.
#include "f32_common.h"

namespace rp {

namespace {

constexpr int kRowF = kDC + 4;  // floats per LDS chunk row (16-byte aligned rows)

template <int NB>
struct Shape {
  static constexpr int MS = 32 * NB;                // candidate slots
  static constexpr int ROWS = MS + 1;               // + x_p in row MS
  static constexpr int SEG = (ROWS * 8 + 63) / 64;  // 16-byte loads per lane per chunk
  static constexpr int NP = NB * (NB + 1) / 2;      // 32 x 32 blocks on and above the diagonal
  static constexpr int NW = NB > 2 ? 2 : 1;         // 64-bit words of a rank mask
  static constexpr int TILE_B = ROWS * kRowF * 4;   // chunk tile
  static constexpr int SP = MS + 4;                 // S~ row stride (16-byte rows, conflict-free scans)
  static constexpr int STILE_B = MS * SP * 4;       // S~ tile (overlays the chunk tile)
  static constexpr int A_B = TILE_B > STILE_B ? TILE_B : STILE_B;
  static constexpr int LDS_B = (A_B + MS * 4 + MS * 4 + 15) & ~15;
};

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

// DIAG: measure instead of prune -- for the listed vertices, every candidate
// pair's S~ is compared with the canonical FP64 S(i, j) (relative error, and
// error over the proven band E_j), and nothing is written.
template <int NA, int NB, bool CSUM, bool VEC, bool DIAG = false>
__global__ __launch_bounds__(512) void prune_f32_kernel(GraphView g, SweepArgs a, F32Args fa,
                                                        DevCounters* ctr) {
  using SH = Shape<NB>;
  constexpr int MS = SH::MS;
  constexpr int NW = SH::NW;
  constexpr int NP = SH::NP;
  constexpr int SP = SH::SP;
  extern __shared__ __align__(16) uint8_t lds_all[];
  const int wave = threadIdx.x >> 6;
  int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (DIAG) {
    if (p >= fa.n_nodes) return;
    p = fa.nodes[p];
  }
  if (p >= g.n) return;
  uint8_t* lds = lds_all + (size_t)wave * SH::LDS_B;  // this wavefront's vertex
  float* T = (float*)lds;                   // chunk tile, ROWS x kRowF
  float* St = (float*)lds;                  // S~ tile, MS x SP, slot order (after the Gram)
  float* sr = (float*)(lds + SH::A_B);      // S(p, slot) 2^2e in FP32
  int32_t* idl = (int32_t*)(sr + MS);       // id by slot, -1 if empty

  const int lane = threadIdx.x & 63;
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int d = g.d;
  const float* X = (const float*)g.X;

  // ---- a1 ------------------------------------------------------------------
  const int m = g.deg[p];
  int idw[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int s = lane + 64 * w;
    int id = -1;
    if (s < MS && s < m) id = g.nbr[p * g.r_max + s];
    if (id == (int)p) id = -1;
    idw[w] = id;
    if (s < MS) idl[s] = id;
  }

  // power-of-two scale: |x_jk - x_pk| <= max|x_j| + max|x_p| < 2^ex, e = 14 - ex
  float mj = 0.f;
#pragma unroll
  for (int w = 0; w < NW; ++w)
    if (idw[w] >= 0) mj = fmaxf(mj, g.maxabs[idw[w]]);
  for (int off = 32; off > 0; off >>= 1) mj = fmaxf(mj, __shfl_xor(mj, off, 64));
  const float bound = mj + g.maxabs[p];
  const int e = frame_exponent(bound);
  const float scf = ldexpf(1.f, e);
  const double sc = ldexp(1.0, e);
  const double sc2 = sc * sc;
  wave_sync();

  // ---- a2 + a3 + a5: streamed chunks ----------------------------------------
  const int nseg = (m + 1) * 8;   // rows 0..m-1, then x_p; 8 x 16 bytes per row
  const int nch = (d + kDC - 1) / kDC;
  const int nbv = (m + 31) >> 5;  // blocks holding listed slots
  float4 buf[SH::SEG];
  auto issue = [&](int c0) {
#pragma unroll
    for (int t = 0; t < SH::SEG; ++t) {
      const int c = lane + 64 * t;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (c < nseg) {
        const int row = c >> 3;
        const int col = c0 + 4 * (c & 7);
        const int rid = row < m ? idl[row] : (int)p;
        if (rid >= 0 && col < d) {
          const float* src = X + (int64_t)rid * d + col;
          if (VEC) {
            v = *(const float4*)src;
          } else {
            v.x = src[0];
            if (col + 1 < d) v.y = src[1];
            if (col + 2 < d) v.z = src[2];
            if (col + 3 < d) v.w = src[3];
          }
        }
      }
      buf[t] = v;
    }
  };

  double sp[NW];
#pragma unroll
  for (int w = 0; w < NW; ++w) sp[w] = 0.0;
  v16f cur[NP], tot[NP];
#pragma unroll
  for (int q = 0; q < NP; ++q) {
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      cur[q][v] = 0.f;
      tot[q][v] = 0.f;
    }
  }

  issue(0);
  for (int ch = 0; ch < nch; ++ch) {
    const int c0 = ch * kDC;
    const int dc = min(kDC, d - c0);
    wave_sync();  // the previous chunk's reads are done
#pragma unroll
    for (int t = 0; t < SH::SEG; ++t) {
      const int c = lane + 64 * t;
      if (c < nseg) {
        const int row = c >> 3;
        const int lrow = row < m ? row : MS;
        *(float4*)(T + lrow * kRowF + 4 * (c & 7)) = buf[t];
      }
    }
    if (ch + 1 < nch) issue(c0 + kDC);
    wave_sync();

    // canonical S(p, j), k ascending
    const float* xp = T + MS * kRowF;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      const int s = lane + 64 * w;
      if (s < MS) {
        const float* xj = T + s * kRowF;
        double acc = sp[w];
        int k = 0;
        for (; k + 4 <= dc; k += 4) {
          const float4 xa = *(const float4*)(xj + k);
          const float4 xb = *(const float4*)(xp + k);
          double t = (double)xa.x - (double)xb.x;
          acc = __fma_rn(t, t, acc);
          t = (double)xa.y - (double)xb.y;
          acc = __fma_rn(t, t, acc);
          t = (double)xa.z - (double)xb.z;
          acc = __fma_rn(t, t, acc);
          t = (double)xa.w - (double)xb.w;
          acc = __fma_rn(t, t, acc);
        }
        for (; k < dc; ++k) {
          const double t = (double)xj[k] - (double)xp[k];
          acc = __fma_rn(t, t, acc);
        }
        sp[w] = acc;
      }
    }

    // Gram on MFMA: rows of block b are slots 32 b + l32; lane half h holds
    // dimensions 8 h .. 8 h + 7 of each 16-wide step.
#pragma unroll
    for (int kk = 0; kk < kDC; kk += 16) {
      if (kk < dc) {
        const float* pq = xp + kk + 8 * half;
        const float4 p0 = *(const float4*)pq;
        const float4 p1 = *(const float4*)(pq + 4);
        v8h hi[NB], lo[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          if (b >= nbv) break;  // uniform
          const float* xr = T + (32 * b + l32) * kRowF + kk + 8 * half;
          const float4 x0 = *(const float4*)xr;
          const float4 x1 = *(const float4*)(xr + 4);
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
            hi[b][i] = h;
            lo[b][i] = (_Float16)(u[i] - (float)h);
          }
        }
        int q = 0;
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
          for (int bj = bi; bj < NB; ++bj, ++q) {
            if (bj < nbv) {
              cur[q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hi[bi], hi[bj], cur[q], 0, 0, 0);
              cur[q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(hi[bi], lo[bj], cur[q], 0, 0, 0);
              cur[q] = __builtin_amdgcn_mfma_f32_32x32x16_f16(lo[bi], hi[bj], cur[q], 0, 0, 0);
            }
          }
        }
      }
    }
    if (CSUM) {
#pragma unroll
      for (int q = 0; q < NP; ++q) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
          tot[q][v] += cur[q][v];
          cur[q][v] = 0.f;
        }
      }
    }
  }

#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const int s = lane + 64 * w;
    if (s < MS) sr[s] = (float)(sp[w] * sc2);
  }
  wave_sync();  // every chunk-tile read is done; sr is visible

  // S~ tile in slot order (both triangles; one writer per entry).
  // Accumulator layout of a 32 x 32 block: lane l holds column l % 32 of rows
  // 8 (v / 4) + 4 (l / 32) + v % 4 in register v.
  {
    int q = 0;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
#pragma unroll
      for (int bj = bi; bj < NB; ++bj, ++q) {
        if (bj < nbv) {
          const int cs = 32 * bj + l32;
          const float scol = sr[cs];
#pragma unroll
          for (int v = 0; v < 16; ++v) {
            const int rs = 32 * bi + 8 * (v >> 2) + 4 * half + (v & 3);
            const float gv = CSUM ? tot[q][v] : cur[q][v];
            const float val = (sr[rs] + scol) - 2.f * gv;
            if (bi != bj) {
              St[rs * SP + cs] = val;
              St[cs * SP + rs] = val;
            } else {
              St[rs * SP + cs] = val;
            }
          }
        }
      }
    }
  }

  if constexpr (DIAG) {
    wave_sync();
    double max_rel = 0.0, sum_rel = 0.0, max_band = 0.0;
    unsigned long long pairs = 0;
    for (int i = 0; i < m && i < MS; ++i) {
      const int idi = idl[i];
      if (idi < 0) continue;  // uniform
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const int j = lane + 64 * w;
        if (j > i && j < m && j < MS && idw[w] >= 0 && idw[w] != idi) {
          const double ex = canon_rows<VEC>(X + (int64_t)idi * d, X + (int64_t)idw[w] * d, d);
          const double ap = (double)St[i * SP + j];
          const double err = fabs(ap - ex * sc2);
          if (ex > 0.0) {
            const double rel = err / (ex * sc2);
            max_rel = fmax(max_rel, rel);
            sum_rel += rel;
          }
          const double s2 = fmax((double)sr[i], (double)sr[j]) * (1.0 + 0x1p-20);
          const double E = fa.c1 * s2 + fa.c2 * sqrt(s2) + fa.c3;
          max_band = fmax(max_band, err / E);
          ++pairs;
        }
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

  // ---- a4: sort by (S(p, j), id); drop repeated ids -------------------------
  constexpr int kSlotBits = NW == 2 ? 7 : 6;
  uint64_t kh[2];
  uint32_t kl[2];
#pragma unroll
  for (int w = 0; w < 2; ++w) {
    kh[w] = ~0ull;
    kl[w] = ~0u;
  }
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    if (idw[w] >= 0) {
      kh[w] = (uint64_t)__double_as_longlong(sp[w]);
      kl[w] = ((uint32_t)idw[w] << kSlotBits) | (uint32_t)(lane + 64 * w);
    }
  }
  bool sorted;  // slot order is rank order
  {
    // a list already in (S, id) order -- every RobustPrune output is -- skips the network
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
      unsorted = unsorted || (lane == 0 && key_less(kh[1], kl[1], lh, ll));
    }
    sorted = __ballot(unsorted) == 0;
    if (!sorted) {
      if (NW == 2) wave_sort128(kh[0], kl[0], kh[1], kl[1], lane);
      else wave_sort2(kh[0], kl[0], lane);
    }
  }
  uint64_t vm[NW];
  int slotw[NW], idr[NW];
  double sw[NW];
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
    const bool valid = kh[w] != ~0ull &&
                       !(kh[w] == ph && (kl[w] >> kSlotBits) == (pl >> kSlotBits));
    vm[w] = __ballot(valid);
    slotw[w] = valid ? (int)(kl[w] & ((1u << kSlotBits) - 1)) : 0;
    idr[w] = valid ? (int)(kl[w] >> kSlotBits) : -1;
    sw[w] = valid ? __longlong_as_double((long long)kh[w]) : 0.0;
  }

  // ---- a6: decision thresholds of this lane's ranks -------------------------
  float P[NW][NA], K[NW][NA];
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const double s2 = sw[w] * sc2;
    const double E = fa.c1 * s2 + fa.c2 * sqrt(s2) + fa.c3;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      // t = fl(S(p, j) fl(den^2 / num^2)) is within 2^-51.4 of den^2 S(p, j) / num^2,
      // so S(i, j) <= t (1 - 2^-50) implies fl(num^2 S(i, j)) <= fl(den^2 S(p, j)),
      // and S(i, j) > t (1 + 2^-49) implies the opposite.
      const double t = sw[w] * a.ratio[ai];
      P[w][ai] = f32_down(t * (1.0 - 0x1p-50) * sc2 - E);
      K[w][ai] = f32_up(t * (1.0 + 0x1p-49) * sc2 + E);
    }
  }

  // ---- a7: greedy, all alphas in lockstep ----------------------------------
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    rmax[ai] = 0;
    for (int ir = 0; ir < fa.nr; ++ir) rmax[ai] = max(rmax[ai], a.out[ai * fa.nr + ir].R);
  }
  uint64_t alive[NA][NW], kept[NA][NW];
  int cnt[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    cnt[ai] = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      alive[ai][w] = vm[w];
      kept[ai][w] = 0;
    }
  }
  unsigned long long rechecks = 0;

  if constexpr (NW == 1) {
    // Rows that can prune.  For a list in rank order, row i can remove some
    // j > i at alpha_k only if S~(i, j) <= K_k(j) for some j, which implies
    // fl(S~(i, j) / s_j) <= kappa_k := max_j fl(K_k(j) / s_j) (FP32 products
    // with the same reciprocal, so the implication survives rounding).  A
    // survivor whose row cannot prune is kept with nothing removed, so the
    // greedy below keeps whole runs of such survivors at once and only reads
    // the rows that can prune.  Lists out of rank order visit every row.
    uint64_t vis[NA];
    if (sorted) {
      const bool v0 = (vm[0] >> lane) & 1ull;
      const double s2 = sw[0] * sc2;
      // 1 / s_j by rank (NaN for empty ranks, whose products are then ignored)
      const float inv = v0 ? (s2 > 0.0 ? (float)(1.0 / s2) : 0.f) : __builtin_nanf("");
      float* invt = sr;  // S(p, .) by slot is no longer needed
      invt[lane] = inv;
      wave_sync();
      float zmin = __builtin_inff();
      const float* myrow = St + lane * SP;
#pragma unroll 4
      for (int j0 = 0; j0 < MS; j0 += 4) {
        const float4 v = *(const float4*)(myrow + j0);
        const float4 iv = *(const float4*)(invt + j0);
        const float z0 = v.x * iv.x, z1 = v.y * iv.y, z2 = v.z * iv.z, z3 = v.w * iv.w;
        zmin = fminf(zmin, j0 + 0 > lane ? z0 : __builtin_inff());
        zmin = fminf(zmin, j0 + 1 > lane ? z1 : __builtin_inff());
        zmin = fminf(zmin, j0 + 2 > lane ? z2 : __builtin_inff());
        zmin = fminf(zmin, j0 + 3 > lane ? z3 : __builtin_inff());
      }
#pragma unroll
      for (int ai = 0; ai < NA; ++ai) {
        float q = v0 ? K[0][ai] * inv : -__builtin_inff();
        for (int off = 32; off > 0; off >>= 1) q = fmaxf(q, __shfl_xor(q, off, 64));
        vis[ai] = __ballot(v0 && zmin <= q);
      }
    } else {
#pragma unroll
      for (int ai = 0; ai < NA; ++ai) vis[ai] = vm[0];
    }

    // Per chain: the survivors before the first survivor i whose row can
    // prune are kept in turn (none removes anything), then i is kept and its
    // row decides the rest; a chain stops at its largest R (trimmed below).
    // Alphas arrive in descending order, so chains visit ever more rows and
    // usually finish in index order: phase s0 advances chains s0..NA-1 while
    // chain s0 has survivors (a finished chain repeats harmless steps).
#pragma unroll
    for (int s0 = 0; s0 < NA; ++s0) {
    while (uniform_u64(alive[s0][0]) != 0) {
      float row[NA];
      int istar[NA];
#pragma unroll
      for (int ai = s0; ai < NA; ++ai) {
        const uint64_t al = uniform_u64(alive[ai][0]);
        int i = ff1_u64(al & vis[ai]);
        const uint64_t upto = i < 0 ? ~0ull : (2ull << i) - 1ull;  // ranks <= i
        const uint64_t batch = al & upto;
        const uint64_t k = uniform_u64(kept[ai][0]) | batch;
        kept[ai][0] = k;
        alive[ai][0] = (i < 0 || __popcll(k) >= rmax[ai]) ? 0ull : al & ~batch;
        i = max(i, 0);
        istar[ai] = i;
        const int slot_i = __builtin_amdgcn_readlane(slotw[0], i);
        row[ai] = St[slot_i * SP + slotw[0]];
      }
      uint64_t amb[NA];
      uint64_t any_amb = 0;
#pragma unroll
      for (int ai = s0; ai < NA; ++ai) {
        const uint64_t pm = __ballot(row[ai] <= P[0][ai]);
        amb[ai] = __ballot(row[ai] <= K[0][ai]) & ~pm & alive[ai][0];
        alive[ai][0] &= ~pm;
        any_amb |= amb[ai];
      }
      if (uniform_u64(any_amb) != 0) {
#pragma unroll
        for (int ai = s0; ai < NA; ++ai) {
          const uint64_t am = uniform_u64(amb[ai]);
          if (am) {
            const int pid = __builtin_amdgcn_readlane(idr[0], istar[ai]);
            bool prune = false;
            if ((am >> lane) & 1ull) {
              const double sx =
                  canon_rows<VEC>(X + (int64_t)pid * d, X + (int64_t)idr[0] * d, d);
              prune = alpha_test_f64(a.num2[ai], a.den2[ai], sx, sw[0]);
            }
            alive[ai][0] &= ~(uint64_t)__ballot(prune);
            rechecks += __popcll(am);
          }
        }
      }
    }
    }
    // a chain that reached its R keeps its first R ranks
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      const uint64_t k = kept[ai][0];
      if (__popcll(k) > rmax[ai]) {
        const int before = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(k >> 32),
                                                          __builtin_amdgcn_mbcnt_lo((uint32_t)k, 0u));
        kept[ai][0] = __ballot(((k >> lane) & 1ull) && before < rmax[ai]);
      }
    }
  } else {
  // One lockstep step advances every chain: keep its lowest survivor i, read
  // row i of S~ (the reads of all chains are in flight together), decide the
  // pairs outside the band, then recheck the pairs inside it.  A finished
  // chain takes i = rank 0, which only re-sets a bit that is already kept or
  // that the final mask with the valid ranks removes.
  for (;;) {
    uint64_t any = 0;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
#pragma unroll
      for (int w = 0; w < NW; ++w) any |= alive[ai][w];
    }
    if (uniform_u64(any) == 0) break;
    float row[NA][NW];
    int istar[NA];
    bool hiw[NA];  // the survivor is in word 1 (ranks 64..127)
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      int i;
      bool w1 = false;
      if (NW == 1) {
        i = ff1_u64(alive[ai][0]);
      } else {
        const int i0 = ff1_u64(alive[ai][0]);
        const int i1 = ff1_u64(alive[ai][NW - 1]);
        w1 = i0 < 0 && i1 >= 0;
        i = w1 ? i1 : i0;
      }
      const bool live = i >= 0;
      i = max(i, 0);
      const uint64_t bit = 1ull << i;
      if (NW == 1) {
        kept[ai][0] |= bit;
        alive[ai][0] &= ~bit;
      } else {
        kept[ai][0] |= w1 ? 0ull : bit;
        alive[ai][0] &= w1 ? ~0ull : ~bit;
        kept[ai][NW - 1] |= w1 ? bit : 0ull;
        alive[ai][NW - 1] &= w1 ? ~bit : ~0ull;
      }
      cnt[ai] += live ? 1 : 0;
      if (cnt[ai] >= rmax[ai]) {  // stop right after the R-th keep
#pragma unroll
        for (int w = 0; w < NW; ++w) alive[ai][w] = 0;
      }
      const int slot_i = __builtin_amdgcn_readlane(w1 ? slotw[NW - 1] : slotw[0], i);
      const float* srow = St + slot_i * SP;
#pragma unroll
      for (int w = 0; w < NW; ++w) row[ai][w] = srow[slotw[w]];
      istar[ai] = i;
      hiw[ai] = w1;
    }
    uint64_t amb[NA][NW];
    uint64_t any_amb = 0;
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
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
#pragma unroll
        for (int w = 0; w < NW; ++w) {
          const uint64_t am = uniform_u64(amb[ai][w]);
          if (am) {
            const int pid =
                __builtin_amdgcn_readlane(hiw[ai] ? idr[NW - 1] : idr[0], istar[ai]);
            bool prune = false;
            if ((am >> lane) & 1ull) {
              const double sx =
                  canon_rows<VEC>(X + (int64_t)pid * d, X + (int64_t)idr[w] * d, d);
              prune = alpha_test_f64(a.num2[ai], a.den2[ai], sx, sw[w]);
            }
            alive[ai][w] &= ~(uint64_t)__ballot(prune);
            rechecks += __popcll(am);
          }
        }
      }
    }
  }
  }
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
#pragma unroll
    for (int w = 0; w < NW; ++w) kept[ai][w] &= vm[w];
  }

  // ---- a8: write every output ------------------------------------------------
  const uint64_t below = (1ull << lane) - 1ull;
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    int tot_k = 0;
    int before[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      before[w] = tot_k;
      tot_k += __popcll(kept[ai][w]);
    }
    for (int ir = 0; ir < fa.nr; ++ir) {
      const SweepOut& out = a.out[ai * fa.nr + ir];
      const int R = out.R;
      const int cntR = tot_k < R ? tot_k : R;
      int32_t* orow = out.nbr + p * R;
#pragma unroll
      for (int w = 0; w < NW; ++w) {
        const uint64_t km = kept[ai][w];
        const int pos = before[w] + __popcll(km & below);
        if (((km >> lane) & 1ull) && pos < R) orow[pos] = idr[w];
      }
      for (int t = cntR + lane; t < R; t += 64) orow[t] = -1;
      if (lane == 0) out.deg[p] = cntR;
    }
  }
  if (lane == 0 && rechecks) atomicAdd(&ctr->rechecks, rechecks);
}

}  // namespace

// the register-streaming kernel (k_prune_f32_reg.hip) for out-lists of at most
// 64 ids with 16-byte row slices; this one for the other shapes
bool prune_f32r_supported(const GraphView& g);
int prune_f32r_wave_lds(const GraphView& g);
hipError_t launch_prune_f32r(const GraphView& g, const SweepArgs& a, F32Args fa,
                             DevCounters* ctr, hipStream_t s);
hipError_t launch_gram_error_f32r(const GraphView& g, const SweepArgs& a, F32Args fa,
                                  DevCounters* ctr, hipStream_t s);

int prune_f32_wave_lds(const GraphView& g) {
  if (prune_f32r_supported(g)) return prune_f32r_wave_lds(g);
  return g.r_max > 64 ? Shape<3>::LDS_B : Shape<2>::LDS_B;
}

bool prune_f32_supported(const GraphView& g) {
  return g.dtype == RP_F32 && g.r_max <= 96 && g.n <= (1ll << 25) && g.maxabs != nullptr;
}

template <int NB, bool CSUM, bool VEC>
static hipError_t launch_shape(const GraphView& g, const SweepArgs& a, const F32Args& fa,
                               DevCounters* ctr, hipStream_t s) {
  const int waves =
      waves_for(TuneKey{kKernelF32, g.dtype, g.d, g.r_max, a.n_alpha, a.n_out}, Shape<NB>::LDS_B);
  const size_t shmem = (size_t)Shape<NB>::LDS_B * waves;
  dim3 grid((unsigned)((g.n + waves - 1) / waves)), block(64 * waves);
#define RP_LAUNCH_F32(NA_)                                                                  \
  case NA_:                                                                                 \
    hipLaunchKernelGGL((prune_f32_kernel<NA_, NB, CSUM, VEC>), grid, block, shmem, s, g, a, \
                       fa, ctr);                                                            \
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
static hipError_t launch_diag(const GraphView& g, const SweepArgs& a, const F32Args& fa,
                              DevCounters* ctr, hipStream_t s) {
  const size_t shmem = Shape<NB>::LDS_B;
  hipLaunchKernelGGL((prune_f32_kernel<1, NB, CSUM, VEC, true>), dim3((unsigned)fa.n_nodes),
                     dim3(64), shmem, s, g, a, fa, ctr);
  return hipGetLastError();
}

template <bool VEC>
static hipError_t diag_vec(const GraphView& g, const SweepArgs& a, F32Args& fa, DevCounters* ctr,
                           hipStream_t s) {
  if (g.r_max > 64) {
    f32_bound_constants(g.d, true, &fa.c1, &fa.c2, &fa.c3);
    return launch_diag<3, true, VEC>(g, a, fa, ctr, s);
  }
  if (g.d > 128) {
    f32_bound_constants(g.d, true, &fa.c1, &fa.c2, &fa.c3);
    return launch_diag<2, true, VEC>(g, a, fa, ctr, s);
  }
  f32_bound_constants(g.d, false, &fa.c1, &fa.c2, &fa.c3);
  return launch_diag<2, false, VEC>(g, a, fa, ctr, s);
}

template <bool VEC>
static hipError_t launch_vec(const GraphView& g, const SweepArgs& a, F32Args& fa,
                             DevCounters* ctr, hipStream_t s) {
  if (g.r_max > 64) {
    f32_bound_constants(g.d, true, &fa.c1, &fa.c2, &fa.c3);
    return launch_shape<3, true, VEC>(g, a, fa, ctr, s);
  }
  if (g.d > 128) {
    f32_bound_constants(g.d, true, &fa.c1, &fa.c2, &fa.c3);
    return launch_shape<2, true, VEC>(g, a, fa, ctr, s);
  }
  f32_bound_constants(g.d, false, &fa.c1, &fa.c2, &fa.c3);
  return launch_shape<2, false, VEC>(g, a, fa, ctr, s);
}

hipError_t launch_gram_error_f32(const GraphView& g, const int32_t* nodes, int64_t n_nodes,
                                GramErrorStats* stats, DevCounters* ctr, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
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
  if (prune_f32r_supported(g)) return launch_gram_error_f32r(g, a, fa, ctr, s);
  const bool vec = (g.d % 4) == 0 && (((uintptr_t)g.X) & 15) == 0;
  return vec ? diag_vec<true>(g, a, fa, ctr, s) : diag_vec<false>(g, a, fa, ctr, s);
}

hipError_t launch_prune_f32(const GraphView& g, const SweepArgs& a_in, DevCounters* ctr,
                            hipStream_t s) {
  if (a_in.n_alpha < 1 || a_in.n_out % a_in.n_alpha != 0) return hipErrorInvalidValue;
  F32Args fa = {};
  fa.nr = a_in.n_out / a_in.n_alpha;
  // the kernel takes the alphas in descending order
  const SweepArgs a = alphas_descending(a_in, fa.nr);
  if (prune_f32r_supported(g)) return launch_prune_f32r(g, a, fa, ctr, s);
  const bool vec = (g.d % 4) == 0 && (((uintptr_t)g.X) & 15) == 0;
  return vec ? launch_vec<true>(g, a, fa, ctr, s) : launch_vec<false>(g, a, fa, ctr, s);
}

}  // namespace rp
