// k_prune_f32.hip -- batched RP-Tuning for float32 points: FP16 MFMA Gram tile
// with a rigorous rounding bound and a canonical FP64 recheck.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep (out-lists of at most 64 ids, any d):
//
//  a1  read:   lane t holds the t-th listed id.
//  a3  p-row:  lane j evaluates the canonical FP64 S(p, j) (sequential fma
//              chain over k) from its own row -- the exact sort key.
//  a4  sort:   bitonic sort of (S(p, j) bits, id, slot) over the 64 lanes;
//              p and repeated ids are dropped.
//  a2  gather: the rows are staged d-chunk by d-chunk in LDS as FP16
//              u = (x - x_p) * 2^e (p-centred, power-of-two scaled so that
//              |u| < 2^14), with coalesced 16-byte loads.
//  a5  Gram:   G~ = U U^T on v_mfma_f32_32x32x16_f16 (FP32 accumulation),
//              upper blocks only; S~(i, j) = (S(p,i) + S(p,j)) 2^2e - 2 G~(i, j)
//              goes to an FP32 LDS tile.  In the centred frame the error of
//              S~ is bounded by E_j ~ (4 u16 + 2 gamma_d) S(p, j) 2^2e (the
//              later rank j has the larger S(p, .)).
//  a6  test:   the pruning condition as defined for float32 data,
//              fl(num^2 S(i,j)) <= fl(den^2 S(p,j)), is decided from S~ when
//              S~ lies outside [P_j, K_j], thresholds that include E_j and
//              the FP64 rounding of both products; pairs inside the band are
//              recomputed in canonical FP64 from the float32 rows.
//  a7  greedy: 64-bit survivor masks, all alphas in lockstep (as for uint8).
//  a8  write:  popcount scatter of the kept ranks, -1 padded.
#include "dev_common.h"

namespace rp {

typedef _Float16 v8h __attribute__((ext_vector_type(8)));
typedef float v16f __attribute__((ext_vector_type(16)));

namespace {

constexpr int kChunk = 128;                         // dimensions per LDS chunk
constexpr int kUStride = kChunk * 2 + 16;           // bytes per FP16 row in the chunk
constexpr int kUBytes = 64 * kUStride;              // 17,408
constexpr int kSTileBytesF = (32 * 64 + 32 * 32) * 4;  // 12,288

__device__ __forceinline__ uint64_t shfl_u64f(uint64_t v, int src) {
  int lo = __shfl((int)(uint32_t)v, src, 64);
  int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Ascending bitonic sort of (hi, lo) pairs across the wavefront.
__device__ __forceinline__ void wave_sort2(uint64_t& hi, uint32_t& lo, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      int ohl = __shfl_xor((int)(uint32_t)hi, j, 64);
      int ohh = __shfl_xor((int)(uint32_t)(hi >> 32), j, 64);
      uint32_t olo = (uint32_t)__shfl_xor((int)lo, j, 64);
      uint64_t ohi = ((uint64_t)(uint32_t)ohh << 32) | (uint32_t)ohl;
      bool mine_less = hi < ohi || (hi == ohi && lo < olo);
      bool up = (lane & k) == 0;
      bool lower = (lane & j) == 0;
      bool take_min = lower == up;
      bool keep_mine = take_min ? mine_less : !mine_less;
      if (!keep_mine) {
        hi = ohi;
        lo = olo;
      }
    }
  }
}

// Next float toward -inf / +inf (finite inputs).
__device__ __forceinline__ float next_down(float f) {
  if (f == 0.f) return -1.401298464e-45f;
  int b = __float_as_int(f);
  return __int_as_float(f > 0.f ? b - 1 : b + 1);
}

__device__ __forceinline__ float next_up(float f) {
  if (f == 0.f) return 1.401298464e-45f;
  int b = __float_as_int(f);
  return __int_as_float(f > 0.f ? b + 1 : b - 1);
}

// FP32 value <= x (round down) and >= x (round up).
__device__ __forceinline__ float f32_down(double x) {
  float f = (float)x;
  if ((double)f > x) f = next_down(f);
  return f;
}

__device__ __forceinline__ float f32_up(double x) {
  float f = (float)x;
  if ((double)f < x) f = next_up(f);
  return f;
}

template <int NA>
__global__ __launch_bounds__(64) void prune_f32_kernel(GraphView g, SweepArgs a, double c1,
                                                       double c2, double c3, DevCounters* ctr) {
  extern __shared__ __align__(16) uint8_t lds[];
  const int lane = threadIdx.x;
  const int64_t p = blockIdx.x;
  const int d = g.d;
  const float* X = (const float*)g.X;
  uint8_t* Ubytes = lds;                              // FP16 chunk tile
  float* Stile = (float*)lds;                         // overlays the chunk tile after the Gram
  const int tile_bytes = kUBytes > kSTileBytesF ? kUBytes : kSTileBytesF;
  float* xp = (float*)(lds + tile_bytes);             // x_p chunk (kChunk floats)
  float* sr = xp + kChunk;                            // S(p, .) * 2^2e by rank (FP32)
  int32_t* idl = (int32_t*)(sr + 64);                 // listed ids by slot

  // ---- a1 ------------------------------------------------------------------
  const int m = g.deg[p];
  const int id = lane < m ? g.nbr[p * g.r_max + lane] : -1;
  idl[lane] = id;

  // ---- a3: canonical FP64 S(p, j) -----------------------------------------
  const float* xprow = X + p * d;
  double s = 0.0;
  if (id >= 0 && id != (int)p) s = canon_sq_f32(xprow, X + (int64_t)id * d, d);

  // ---- a4: sort by (S(p, j), id) ---------------------------------------------
  const bool listed = id >= 0 && id != (int)p;
  uint64_t khi = listed ? (uint64_t)__double_as_longlong(s) : ~0ull;
  uint32_t klo = listed ? (((uint32_t)id << 6) | (uint32_t)lane) : ~0u;
  wave_sort2(khi, klo, lane);
  {
    uint64_t phi = shfl_u64f(khi, lane > 0 ? lane - 1 : 0);
    uint32_t plo = (uint32_t)__shfl((int)klo, lane > 0 ? lane - 1 : 0, 64);
    bool dup = lane > 0 && khi != ~0ull && khi == phi && (klo >> 6) == (plo >> 6);
    if (dup) khi = ~0ull - 1;
  }
  const bool valid = khi < ~0ull - 1;
  const uint64_t valid_mask = __ballot(valid);
  const int slot = (int)(klo & 63);
  const double s_rank = valid ? __longlong_as_double((long long)khi) : 0.0;
  const int id_rank = valid ? (int)(klo >> 6) : -1;

  // power-of-two scale: |u_k| <= |u| = sqrt(S(p, j)) <= sqrt(max S) -> < 2^14
  double smax = s_rank;
  for (int off = 32; off > 0; off >>= 1) smax = fmax(smax, __shfl_xor(smax, off, 64));
  int e = 0;
  if (smax > 0.0) {
    int ex;
    frexp(sqrt(smax), &ex);  // sqrt(smax) < 2^ex
    e = 14 - ex;
  }
  const double sc = ldexp(1.0, e);
  const double sc2 = sc * sc;
  sr[lane] = (float)(s_rank * sc2);

  // ---- a2 + a5: chunked gather into FP16 and MFMA ----------------------------
  const int l32 = lane & 31;
  const int half = lane >> 5;
  const int sl0 = __shfl(slot, l32, 64);
  const int sl1 = __shfl(slot, 32 + l32, 64);
  v16f acc00 = {0}, acc01 = {0}, acc11 = {0};
  const float scf = (float)sc;
  for (int c0 = 0; c0 < d; c0 += kChunk) {
    const int dc = min(kChunk, d - c0);
    __syncthreads();  // previous chunk's MFMA reads are done
    for (int k = lane; k < dc; k += 64) xp[k] = xprow[c0 + k];
    __syncthreads();
    // 4 floats (16 B) per lane per load; rows by slot
    const int q4 = (dc + 3) >> 2;
    for (int c = lane; c < 64 * q4; c += 64) {
      const int row = c / q4;
      const int col = (c - row * q4) * 4;
      const int rid = idl[row];
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (rid >= 0) {
        const float* src = X + (int64_t)rid * d + c0 + col;
        if (col + 4 <= dc && ((((uintptr_t)src) & 15) == 0)) {
          v = *(const float4*)src;
        } else {
          if (col + 0 < dc) v.x = src[0];
          if (col + 1 < dc) v.y = src[1];
          if (col + 2 < dc) v.z = src[2];
          if (col + 3 < dc) v.w = src[3];
        }
        v.x = (col + 0 < dc) ? (v.x - xp[col + 0]) * scf : 0.f;
        v.y = (col + 1 < dc) ? (v.y - xp[col + 1]) * scf : 0.f;
        v.z = (col + 2 < dc) ? (v.z - xp[col + 2]) * scf : 0.f;
        v.w = (col + 3 < dc) ? (v.w - xp[col + 3]) * scf : 0.f;
      }
      _Float16* dst = (_Float16*)(Ubytes + row * kUStride) + col;
      dst[0] = (_Float16)v.x;
      dst[1] = (_Float16)v.y;
      dst[2] = (_Float16)v.z;
      dst[3] = (_Float16)v.w;
    }
    // zero the padding up to a multiple of 16 dimensions
    const int dc16 = (dc + 15) & ~15;
    for (int c = lane; c < 64 * (dc16 - 4 * q4); c += 64) {
      const int row = c / (dc16 - 4 * q4);
      const int col = 4 * q4 + (c - row * (dc16 - 4 * q4));
      ((_Float16*)(Ubytes + row * kUStride))[col] = (_Float16)0.f;
    }
    __syncthreads();
    for (int kk = 0; kk < dc16; kk += 16) {
      const int off = (kk + half * 8) * 2;
      v8h f0 = *(const v8h*)(Ubytes + sl0 * kUStride + off);
      v8h f1 = *(const v8h*)(Ubytes + sl1 * kUStride + off);
      acc00 = __builtin_amdgcn_mfma_f32_32x32x16_f16(f0, f0, acc00, 0, 0, 0);
      acc01 = __builtin_amdgcn_mfma_f32_32x32x16_f16(f0, f1, acc01, 0, 0, 0);
      acc11 = __builtin_amdgcn_mfma_f32_32x32x16_f16(f1, f1, acc11, 0, 0, 0);
    }
  }
  __syncthreads();

  // S~ tile (rank order): lane l holds column l % 32 of rows 8(v/4) + 4(l/32) + v%4.
  {
    const float scol0 = sr[l32];
    const float scol1 = sr[32 + l32];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v >> 2) + 4 * half + (v & 3);
      const float srow0 = sr[r];
      const float srow1 = sr[32 + r];
      Stile[r * 64 + l32] = (srow0 + scol0) - 2.f * acc00[v];
      Stile[r * 64 + 32 + l32] = (srow0 + scol1) - 2.f * acc01[v];
      Stile[32 * 64 + r * 32 + l32] = (srow1 + scol1) - 2.f * acc11[v];
    }
  }
  __syncthreads();

  // ---- a6: decision bands per alpha -------------------------------------------
  // E_j: |S~(i, j) - S(i, j) 2^2e| for every i before j (S(p, i) <= S(p, j)).
  const double Ej = c1 * s_rank * sc2 + c2 * sqrt(s_rank) * sc + c3;
  float P[NA], K[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    const double B = (double)a.den2[ai] * s_rank;      // fl(den^2 S(p, j)), as defined
    const double t = B / (double)a.num2[ai];
    const double tlo = t * (1.0 - 0x1p-50);
    const double thi = t * (1.0 + 0x1p-49);
    P[ai] = f32_down(tlo * sc2 - Ej);
    K[ai] = f32_up(thi * sc2 + Ej);
  }

  // ---- a7: greedy ----------------------------------------------------------------
  int rmax[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) rmax[ai] = 0;
  for (int o = 0; o < a.n_out; ++o) {
#pragma unroll
    for (int ai = 0; ai < NA; ++ai)
      if (a.out[o].alpha_idx == ai) rmax[ai] = max(rmax[ai], a.out[o].R);
  }
  uint64_t alive[NA], kept[NA];
  int cnt[NA], cur[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    alive[ai] = valid_mask;
    kept[ai] = 0;
    cnt[ai] = 0;
    cur[ai] = 0;
  }
  unsigned long long rechecks = 0;
  const int col_hi = 32 * 64 + (lane >= 32 ? lane - 32 : lane);
  for (;;) {
    bool any = false;
    float row[NA];
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      row[ai] = 0.f;
      if (alive[ai] != 0 && cnt[ai] < rmax[ai]) {
        const int i = __ffsll((long long)alive[ai]) - 1;
        kept[ai] |= 1ull << i;
        alive[ai] &= ~(1ull << i);
        ++cnt[ai];
        cur[ai] = i;
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
      if (alive[ai] != 0) {
        const uint64_t pm = __ballot(row[ai] <= P[ai]);
        const uint64_t am = __ballot(row[ai] > P[ai] && row[ai] <= K[ai]) & alive[ai];
        alive[ai] &= ~pm;
        if (am) {
          // canonical FP64 for the pairs inside the band
          const int pid = __shfl(id_rank, cur[ai], 64);
          bool prune = false;
          if ((am >> lane) & 1ull) {
            const double sij = canon_sq_f32(X + (int64_t)pid * d, X + (int64_t)id_rank * d, d);
            prune = alpha_test_f64(a.num2[ai], a.den2[ai], sij, s_rank);
          }
          alive[ai] &= ~(uint64_t)__ballot(prune);
          rechecks += __popcll(am);
        }
      }
    }
  }

  // ---- a8: write -----------------------------------------------------------------
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
  if (lane == 0 && rechecks) atomicAdd(&ctr->rechecks, rechecks);
}

}  // namespace

bool prune_f32_supported(const GraphView& g) {
  return g.dtype == RP_F32 && g.r_max <= 64 && g.n <= (1ll << 26);
}

// Bound constants of |S~ - S 2^2e| <= c1 S(p, j) 2^2e + c2 sqrt(S(p, j)) 2^e + c3
// for every rank i before j (so S(p, i) <= S(p, j)):
//   eps   = 2^-11 + 2^-23: rounding of u = (x - x_p) 2^e to FP16 after the FP32
//           subtraction (relative);
//   eps_a = 2^-14: absolute error of an FP16 element near zero, even if the
//           matrix unit flushes subnormal inputs;
//   gamma = gamma_{d+2} (FP32 accumulation of the exact FP16 products);
//   |G~ - G| <= (2 eps + gamma) |u_i||u_j| + eps_a sqrt(d) (|u_i| + |u_j|) + d eps_a^2,
//   and forming S~ = (S(p,i) + S(p,j)) 2^2e - 2 G~ in FP32 adds 8 * 2^-24 S(p,j) 2^2e.
// Every coefficient is doubled; the FP64 threshold's own rounding is covered
// separately by the (1 -/+ 2^-50) factors.
static void f32_bound_constants(int d, double* c1, double* c2, double* c3) {
  const double eps = 0x1p-11 + 0x1p-23;
  const double eps_a = 0x1p-14;
  const double u32 = 0x1p-24;
  const double g = (d + 2) * u32 / (1.0 - (d + 2) * u32);
  *c1 = 2.0 * (4.0 * eps + 2.0 * g * (1.0 + eps) * (1.0 + eps) + 8.0 * u32);
  *c2 = 2.0 * 4.0 * eps_a * (1.0 + eps) * (1.0 + g) * sqrt((double)d);
  *c3 = 2.0 * 2.0 * d * eps_a * eps_a * (1.0 + g);
}

hipError_t launch_prune_f32(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                            hipStream_t s) {
  double c1, c2, c3;
  f32_bound_constants(g.d, &c1, &c2, &c3);
  const int tile = kUBytes > kSTileBytesF ? kUBytes : kSTileBytesF;
  const size_t shmem = (size_t)tile + kChunk * 4 + 64 * 4 + 64 * 4;
  dim3 grid((unsigned)g.n), block(64);
#define RP_LAUNCH_F32(NA_)                                                                    \
  case NA_:                                                                                   \
    hipLaunchKernelGGL(prune_f32_kernel<NA_>, grid, block, shmem, s, g, a, c1, c2, c3, ctr); \
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

}  // namespace rp
