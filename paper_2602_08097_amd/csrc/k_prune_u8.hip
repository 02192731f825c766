// k_prune_u8.hip -- batched RP-Tuning for uint8 points on int8 MFMA.
//
// One wavefront runs RobustPrune(p, N_out(p), alpha, R) (Algorithm 1) for one
// vertex p at every alpha of a sweep from a single gather of the candidate
// rows.  For out-lists of at most 64 ids and d a multiple of 16 (d <= 256):
//
//  a1  read:   lane t holds the t-th listed id.
//  a2  gather: coalesced 16-byte loads, d/16 consecutive lanes per row, all
//              of a lane's loads in flight together, stored to LDS as int8
//              u = x - 128 (the shift leaves every difference unchanged).
//  a3  p-row:  S(p, j) = |u_p|^2 + |u_j|^2 - 2 <u_p, u_j>, exact in int32,
//              with 4-way int8 dot products.
//  a4  sort:   a 64-lane bitonic sort of keys (S(p, j), id, slot) packed in
//              64 bits, lane exchanges by DPP and swizzles.  The repeated
//              argmin of Algorithm 1 over a shrinking candidate set visits the
//              candidates in this order; p and repeated ids are dropped.
//  a5  Gram:   G = U U^T over the rank-ordered rows on
//              v_mfma_i32_32x32x32_i8 (exact int32 accumulation); blocks on
//              and above the diagonal only; S(i, j) = |u_i|^2 + |u_j|^2
//              - 2 G(i, j) is written to a 12 KiB LDS tile.
//  a6  test:   alpha * D(p*, p') <= D(p, p') on squares is
//              num^2 S(p*, p') <= den^2 S(p, p')  <=>  S(p*, p') <= T(p'),
//              T(p') = floor(den^2 S(p, p') / num^2), exact for integer S.
//  a7  greedy: per alpha a 64-bit survivor mask; p* = lowest surviving rank
//              is kept, its S row is read from LDS and one ballot of
//              S(p*, .) <= T removes p* itself (S = 0) and every candidate it
//              prunes.  All alphas advance in lockstep without branches, so
//              their LDS reads are in flight together.  A chain stops at the
//              largest R requested for its alpha; a smaller R is a prefix.
//  a8  write:  kept ranks are scattered to their positions (popcount of the
//              kept ranks before them), -1 padded.
#include "dev_common.h"

namespace rp {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

namespace {

constexpr int kSTileBytes = 3072;  // count tile, 3 KiB: the blocks on and above the diagonal
constexpr int kMaxDimU8 = 256;
constexpr int kGatherBatch = 9;  // 16-byte loads in flight per lane (65 rows x 128 B = 520)

__host__ __device__ constexpr int u_stride(int d) { return d + 16; }


// floor(den2 * s / num2) for s < 2^28, exact: s * fl(den2 / num2) is within
// 2^-24 of the quotient, so one integer correction step settles it.
__device__ __forceinline__ int32_t alpha_threshold(uint32_t num2, uint32_t den2, double ratio,
                                                   uint32_t s) {
  const uint64_t B = (uint64_t)den2 * s;
  uint32_t t = (uint32_t)((double)s * ratio);
  const uint64_t nt = (uint64_t)num2 * t;
  if (nt > B) t -= 1;
  else if (nt + num2 <= B) t += 1;
  return (int32_t)t;
}

// ---------------------------------------------------------------------------
// Per-vertex pieces of the kernel.
// ---------------------------------------------------------------------------

struct Tile {
  int8_t* U;        // candidate rows (slot order) + x_p, as u = x - 128
  uint8_t* C;       // count tile (overlays U after the Gram)
  int32_t* nr;      // |u|^2 by rank
  int stride;       // bytes per U row
};

__device__ __forceinline__ Tile make_tile(uint8_t* lds, int d) {
  Tile t;
  t.stride = u_stride(d);
  t.U = (int8_t*)lds;
  t.C = lds;
  const int tile_bytes = max(65 * t.stride, kSTileBytes);
  t.nr = (int32_t*)(lds + tile_bytes);
  return t;
}

// a1: the list of p (row and degree loads in flight together).
__device__ __forceinline__ int load_list(const GraphView& g, int64_t p, int lane) {
  const int raw = lane < g.r_max ? g.nbr[p * g.r_max + lane] : -1;
  const int m = g.deg[p];
  return lane < m ? raw : -1;
}

// Chunk c of the gather (c = lane + 64 t): row c / cpr (64 = x_p), 16-byte column c % cpr.
__device__ __forceinline__ void chunk_pos(int c, int cpr, float inv_cpr, int& row, int& col) {
  row = (int)(((float)c + 0.5f) * inv_cpr);
  col = c - row * cpr;
}

struct Front {
  uint64_t valid_mask;
  int id_rank;
};

// a3..a6 on rows already in the U tile: p-row, sort, Gram, thresholds and the
// count tile.  Alphas arrive in ascending order, so their thresholds
// T_0(j) >= T_1(j) >= ... and the alphas whose test holds for a pair (i, j)
// are a prefix 0..c-1; the tile stores c(i, j) = #{k : S(i, j) <= T_k(j)} and
// chain k prunes j from i exactly when c(i, j) > k.
template <int NA>
__device__ __forceinline__ Front node_front(const Tile& tl, const SweepArgs& a, int d, int64_t p,
                                            int id, int lane, int idbits) {
  const int stride = tl.stride;
  // ---- a3: p-row S(p, j) and |u_j|^2 -------------------------------------
  int32_t nj = 0, dotp = 0, np = 0;
  {
    const int8_t* uj = tl.U + lane * stride;
    const int8_t* up = tl.U + 64 * stride;
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
  // A list already in (S, id) order -- every RobustPrune output is -- skips
  // the sorting network.
  uint64_t prev = shfl_u64(key, lane > 0 ? lane - 1 : 0);
  if (__ballot(lane > 0 && key < prev)) {
    key = wave_sort(key, lane);
    prev = shfl_u64(key, lane > 0 ? lane - 1 : 0);
  }
  {
    const bool dup = lane > 0 && key != kInvalid && (key >> 6) == (prev >> 6);
    if (dup) key = kInvalid - 1;  // never alive
  }
  const bool valid = key < kInvalid - 1;
  Front f;
  f.valid_mask = __ballot(valid);
  const int slot = (int)(key & 63);
  const uint32_t s_rank = valid ? (uint32_t)(key >> shift) : 0u;
  f.id_rank = valid ? (int)((key >> 6) & ((1ull << idbits) - 1)) : -1;
  tl.nr[lane] = __shfl(nj, slot, 64);

  // ---- a6: thresholds of this rank, then of the lane's two tile columns ---
  const int l32 = lane & 31;
  const int half = lane >> 5;
  int32_t T0[NA], T1[NA];
#pragma unroll
  for (int k = 0; k < NA; ++k) {
    const int32_t t = alpha_threshold(a.num2[k], a.den2[k], a.ratio[k], s_rank);
    T0[k] = __shfl(t, l32, 64);        // column l32
    T1[k] = __shfl(t, 32 + l32, 64);   // column 32 + l32
  }

  // ---- a5: Gram tile on MFMA (rank order) -------------------------------
  const int sl0 = __shfl(slot, l32, 64);        // row of rank l32
  const int sl1 = __shfl(slot, 32 + l32, 64);   // row of rank 32 + l32
  v16i acc00 = {0}, acc01 = {0}, acc11 = {0};
  const int d32 = (d + 31) & ~31;
  for (int kk = 0; kk < d32; kk += 32) {
    const int off = kk + half * 16;
    v4i f0 = {0, 0, 0, 0}, f1 = {0, 0, 0, 0};
    if (off < d) {
      f0 = *(const v4i*)(tl.U + sl0 * stride + off);
      f1 = *(const v4i*)(tl.U + sl1 * stride + off);
    }
    acc00 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0, f0, acc00, 0, 0, 0);
    acc01 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f0, f1, acc01, 0, 0, 0);
    acc11 = __builtin_amdgcn_mfma_i32_32x32x32_i8(f1, f1, acc11, 0, 0, 0);
  }
  wave_sync();  // every U read is done before the count tile overwrites it

  // Count tile, 3072 bytes: columns 0..31 of rows 0..31 at byte 32 i + c;
  // columns 32..63 of rows 0..63 at byte 1024 + 32 i + (c - 32).  Row i is
  // then read by lane c at byte 32 i + (c % 32) + 1024 (c / 32).
  // Accumulator layout of a 32 x 32 block: lane l holds column l % 32 of rows
  // 8 (v / 4) + 4 (l / 32) + v % 4 in register v.
  {
    const int32_t ncol0 = tl.nr[l32];
    const int32_t ncol1 = tl.nr[32 + l32];
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const int r = 8 * (v >> 2) + 4 * half + (v & 3);
      const int32_t nrow0 = tl.nr[r];
      const int32_t nrow1 = tl.nr[32 + r];
      const int32_t s00 = nrow0 + ncol0 - 2 * acc00[v];
      const int32_t s01 = nrow0 + ncol1 - 2 * acc01[v];
      const int32_t s11 = nrow1 + ncol1 - 2 * acc11[v];
      uint32_t c00 = 0, c01 = 0, c11 = 0;
#pragma unroll
      for (int k = 0; k < NA; ++k) {
        c00 += (uint32_t)(s00 <= T0[k]);
        c01 += (uint32_t)(s01 <= T1[k]);
        c11 += (uint32_t)(s11 <= T1[k]);
      }
      asm("" : "+v"(c00), "+v"(c01), "+v"(c11));  // keep the counts 32-bit (carry adds)
      tl.C[r * 32 + l32] = (uint8_t)c00;
      tl.C[1024 + r * 32 + l32] = (uint8_t)c01;
      tl.C[1024 + (32 + r) * 32 + l32] = (uint8_t)c11;
    }
  }
  return f;
}

// a7 + a8 on the count tile: greedy, outputs of p.
template <int NA, int NR, bool CAP>
__device__ __forceinline__ void node_back(const Tile& tl, const SweepArgs& a, int64_t p,
                                          const Front& f, int lane) {
  // ---- a7: greedy keep / discard, all alphas in lockstep ----------------
  // outputs are alpha-major: output ai * NR + ir has alpha ai, bound R_ir
  int rmax[NA];
  if (CAP) {
#pragma unroll
    for (int ai = 0; ai < NA; ++ai) {
      rmax[ai] = 0;
#pragma unroll
      for (int ir = 0; ir < NR; ++ir) rmax[ai] = max(rmax[ai], a.out[ai * NR + ir].R);
    }
  }
  uint64_t alive[NA], kept[NA];
  int cnt[NA];
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    alive[ai] = f.valid_mask;
    kept[ai] = 0;
    cnt[ai] = 0;
  }
  const int lbase = (lane & 31) + 1024 * (lane >> 5);
  // Chain k steps: keep its lowest survivor i, read row i of the count tile,
  // drop i itself (its count passes every threshold) and what it prunes.
  // Phase s advances chains s..NA-1 in lockstep while chain s has survivors;
  // chains are in ascending alpha and usually finish in that order, so the
  // phases skip most steps of finished chains (a chain that finishes early
  // only repeats harmless steps on an empty mask).
#pragma unroll
  for (int s0 = 0; s0 < NA; ++s0) {
    while (alive[s0] != 0) {
      uint32_t row[NA];
#pragma unroll
      for (int ai = s0; ai < NA; ++ai) {
        // s_ff1 gives -1 for an empty mask; clamping to rank 0 then only
        // re-sets a bit that is already kept, or that the final mask with
        // the valid ranks removes.
        const uint64_t al = uniform_u64(alive[ai]);
        int i;
        asm("s_ff1_i32_b64 %0, %1" : "=s"(i) : "s"(al));
        i = max(i, 0);
        uint64_t k = uniform_u64(kept[ai]);
        asm("s_bitset1_b64 %0, %1" : "+s"(k) : "s"(i));
        kept[ai] = k;
        if (CAP) {
          cnt[ai] += al != 0 ? 1 : 0;
          if (cnt[ai] >= rmax[ai]) alive[ai] = 0;        // stop right after the R-th keep
        }
        row[ai] = tl.C[i * 32 + lbase];
      }
#pragma unroll
      for (int ai = s0; ai < NA; ++ai)
        alive[ai] &= ~(uint64_t)__ballot(row[ai] > (uint32_t)ai);
    }
  }
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) kept[ai] &= f.valid_mask;

  // ---- a8: write every output -------------------------------------------
#pragma unroll
  for (int ai = 0; ai < NA; ++ai) {
    const uint64_t km = kept[ai];
    const int tot = __popcll(km);
    const bool mine = (km >> lane) & 1ull;
    const int pos = __popcll(km & ((1ull << lane) - 1ull));
#pragma unroll
    for (int ir = 0; ir < NR; ++ir) {
      const SweepOut& out = a.out[ai * NR + ir];
      const int R = out.R;
      const int cntR = tot < R ? tot : R;
      int32_t* orow = out.nbr + p * R;
      if (mine && pos < R) orow[pos] = f.id_rank;
      for (int t = cntR + lane; t < R; t += 64) orow[t] = -1;
      if (lane == 0) out.deg[p] = cntR;
    }
  }
}

// One wavefront per vertex (any d multiple of 16 up to 256), blockDim.x / 64
// vertices per workgroup, each wavefront with its own `wave_lds` bytes of LDS.
template <int NA, int NR, bool CAP>
__global__ __launch_bounds__(512) void prune_u8_kernel(GraphView g, SweepArgs a, int32_t idbits,
                                                       int32_t wave_lds) {
  extern __shared__ __align__(16) uint8_t lds_all[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (p >= g.n) return;
  uint8_t* lds = lds_all + (size_t)wave * wave_lds;
  const int d = g.d;
  const Tile tl = make_tile(lds, d);
  int32_t* idl = tl.nr + 64;  // listed ids by slot, then p
  const uint8_t* X = (const uint8_t*)g.X;

  const int id = load_list(g, p, lane);
  idl[lane] = id;
  if (lane == 0) idl[64] = (int)p;
  wave_sync();

  // ---- a2: coalesced gather into LDS (u = x - 128) -----------------------
  // Every load of a batch is issued before any of its stores.
  {
    const int cpr = d >> 4;
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
          int row, col;
          chunk_pos(c, cpr, inv_cpr, row, col);
          const int rid = idl[row];
          dst[t] = row * tl.stride + col * 16;
          if (rid >= 0) buf[t] = *(const uint4*)(X + (int64_t)rid * d + col * 16);
        }
      }
#pragma unroll
      for (int t = 0; t < kGatherBatch; ++t) {
        if (dst[t] >= 0) {
          uint4 v = buf[t];
          v.x ^= 0x80808080u; v.y ^= 0x80808080u; v.z ^= 0x80808080u; v.w ^= 0x80808080u;
          *(uint4*)(tl.U + dst[t]) = v;
        }
      }
    }
  }
  wave_sync();
  const Front f = node_front<NA>(tl, a, d, p, id, lane, idbits);
  wave_sync();
  node_back<NA, NR, CAP>(tl, a, p, f, lane);
}

struct Launch {
  int idbits;
  int wave_lds;  // LDS bytes per wavefront
  int waves;     // vertices per workgroup
};

template <int NA, int NR>
hipError_t launch_nr(const GraphView& g, const SweepArgs& a, const Launch& L, hipStream_t s) {
  bool cap = false;
  for (int o = 0; o < a.n_out; ++o) cap = cap || a.out[o].R < g.r_max;
  const dim3 grid((unsigned)((g.n + L.waves - 1) / L.waves)), block(64 * L.waves);
  const size_t shmem = (size_t)L.wave_lds * L.waves;
  if (cap)
    hipLaunchKernelGGL((prune_u8_kernel<NA, NR, true>), grid, block, shmem, s, g, a, L.idbits,
                       L.wave_lds);
  else
    hipLaunchKernelGGL((prune_u8_kernel<NA, NR, false>), grid, block, shmem, s, g, a, L.idbits,
                       L.wave_lds);
  return hipGetLastError();
}

template <int NA>
hipError_t launch_na(const GraphView& g, const SweepArgs& a, const Launch& L, hipStream_t s) {
  switch (a.n_out / NA) {
    case 1: return launch_nr<NA, 1>(g, a, L, s);
    case 2: return launch_nr<NA, 2>(g, a, L, s);
    case 3: return launch_nr<NA, 3>(g, a, L, s);
    case 4: return launch_nr<NA, 4>(g, a, L, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

int prune_u8_wave_lds(const GraphView& g) {
  const int stride = u_stride(g.d);
  return (max(65 * stride, kSTileBytes) + (64 + 68) * (int)sizeof(int32_t) + 15) & ~15;
}

bool prune_u8_supported(const GraphView& g) {
  return g.dtype == RP_U8 && g.r_max <= 64 && (g.d % 16) == 0 && g.d <= kMaxDimU8 &&
         g.n <= (1ll << 30);
}

hipError_t launch_prune_u8(const GraphView& g, const SweepArgs& a_in, DevCounters* ctr,
                           hipStream_t s) {
  (void)ctr;
  // the kernel takes the alphas in ascending order (num_a den_b vs num_b den_a)
  SweepArgs a = a_in;
  int order[kMaxAlphas];
  for (int i = 0; i < a_in.n_alpha; ++i) order[i] = i;
  for (int i = 1; i < a_in.n_alpha; ++i) {
    int v = order[i], j = i - 1;
    // compare alpha_v < alpha_order[j] on squares: num2_v den2_o < num2_o den2_v
    while (j >= 0 && (uint64_t)a_in.num2[v] * a_in.den2[order[j]] <
                         (uint64_t)a_in.num2[order[j]] * a_in.den2[v]) {
      order[j + 1] = order[j];
      --j;
    }
    order[j + 1] = v;
  }
  // outputs are alpha-major (o = alpha * n_R + iR); permute them with the alphas
  const int nr = a_in.n_out / a_in.n_alpha;
  for (int k = 0; k < a_in.n_alpha; ++k) {
    a.num2[k] = a_in.num2[order[k]];
    a.den2[k] = a_in.den2[order[k]];
    a.ratio[k] = a_in.ratio[order[k]];
    for (int ir = 0; ir < nr; ++ir) {
      a.out[k * nr + ir] = a_in.out[order[k] * nr + ir];
      a.out[k * nr + ir].alpha_idx = k;
    }
  }
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
