// rp_internal.h -- shared definitions of the HIP library (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rp.h"

namespace rp {

constexpr int kWave = 64;           // CDNA wavefront width
constexpr int kMaxRmax = 256;       // largest stored out-degree r_max
constexpr int kMaxDim = 4096;       // largest point dimension
constexpr int kMaxAlphas = 8;       // alphas per sweep
constexpr int kMaxRs = 4;           // degree bounds per sweep
constexpr int kMaxOutputs = kMaxAlphas * kMaxRs;
constexpr int kMaxL = 1024;         // largest search list size

// Device-side counters (mirrors rp_counters).
struct DevCounters {
  unsigned long long rechecks;  // canonical FP64 re-evaluations
  unsigned long long errors;    // adjacency validation failures
};

// One sweep output: alpha as (num^2, den^2) and its degree bound / buffers.
struct SweepOut {
  int32_t* nbr;
  int32_t* deg;
  int32_t R;
  int32_t alpha_idx;
};

struct SweepArgs {
  uint32_t num2[kMaxAlphas];
  uint32_t den2[kMaxAlphas];
  double ratio[kMaxAlphas];  // den^2 / num^2 rounded to FP64 (a first guess only)
  int32_t n_alpha;
  int32_t n_out;
  SweepOut out[kMaxOutputs];
};

struct GraphView {
  const void* X;
  int32_t dtype;
  int64_t n;
  int32_t d;
  const int32_t* nbr;
  const int32_t* deg;
  int32_t r_max;
  int32_t start;
  const uint32_t* norms;  // |x|^2 per point (uint8 points; library-owned), else null
  const float* maxabs;    // max_k |x_k| per point (float32 points; library-owned), else null
};

// Kernel launchers (each returns hipGetLastError() of its launch).
hipError_t launch_validate(const GraphView& g, DevCounters* ctr, hipStream_t s);
hipError_t launch_norms_u8(const GraphView& g, uint32_t* norms, hipStream_t s);
hipError_t launch_maxabs_f32(const GraphView& g, float* maxabs, hipStream_t s);
hipError_t launch_prune_plain(const GraphView& g, uint32_t num2, uint32_t den2, int32_t R,
                              int32_t* out_nbr, int32_t* out_deg, DevCounters* ctr,
                              hipStream_t s);
hipError_t launch_prune_batched(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                                hipStream_t s);
hipError_t launch_search(const GraphView& g, const void* Q, int64_t nq, int32_t k, int32_t L,
                         int32_t* out_ids, double* out_dist, int32_t* out_hops,
                         hipStream_t s);

// FP32 direct-difference distance bound: |S~ - S| <= gamma_{d+2} S for a
// sequential fmaf accumulation of squared FP32 differences; doubled and
// widened to cover the canonical FP64 value's own error and the FP64
// arithmetic of the comparison.
inline double f32_rel_bound(int d) {
  const double u = 5.9604644775390625e-08;  // 2^-24
  const double g = (d + 2) * u / (1.0 - (d + 2) * u);
  return 2.0 * g + 4e-12;
}

}  // namespace rp
