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
  double ratio[kMaxAlphas];  // den^2 / num^2 rounded to FP64 (float32 kernels)
  // FP32 bounds of den^2 / num^2 below and above (float32 kernel; set by its launcher)
  float ratio_dn[kMaxAlphas];
  float ratio_up[kMaxAlphas];
  // floor(2^60 den^2 / num^2) + 1 (uint8 kernel; set by its launcher)
  uint64_t thr_mul[kMaxAlphas];
  int32_t n_alpha;
  int32_t n_out;
  // 0: RobustPrune (candidates in ascending (S(p, .), id) order); 1:
  // UnsortedRobustPrune (candidates in stored list order, first occurrence of
  // a repeated id)
  int32_t unsorted;
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
  // per vertex, the power-of-two scale exponent of the vertex's frame for the
  // float32 prune (from its own list and max|x|; library-owned), else null
  const int8_t* frame_e;
};

// Measured error of the float32 kernel's approximate distances (device).
struct GramErrorStats {
  double max_rel;    // max |S~ - S| / S over candidate pairs with S > 0
  double sum_rel;
  unsigned long long pairs;
  double max_band;   // max |S~ - S| / E_j: the proven bound holds while this is <= 1
};

// One query of a batched search: its row and its outputs (device pointers;
// dist and hops nullable).
struct SearchJob {
  const void* q;
  int32_t* ids;
  double* dist;
  int32_t* hops;
};

// Kernel launchers (each returns hipGetLastError() of its launch).
hipError_t launch_validate(const GraphView& g, DevCounters* ctr, hipStream_t s);
hipError_t launch_norms_u8(const GraphView& g, uint32_t* norms, hipStream_t s);
hipError_t launch_maxabs_f32(const GraphView& g, float* maxabs, DevCounters* ctr, hipStream_t s);
hipError_t launch_frame_exponents_f32(const GraphView& g, int8_t* e, hipStream_t s);
hipError_t launch_prune_plain(const GraphView& g, uint32_t num2, uint32_t den2, int32_t R,
                              int32_t* out_nbr, int32_t* out_deg, DevCounters* ctr,
                              hipStream_t s, bool unsorted = false);
hipError_t launch_prune_batched(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                                hipStream_t s);
hipError_t launch_gram_error_f32(const GraphView& g, const int32_t* nodes, int64_t n_nodes,
                                 GramErrorStats* stats, DevCounters* ctr, hipStream_t s);
// Exact K-NN of uint8 points (k_knn_u8.hip): supported dimensions, the number
// of candidate slices for a call, the workspace those slices need (0 for one
// slice), and the launch.
rp_status knn_args(const uint8_t* points, int64_t n, int32_t d, const int32_t* query_ids,
                   int64_t nq, const int32_t* cand_ids, int64_t nc, int32_t K,
                   const int32_t* out_ids);
bool knn_u8_supported(int d);
int knn_u8_slices(int64_t nq, int64_t nc);
size_t knn_u8_workspace_bytes(int64_t nq, int slices);
hipError_t launch_knn_u8(const uint8_t* X, int64_t n, int32_t d, const int32_t* qids, int64_t nq,
                         const int32_t* cids, int64_t nc, int32_t K, int32_t* out,
                         uint64_t* workspace, int slices, hipStream_t s);
void f32_band(int d, double* c);               // c1, c2, c3 of the float32 band; chunk
// Slow-preprocessing build (k_slow_build.hip): workgroups, workspace, launch.
int slow_build_groups(int64_t n);
size_t slow_build_workspace_bytes(int64_t n, int groups);
hipError_t launch_slow_build(const void* X, int32_t dtype, int64_t n, int32_t d, uint32_t num2,
                             uint32_t den2, int32_t R, int32_t* out_nbr, int32_t* out_deg,
                             void* workspace, int groups, hipStream_t s);
bool prune_f32_shape_ok(const GraphView& g);   // shape the float32 batched kernel serves
bool prune_f32_supported(const GraphView& g);  // ... and its frame exponents are set
hipError_t launch_search(const GraphView& g, const void* Q, int64_t nq, int32_t k, int32_t L,
                         int32_t* out_ids, double* out_dist, int32_t* out_hops,
                         hipStream_t s);
hipError_t launch_search_jobs(const GraphView& g, const SearchJob* jobs, int64_t n, int32_t k,
                              int32_t L, hipStream_t s);

// FP32 direct-difference distance bound: |S~ - S| <= gamma_{d+2} S for a
// sequential fmaf accumulation of squared FP32 differences; doubled and
// widened to cover the canonical FP64 value's own error and the FP64
// arithmetic of the comparison.
inline double f32_rel_bound(int d) {
  const double u = 5.9604644775390625e-08;  // 2^-24
  const double g = (d + 2) * u / (1.0 - (d + 2) * u);
  return 2.0 * g + 4e-12;
}

// Launch tuning: vertices per workgroup (one wavefront each) of the batched
// prune kernels, per graph shape and sweep shape.  Untuned shapes use 1.
constexpr int kKernelU8 = 1;
constexpr int kKernelF32 = 2;
constexpr int kKernelU8Wide = 3;
// LDS one workgroup may take on the current device (163,840 bytes on
// gfx950; 65,536 if the runtime cannot tell), queried once per device.
int max_lds_per_group();
struct TuneKey {
  int32_t kernel, dtype, d, r_max, n_alpha, n_out;
};
int tuned_waves(const TuneKey& k);           // 0 if the shape is not tuned
void set_tuned_waves(const TuneKey& k, int waves);
int batched_kernel(const GraphView& g);      // kKernelU8, kKernelU8Wide, kKernelF32 or 0 (plain)
int batched_wave_lds(const GraphView& g);    // LDS bytes per wavefront of that kernel
// waves per workgroup to launch with: the tuned value, else 1; never more than
// the LDS per workgroup allows
inline int waves_for(const TuneKey& k, int wave_lds) {
  int w = tuned_waves(k);
  if (w < 1) w = 1;
  while (w > 1 && (size_t)w * wave_lds > (size_t)max_lds_per_group()) w >>= 1;
  return w;
}

// Error state and argument checks shared by the C-ABI entry points
// (rp_api.hip, rp_serve.hip).
rp_status fail(rp_status st, const char* fmt, ...);
rp_status ok();
const char* last_error();
bool device_range(const void* p, size_t bytes);
size_t elem_size(int32_t dt);
rp_status check_alpha(rp_alpha a);

}  // namespace rp

// A graph handle: the view the kernels read, its counters and ownership.
struct rp_graph {
  rp::GraphView view;
  rp::DevCounters* ctr;
  rp_graph* base;  // non-null for derived handles
  int device;
  int64_t nodes;   // vertex-prunes enqueued, counted on the host
  void* aux;       // per-point array owned by a base handle, shared by derived ones:
                   // |x|^2 (uint8 points) or max_k |x_k| (float32 points)
  void* frame_e;   // per-vertex frame exponents of this handle's lists (float32), or null
};
