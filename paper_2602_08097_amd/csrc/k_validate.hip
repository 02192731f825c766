// k_validate.hip -- adjacency validation at load time: every degree must lie in
// [0, r_max] and every listed id in [0, n).  One lane per vertex; failures are
// counted into DevCounters::errors.
#include "dev_common.h"

namespace rp {

__global__ void validate_kernel(GraphView g, DevCounters* ctr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (p < g.n) {
    const int m = g.deg[p];
    if (m < 0 || m > g.r_max) {
      bad = true;
    } else {
      const int32_t* row = g.nbr + p * g.r_max;
      for (int t = 0; t < m; ++t) {
        int id = row[t];
        if (id < 0 || (int64_t)id >= g.n) bad = true;
      }
    }
  }
  unsigned long long cnt = __popcll(__ballot(bad));
  if ((threadIdx.x & (kWave - 1)) == 0 && cnt) atomicAdd(&ctr->errors, cnt);
}

// |x_p|^2 of every uint8 point (exact), for the search distances.
__global__ void norms_u8_kernel(const uint8_t* __restrict__ X, int64_t n, int d,
                                uint32_t* __restrict__ norms) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint8_t* x = X + p * d;
  uint32_t acc = 0;
  for (int k = 0; k < d; ++k) acc += (uint32_t)x[k] * x[k];
  norms[p] = acc;
}

hipError_t launch_norms_u8(const GraphView& g, uint32_t* norms, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (g.n + block - 1) / block;
  hipLaunchKernelGGL(norms_u8_kernel, dim3((unsigned)grid), dim3(block), 0, s,
                     (const uint8_t*)g.X, g.n, g.d, norms);
  return hipGetLastError();
}

// max_k |x_k| of every float32 point, for the MFMA scale of a vertex's frame;
// points with a NaN or infinite coordinate are counted into ctr->errors (the
// distances of Section 4 are defined on finite coordinates only).
__global__ void maxabs_f32_kernel(const float* __restrict__ X, int64_t n, int d,
                                  float* __restrict__ maxabs, DevCounters* ctr) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  bool bad = false;
  if (p < n) {
    const float* x = X + p * d;
    float acc = 0.f;
    for (int k = 0; k < d; ++k) {
      const float a = fabsf(x[k]);
      bad = bad || !(a <= 3.40282347e38f);  // NaN or infinity
      acc = fmaxf(acc, a);
    }
    maxabs[p] = acc;
  }
  unsigned long long cnt = __popcll(__ballot(bad));
  if ((threadIdx.x & (kWave - 1)) == 0 && cnt) atomicAdd(&ctr->errors, cnt);
}

hipError_t launch_maxabs_f32(const GraphView& g, float* maxabs, DevCounters* ctr, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (g.n + block - 1) / block;
  hipLaunchKernelGGL(maxabs_f32_kernel, dim3((unsigned)grid), dim3(block), 0, s,
                     (const float*)g.X, g.n, g.d, maxabs, ctr);
  return hipGetLastError();
}

// Frame exponent of every vertex: from the max |x_k| of its listed ids (p
// itself and -1 excluded) plus its own, one wavefront per vertex.
__global__ void frame_exponents_f32_kernel(GraphView g, int8_t* __restrict__ e) {
  const int lane = threadIdx.x & 63;
  const int64_t p = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (p >= g.n) return;
  const int m = g.deg[p];
  float mj = 0.f;
  for (int s = lane; s < m; s += 64) {
    const int id = g.nbr[p * g.r_max + s];
    if (id >= 0 && id != (int)p) mj = fmaxf(mj, g.maxabs[id]);
  }
  for (int off = 32; off > 0; off >>= 1) mj = fmaxf(mj, __shfl_xor(mj, off, 64));
  // the bound in FP64: the sum of two finite floats stays finite
  if (lane == 0) e[p] = (int8_t)frame_exponent((double)mj + (double)g.maxabs[p]);
}

hipError_t launch_frame_exponents_f32(const GraphView& g, int8_t* e, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (g.n + 3) / 4;
  hipLaunchKernelGGL(frame_exponents_f32_kernel, dim3((unsigned)grid), dim3(block), 0, s, g, e);
  return hipGetLastError();
}

hipError_t launch_validate(const GraphView& g, DevCounters* ctr, hipStream_t s) {
  const int block = 256;
  const int64_t grid = (g.n + block - 1) / block;
  hipLaunchKernelGGL(validate_kernel, dim3((unsigned)grid), dim3(block), 0, s, g, ctr);
  return hipGetLastError();
}

}  // namespace rp
