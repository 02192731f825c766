// rp_noalloc.hip -- rp_knn_u8_noalloc: the exact K-NN entry point for callers
// that cannot allocate (code under HIP graph capture, serving loops, hosts
// that forbid device allocation).  Its workspace is the file-scope device
// array below, one copy per GPU, held until the process ends.
#include <mutex>

#include "rp_internal.h"

namespace rp {

namespace {

// The partial lists of the candidate slices: slices x nq x 1 KiB.
constexpr size_t kNoallocBytes = (size_t)64 << 20;
static __device__ __align__(256) uint64_t scratch[kNoallocBytes / 8];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_ptr[kMaxDevices];  // the device address of `scratch` on each GPU

// The device address of this GPU's copy of the array (looked up once per
// device, with that device current).  The array's name is a host-side
// stand-in, never passed to a kernel.
rp_status scratch_of_current_device(uint64_t** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(RP_EDEVICE, "hipGetDevice failed");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(RP_EDEVICE, "hipGetSymbolAddress of the workspace failed: %s",
                  hipGetErrorString(e));
    }
    g_ptr[dev] = p;
  }
  *out = (uint64_t*)g_ptr[dev];
  return RP_OK;
}

}  // namespace

}  // namespace rp

extern "C" rp_status rp_knn_u8_noalloc(const uint8_t* points, int64_t n, int32_t d,
                                       const int32_t* query_ids, int64_t nq,
                                       const int32_t* cand_ids, int64_t nc, int32_t K,
                                       int32_t slices, int32_t* out_ids, void* stream) {
  rp_status st = rp::knn_args(points, n, d, query_ids, nq, cand_ids, nc, K, out_ids);
  if (st != RP_OK) return st;
  if (slices < 0 || slices > 64) return rp::fail(RP_EINVAL, "slices must be in [0, 64]");
  if (nq == 0) return rp::ok();
  const size_t per_slice = (size_t)nq * 1024;  // one 128-key partial list per query
  if (slices == 0) {
    // the library's choice for this shape, reduced until it fits
    slices = rp::knn_u8_slices(nq, nc);
    while (slices > 1 && (size_t)slices * per_slice > rp::kNoallocBytes) --slices;
  }
  const size_t need = rp::knn_u8_workspace_bytes(nq, slices);
  if (need > rp::kNoallocBytes)
    return rp::fail(RP_EINVAL,
                    "%d slices of %lld queries need %zu bytes of workspace; the fixed "
                    "workspace holds %zu",
                    slices, (long long)nq, need, rp::kNoallocBytes);
  uint64_t* ws = nullptr;
  if (need) {
    st = rp::scratch_of_current_device(&ws);
    if (st != RP_OK) return st;
  }
  const hipError_t e = rp::launch_knn_u8(points, n, d, query_ids, nq, cand_ids, nc, K, out_ids,
                                         ws, slices, (hipStream_t)stream);
  if (e != hipSuccess) return rp::fail(RP_EDEVICE, "knn_u8: %s", hipGetErrorString(e));
  return rp::ok();
}
