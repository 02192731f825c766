// k_prune_batched.hip -- dispatch of the batched RP-Tuning sweep.
//
// uint8 points with out-lists of at most 64 ids run the int8-MFMA kernel
// (k_prune_u8.hip), of 65..128 ids at d <= 128 its four-block form
// (k_prune_u8_wide.hip); float32 points with out-lists of at most 128 ids run
// the FP16-MFMA kernel with FP64 recheck (k_prune_f32.hip); other shapes run
// the plain kernel once per output.
#include <map>
#include <mutex>
#include <tuple>

#include "dev_common.h"

namespace rp {

namespace {
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int, int, int, int>, int> g_tune;

std::tuple<int, int, int, int, int, int> key_of(const TuneKey& k) {
  return std::make_tuple(k.kernel, k.dtype, k.d, k.r_max, k.n_alpha, k.n_out);
}
}  // namespace

int tuned_waves(const TuneKey& k) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(key_of(k));
  return it == g_tune.end() ? 0 : it->second;
}

void set_tuned_waves(const TuneKey& k, int waves) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  if (waves < 1) g_tune.erase(key_of(k));
  else g_tune[key_of(k)] = waves;
}

namespace {
constexpr int kLdsDevices = 64;
std::mutex g_lds_mu;
int g_lds[kLdsDevices];  // 0 = not queried yet
}  // namespace

int max_lds_per_group() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kLdsDevices) {
    (void)hipGetLastError();
    return 65536;
  }
  std::lock_guard<std::mutex> lk(g_lds_mu);
  if (g_lds[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess ||
        v < 65536) {
      (void)hipGetLastError();
      v = 65536;
    }
    g_lds[dev] = v;
  }
  return g_lds[dev];
}

bool prune_u8_supported(const GraphView& g);
hipError_t launch_prune_u8(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                           hipStream_t s);
bool prune_u8_wide_supported(const GraphView& g);
hipError_t launch_prune_u8_wide(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                                hipStream_t s);
int prune_u8_wide_wave_lds(const GraphView& g);
bool prune_f32_supported(const GraphView& g);
int prune_u8_wave_lds(const GraphView& g);
int prune_f32_wave_lds(const GraphView& g);
hipError_t launch_prune_f32(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                            hipStream_t s);

int batched_kernel(const GraphView& g) {
  if (prune_u8_supported(g)) return kKernelU8;
  if (prune_u8_wide_supported(g)) return kKernelU8Wide;
  if (prune_f32_supported(g)) return kKernelF32;
  return 0;
}

int batched_wave_lds(const GraphView& g) {
  if (prune_u8_supported(g)) return prune_u8_wave_lds(g);
  if (prune_u8_wide_supported(g)) return prune_u8_wide_wave_lds(g);
  if (prune_f32_supported(g)) return prune_f32_wave_lds(g);
  return 0;
}

hipError_t launch_prune_batched(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                                hipStream_t s) {
  if (prune_u8_supported(g)) return launch_prune_u8(g, a, ctr, s);
  if (prune_u8_wide_supported(g)) return launch_prune_u8_wide(g, a, ctr, s);
  if (prune_f32_supported(g)) return launch_prune_f32(g, a, ctr, s);
  for (int o = 0; o < a.n_out; ++o) {
    const SweepOut& out = a.out[o];
    hipError_t e = launch_prune_plain(g, a.num2[out.alpha_idx], a.den2[out.alpha_idx], out.R,
                                      out.nbr, out.deg, ctr, s, a.unsorted != 0);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rp
