// k_prune_batched.hip -- dispatch of the batched RP-Tuning sweep.
//
// Out-lists of at most 64 ids run the int8-MFMA kernel for uint8 points
// (k_prune_u8.hip) or the FP16-MFMA kernel with FP64 recheck for float32
// points (k_prune_f32.hip); other shapes run the plain kernel once per output.
#include "dev_common.h"

namespace rp {

bool prune_u8_supported(const GraphView& g);
hipError_t launch_prune_u8(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                           hipStream_t s);
bool prune_f32_supported(const GraphView& g);
hipError_t launch_prune_f32(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                            hipStream_t s);

hipError_t launch_prune_batched(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                                hipStream_t s) {
  if (prune_u8_supported(g)) return launch_prune_u8(g, a, ctr, s);
  if (prune_f32_supported(g)) return launch_prune_f32(g, a, ctr, s);
  for (int o = 0; o < a.n_out; ++o) {
    const SweepOut& out = a.out[o];
    hipError_t e = launch_prune_plain(g, a.num2[out.alpha_idx], a.den2[out.alpha_idx], out.R,
                                      out.nbr, out.deg, ctr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rp
