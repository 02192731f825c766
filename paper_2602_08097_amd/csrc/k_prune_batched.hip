// k_prune_batched.hip -- batched RP-Tuning (temporary: one plain pass per output).
#include "dev_common.h"

namespace rp {

hipError_t launch_prune_batched(const GraphView& g, const SweepArgs& a, DevCounters* ctr,
                                hipStream_t s) {
  for (int o = 0; o < a.n_out; ++o) {
    const SweepOut& out = a.out[o];
    hipError_t e = launch_prune_plain(g, a.num2[out.alpha_idx], a.den2[out.alpha_idx], out.R,
                                      out.nbr, out.deg, ctr, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace rp
