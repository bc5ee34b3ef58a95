// rt_sweep_f64.hip -- the fused sweep instantiated for double arithmetic,
// step coefficients streamed as (E, w) pairs.
#include "rt_sweep_kernel.h"

namespace rt {

hipError_t launch_sweep_f64(int L, int W, bool pf, const SweepArgs &a, int nblocks, int ns_max,
                            hipStream_t s) {
    return sweep::launch_any<double, kCoefPairs>(L, W, pf, a, nblocks, ns_max, s);
}

}  // namespace rt
