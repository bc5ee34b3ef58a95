// rt_sweep_f32_w.hip -- the fused sweep instantiated for float arithmetic,
// w streamed and E derived.
#include "rt_sweep_kernel.h"

namespace rt {

hipError_t launch_sweep_f32_w(int L, int W, bool pf, const SweepArgs &a, int nblocks, int ns_max,
                              hipStream_t s) {
    return sweep::launch_any<float, kCoefW>(L, W, pf, a, nblocks, ns_max, s);
}

}  // namespace rt
