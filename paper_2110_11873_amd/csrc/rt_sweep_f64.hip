// rt_sweep_f64.hip -- the fused sweep instantiated for double arithmetic.
#include "rt_sweep_kernel.h"

namespace rt {

hipError_t launch_sweep_f64(int L, int W, bool pf, const SweepArgs &a, int nblocks, int ns_max,
                            hipStream_t s) {
    switch (L) {
        case 4: return sweep::launch<double, 4>(a, W, pf, nblocks, ns_max, s);
        case 8: return sweep::launch<double, 8>(a, W, pf, nblocks, ns_max, s);
        case 16: return sweep::launch<double, 16>(a, W, pf, nblocks, ns_max, s);
        case 32: return sweep::launch<double, 32>(a, W, pf, nblocks, ns_max, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rt
