// rt_sweep_f32.hip -- the fused sweep instantiated for float arithmetic.
#include "rt_sweep_kernel.h"

namespace rt {

hipError_t launch_sweep_f32(int L, int W, bool pf, const SweepArgs &a, int nblocks, int ns_max,
                            hipStream_t s) {
    switch (L) {
        case 4: return sweep::launch<float, 4>(a, W, pf, nblocks, ns_max, s);
        case 8: return sweep::launch<float, 8>(a, W, pf, nblocks, ns_max, s);
        case 16: return sweep::launch<float, 16>(a, W, pf, nblocks, ns_max, s);
        case 32: return sweep::launch<float, 32>(a, W, pf, nblocks, ns_max, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace rt
