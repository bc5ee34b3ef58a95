// rt_noalloc.hip -- rt_apply_op_noalloc: the FP64 operator for callers that
// cannot allocate device memory at call time.
//
// rt_apply_op's sweep writes one slot of partial quadrature sums per
// workgroup into a buffer the handle owns, and its finalize pass reads them.
// This variant keeps those partial sums in a fixed file-scope device array
// instead (one copy per GPU, held until the process ends), so the call itself
// touches no allocator.  The array's device address is looked up once per
// device with that device current; host code only ever uses that address.
// The partial sums need no clearing: every workgroup writes all of its slot
// before the finalize pass reads it.  Calls that overlap in time on one GPU
// share the array and race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>
#include <string>

#include "rt_internal.h"

namespace rt {
namespace {

constexpr long long kScratchDoubles = RT_NOALLOC_MAX_PARTIAL;
__device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device (looked up on the
// first call per device).
int scratch_ptr(int dev, double **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(RT_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(RT_EDEVICE, std::string("hipGetSymbolAddress of the scratch array: ") +
                                        hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = static_cast<double *>(p);
    }
    *out = g_scratch_ptr[dev];
    return RT_OK;
}

}  // namespace
}  // namespace rt

using namespace rt;

extern "C" int rt_apply_op_noalloc(rt_handle *h, const double *sigma_in, double *sigma_out,
                                   void *stream) {
    if (!h || !sigma_in || !sigma_out) return fail(RT_EINVAL, "NULL handle or vector");
    if (((uintptr_t)sigma_in & 15u) || ((uintptr_t)sigma_out & 15u))
        return fail(RT_EINVAL, "vectors must be 16-byte aligned");
    if (h->fs == RT_FS_DELO_PARABOLIC)
        return fail(RT_EINVAL, "rt_apply_op_noalloc supports the two-point formal solvers only");
    if (h->n_partial_main > kScratchDoubles)
        return fail(RT_EINVAL, "the handle's sweep needs " + std::to_string(h->n_partial_main) +
                                   " partial sums, more than the " +
                                   std::to_string(kScratchDoubles) +
                                   " the allocation-free operator holds (RT_NOALLOC_MAX_PARTIAL)");
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fail(RT_EDEVICE, "hipGetDevice failed");
    }
    if (dev != h->device) return fail(RT_EINVAL, "call with the handle's device current");
    double *partial = nullptr;
    const int rc = scratch_ptr(dev, &partial);
    if (rc != RT_OK) return rc;
    const hipError_t e = apply_operator_into(h, sigma_in, sigma_out, partial, (hipStream_t)stream);
    if (e != hipSuccess) return fail(RT_EDEVICE, std::string("rt_apply_op_noalloc: ") +
                                                     hipGetErrorString(e));
    return RT_OK;
}
