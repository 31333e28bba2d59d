// awe_misfit_noalloc: the misfit of Eq. (2) for callers that cannot allocate
// device memory (code under HIP graph capture, tight serving loops).  The
// per-block partial sums that awe_misfit allocates on every call live here in
// a file-scope device array instead; the result goes to device memory and
// nothing is synchronised, so the call is a pure enqueue.
#include <hip/hip_runtime.h>

#include <mutex>

#include "awe.h"
#include "awe_internal.hpp"
#include "engine.hpp"

using awe::fail;

namespace {

// One FP64 partial per reduction block: every call's first kernel writes all
// kReduceBlocks of them before the second reads them, so nothing needs
// clearing.  Each device holds its own copy (8 KiB) until the process ends.
constexpr int kScratchDoubles = awe::kReduceBlocks;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch` per device (set once)

// The device address of this device's `scratch`, looked up once per device
// with that device current.  The array's name is a host-side stand-in and is
// never passed to a kernel.
awe_status scratch_for(int dev, double** out) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(AWE_EHIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = static_cast<double*>(g_scratch_ptr[dev]);
    return AWE_OK;
}

}  // namespace

extern "C" awe_status awe_misfit_noalloc(const float* traces, const float* d_obs, int64_t n, float* resid,
                                         double* phi_dev, awe_stream s) {
    if (!phi_dev) return fail(AWE_EINVAL, "phi_dev pointer is NULL");
    if (n < 0) return fail(AWE_EINVAL, "n must be >= 0");
    if (n > 0 && (!traces || !d_obs)) return fail(AWE_EINVAL, "NULL trace pointer");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(AWE_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(AWE_EINVAL, "device %d beyond the %d supported", dev, kMaxDevices);
    double* part = nullptr;
    awe_status st = scratch_for(dev, &part);
    if (st) return st;
    // The partials need kReduceBlocks doubles whatever n is (the blocks
    // stride over the data): the scratch array always suffices.
    static_assert(kScratchDoubles >= awe::kReduceBlocks, "scratch smaller than the reduction's partials");
    e = awe::launch_misfit(traces, d_obs, n, resid, part, awe::kReduceBlocks, phi_dev, reinterpret_cast<hipStream_t>(s));
    if (e != hipSuccess) return fail(AWE_EHIP, "misfit: %s", hipGetErrorString(e));
    return AWE_OK;
}
