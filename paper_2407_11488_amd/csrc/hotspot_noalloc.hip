// hotspot_run_noalloc: hotspot_run for callers that cannot allocate device
// memory. A run of more than one launch alternates between the output and a
// work grid; here that grid is a fixed array of the library's own device
// code, present on every GPU the library runs on until the process ends, so
// the call allocates nothing.
#include <hip/hip_runtime.h>

#include <mutex>

#include "hotspot.h"
#include "internal.h"

namespace conv2d {
namespace {

// The fixed work grid (HOTSPOT_NOALLOC_CELLS floats, 64 MiB): a 4096 x 4096
// grid, or any grid of at most that many cells. Host code never passes this
// name to a kernel (it is a host-side stand-in for the device symbol); it
// uses the device address that hipGetSymbolAddress returns for the current
// device.
__device__ __align__(256) float scratch[HOTSPOT_NOALLOC_CELLS];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
float* g_ptr[kMaxDevices] = {};

// The current device's address of `scratch`, looked up once per device.
int scratch_ptr(float** out)
{
    int dev = -1;
    CONV2D_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(CONV2D_EINVAL, "device index out of range");
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(CONV2D_EHIP, "hipGetSymbolAddress(scratch) returned NULL");
        g_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_ptr[dev];
    return CONV2D_OK;
}

}  // namespace
}  // namespace conv2d

using namespace conv2d;

extern "C" int hotspot_run_noalloc(hotspot_plan_t plan, const float* d_temp, const float* d_power, float* d_out,
                                   int steps, hotspot_coeffs k, void* stream)
{
    clear_error();
    if (!plan) return fail(CONV2D_EINVAL, "plan is NULL");
    float* work = nullptr;
    int rc = scratch_ptr(&work);
    if (rc) return rc;
    return hotspot_run_fixed_work(plan, d_temp, d_power, d_out, work, (size_t)HOTSPOT_NOALLOC_CELLS, steps, k,
                                  stream);
}
