// woi_noalloc.hip -- woi_estimate for callers that cannot allocate device memory.
//
// The per-point path's partial sums live in one file-scope device array of
// WOI_NOALLOC_SCRATCH_BYTES (each device holds its own copy until the process ends).  Its
// device address is taken once per device with hipGetSymbolAddress, with that device
// current, and only that address is handed to the kernels.  Every call on a device shares
// the array: calls that overlap on one device race.  The walk kernel writes every partial
// slot it uses before the reduction reads it, so nothing needs clearing between calls.
#include <hip/hip_runtime.h>

#include <mutex>

#include "woi.h"
#include "woi_internal.h"

namespace {

constexpr int kMaxDevices = 64;
__device__ __align__(256) double scratch[WOI_NOALLOC_SCRATCH_BYTES / sizeof(double)];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};   // device address of `scratch` per device (null: not yet taken)

}  // namespace

extern "C" woi_status woi_estimate_noalloc(const woi_problem* p, const double* points, int64_t P, const woi_query* q,
                                           double* mean, double* se, double* grad, double* grad_se,
                                           uint64_t* counters, void* stream) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return woi::set_error(WOI_E_DEVICE, "no HIP device (or device index above %d)", kMaxDevices - 1);
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_scratch[dev]) {
            void* a = nullptr;
            const hipError_t e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !a)
                return woi::set_error(WOI_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            g_scratch[dev] = a;
        }
        ptr = g_scratch[dev];
    }
    return woi::estimate_into(p, points, P, q, mean, se, grad, grad_se, static_cast<double*>(ptr),
                              WOI_NOALLOC_SCRATCH_BYTES, counters, stream);
}
