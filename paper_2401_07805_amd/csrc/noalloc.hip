// Static scratch of the allocation-free apply (vpp_apply_noalloc): the
// shared-face partials of the tile kernel live in one file-scope device array
// instead of a problem's workspace, so the entry point never allocates.  The
// array exists once per device the library is loaded on, for the lifetime of
// the process; its device address is looked up once per device, with that
// device current, and only that address is handed to kernels.
#include <hip/hip_runtime.h>

#include <mutex>

#include "noalloc.h"

namespace vpp {

static __device__ __align__(256) double scratch[kNoallocScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
double* g_ptr[kMaxDevices] = {};
}  // namespace

hipError_t noalloc_scratch(int device, double** out)
{
    *out = nullptr;
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;   // the caller makes `device` current
        void* ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        if (!ptr) return hipErrorInvalidSymbol;
        g_ptr[device] = static_cast<double*>(ptr);
    }
    *out = g_ptr[device];
    return hipSuccess;
}

}  // namespace vpp
