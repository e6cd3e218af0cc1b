// Static scratch of the allocation-free apply (implemented in noalloc.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>

namespace vpp {

// 48 MiB of FP64 partials: the shared-face partials of a 64^3 Q2, 43^3 Q3 or
// 32^3 Q4 mesh with the configurations vpp_apply_noalloc runs fit.
constexpr size_t kNoallocScratchDoubles = size_t(6) << 20;

// Device address of the static scratch on `device`, which must be the
// current device; looked up (hipGetSymbolAddress) on the first call for that
// device and kept.
hipError_t noalloc_scratch(int device, double** out);

}  // namespace vpp
