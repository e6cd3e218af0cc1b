// F64 apply kernels of degree 4 (one translation unit per precision and
// degree, so that the template-heavy units compile in parallel).
#include "apply_configs.h"

namespace vpp {

hipError_t launch_apply_f64_k4(const LaunchCfg& c, const ApplyArgs<double>& a, hipStream_t s)
{
    return launch_apply_t<double, 4>(c, a, s);
}

unsigned long long bounds_count_apply_f64_k4() { return bc_count_here(); }

}  // namespace vpp
