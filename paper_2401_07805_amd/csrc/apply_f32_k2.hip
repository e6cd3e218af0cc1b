// F32 apply kernels of degree 2 (one translation unit per precision and
// degree, so that the template-heavy units compile in parallel).
#include "apply_configs.h"

namespace vpp {

hipError_t launch_apply_f32_k2(const LaunchCfg& c, const ApplyArgs<float>& a, hipStream_t s)
{
    return launch_apply_t<float, 2>(c, a, s);
}

unsigned long long bounds_count_apply_f32_k2() { return bc_count_here(); }

}  // namespace vpp
