// F32 apply kernels of degree 3 (one translation unit per precision and
// degree, so that the template-heavy units compile in parallel).
#include "apply_configs.h"

namespace vpp {

hipError_t launch_apply_f32_k3(const LaunchCfg& c, const ApplyArgs<float>& a, hipStream_t s)
{
    return launch_apply_t<float, 3>(c, a, s);
}

unsigned long long bounds_count_apply_f32_k3() { return bc_count_here(); }

}  // namespace vpp
