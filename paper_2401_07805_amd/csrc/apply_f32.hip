// FP32 apply kernels (all instantiated configurations).
#include "apply_configs.h"

namespace vpp {

hipError_t launch_apply_f32(const LaunchCfg& c, int k, const ApplyArgs<float>& a, hipStream_t s)
{
    return launch_apply_t<float>(c, k, a, s);
}

}  // namespace vpp
