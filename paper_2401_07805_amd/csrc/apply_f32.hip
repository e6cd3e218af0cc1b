// FP32 apply: dispatch by degree to the per-degree units (apply_f32_k*.hip).
#include "apply_configs.h"

namespace vpp {

hipError_t launch_apply_f32(const LaunchCfg& c, int k, const ApplyArgs<float>& a, hipStream_t s)
{
    switch (k) {
    case 2: return launch_apply_f32_k2(c, a, s);
    case 3: return launch_apply_f32_k3(c, a, s);
    case 4: return launch_apply_f32_k4(c, a, s);
    default: return hipErrorInvalidValue;
    }
}


}  // namespace vpp
