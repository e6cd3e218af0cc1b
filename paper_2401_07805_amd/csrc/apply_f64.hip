// FP64 apply: dispatch by degree to the per-degree units (apply_f64_k*.hip), and
// the configuration lists.
#include "apply_configs.h"

namespace vpp {

hipError_t launch_apply_f64(const LaunchCfg& c, int k, const ApplyArgs<double>& a, hipStream_t s)
{
    switch (k) {
    case 2: return launch_apply_f64_k2(c, a, s);
    case 3: return launch_apply_f64_k3(c, a, s);
    case 4: return launch_apply_f64_k4(c, a, s);
    default: return hipErrorInvalidValue;
    }
}

bool apply_config_supported(const LaunchCfg& c, int k)
{
#define VPP_SUP(K, V, TX, TY, TZ) \
    if (k == K && c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ) return true;
    VPP_APPLY_CONFIGS(VPP_SUP)
#undef VPP_SUP
    return false;
}

int list_apply_configs(int k, LaunchCfg* out, int cap)
{
    int n = 0;
#define VPP_LIST(K, V, TX, TY, TZ)                          \
    if (k == K) {                                           \
        if (n < cap && out) out[n] = LaunchCfg{V, {TX, TY, TZ}}; \
        ++n;                                                \
    }
    VPP_APPLY_CONFIGS(VPP_LIST)
#undef VPP_LIST
    return n;
}

bool arith_config_supported(const LaunchCfg& c, int k)
{
#define VPP_ASUP(K, V, TX, TY, TZ) \
    if (k == K && c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ) return true;
    VPP_ARITH_CONFIGS(VPP_ASUP)
#undef VPP_ASUP
    return false;
}

int list_arith_configs(int k, LaunchCfg* out, int cap)
{
    int n = 0;
#define VPP_ALIST(K, V, TX, TY, TZ)                              \
    if (k == K) {                                                \
        if (n < cap && out) out[n] = LaunchCfg{V, {TX, TY, TZ}}; \
        ++n;                                                     \
    }
    VPP_ARITH_CONFIGS(VPP_ALIST)
#undef VPP_ALIST
    return n;
}

bool mass_config_supported(const LaunchCfg& c, int k)
{
#define VPP_MSUP(K, V, TX, TY, TZ) \
    if (k == K && c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ) return true;
    VPP_MASS_CONFIGS(VPP_MSUP)
#undef VPP_MSUP
    return false;
}

int list_mass_configs(int k, LaunchCfg* out, int cap)
{
    int n = 0;
#define VPP_MLIST(K, V, TX, TY, TZ)                              \
    if (k == K) {                                                \
        if (n < cap && out) out[n] = LaunchCfg{V, {TX, TY, TZ}}; \
        ++n;                                                     \
    }
    VPP_MASS_CONFIGS(VPP_MLIST)
#undef VPP_MLIST
    return n;
}


}  // namespace vpp
