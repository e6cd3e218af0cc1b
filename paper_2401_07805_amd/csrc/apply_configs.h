// Instantiated apply configurations and the generic launcher.
#pragma once
#include "apply_impl.h"

namespace vpp {

// Instantiated configurations: (k, variant, tile).
#define VPP_APPLY_CONFIGS(X)  \
    X(2, 0, 8, 8, 4)          \
    X(2, 0, 16, 4, 4)         \
    X(2, 0, 8, 4, 4)          \
    X(2, 0, 4, 4, 4)          \
    X(2, 1, 4, 4, 4)          \
    X(2, 1, 8, 4, 2)          \
    X(3, 1, 4, 4, 2)          \
    X(3, 1, 4, 2, 2)          \
    X(3, 1, 8, 2, 2)          \
    X(4, 1, 4, 2, 2)          \
    X(4, 1, 2, 2, 2)          \
    X(4, 1, 4, 4, 1)

template <int K, typename T, int V, int TX, int TY, int TZ>
inline hipError_t launch_one(const ApplyArgs<T>& a, int nblocks, hipStream_t s)
{
    if constexpr (V == 0)
        hipLaunchKernelGGL((apply_cell_kernel<K, T, TX, TY, TZ>), dim3(nblocks), dim3(TX * TY * TZ), 0, s, a);
    else
        hipLaunchKernelGGL((apply_plane_kernel<K, T, TX, TY, TZ>), dim3(nblocks), dim3((K + 1) * TX * TY * TZ), 0,
                           s, a);
    return hipGetLastError();
}

template <typename T>
inline hipError_t launch_apply_t(const LaunchCfg& c, int k, const ApplyArgs<T>& a, int nblocks, hipStream_t s)
{
#define VPP_LAUNCH(K, V, TX, TY, TZ)                                                         \
    if (k == K && c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ) \
        return launch_one<K, T, V, TX, TY, TZ>(a, nblocks, s);
    VPP_APPLY_CONFIGS(VPP_LAUNCH)
#undef VPP_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace vpp
