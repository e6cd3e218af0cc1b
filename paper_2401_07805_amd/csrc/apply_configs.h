// Instantiated apply configurations and the generic launcher.
#pragma once
#include "apply_impl.h"

namespace vpp {

// Instantiated configurations: (k, variant, tile).
#define VPP_APPLY_CONFIGS(X)  \
    X(2, 4, 8, 8, 8)          \
    X(2, 4, 32, 4, 4)         \
    X(2, 4, 16, 8, 4)         \
    X(2, 4, 16, 4, 4)         \
    X(2, 4, 8, 8, 4)          \
    X(2, 4, 8, 4, 4)          \
    X(2, 0, 16, 4, 4)         \
    X(2, 0, 8, 4, 4)          \
    X(2, 1, 8, 4, 2)          \
    X(3, 2, 8, 8, 4)          \
    X(3, 2, 8, 4, 4)          \
    X(3, 2, 4, 4, 4)          \
    X(3, 2, 8, 4, 2)          \
    X(3, 4, 8, 4, 4)          \
    X(3, 4, 4, 4, 4)          \
    X(3, 1, 4, 4, 2)          \
    X(3, 1, 4, 2, 2)          \
    X(3, 1, 8, 2, 2)          \
    X(4, 1, 4, 2, 2)          \
    X(4, 1, 2, 2, 2)          \
    X(4, 1, 4, 4, 1)

// Configurations also instantiated with the mass shift mu M of the level-set
// filter operators (variant 4: the mass term sits in cell_operator; variant 1:
// in the plane kernel's Gauss-point step).
#define VPP_MASS_CONFIGS(X) \
    X(2, 4, 16, 8, 4)       \
    X(2, 4, 32, 4, 4)       \
    X(2, 4, 8, 4, 4)        \
    X(3, 4, 8, 4, 4)        \
    X(4, 1, 4, 2, 2)        \
    X(4, 1, 2, 2, 2)

// Configurations also instantiated with the arithmetic density mean (laws 2
// and 3 of coef_scaled; the contrast of App. D): one per degree, the default
// configuration of a new problem.
#define VPP_ARITH_CONFIGS(X) \
    X(2, 4, 8, 8, 4)         \
    X(3, 1, 4, 4, 2)         \
    X(4, 1, 4, 2, 2)

template <int K, typename T, int V, int TX, int TY, int TZ, int HV, bool DOT, bool MASS>
inline auto kernel_ptr()
{
    static_assert(!MASS || V == 4 || V == 1, "the mass shift is instantiated for variants 1 and 4");
    if constexpr (V == 0) return &apply_cell_kernel<K, T, TX, TY, TZ, HV, DOT>;
    else if constexpr (V == 1) return &apply_plane_kernel<K, T, TX, TY, TZ, HV, DOT, MASS>;
    else if constexpr (V == 2) return &apply_half_kernel<K, T, TX, TY, TZ, HV, DOT>;
    else return &apply_slot_kernel<K, T, TX, TY, TZ, HV, DOT, MASS>;
}

template <int K, typename T, int V, int TX, int TY, int TZ, int HV, bool DOT, bool MASS>
inline hipError_t launch_hv(const ApplyArgs<T>& a, hipStream_t s)
{
    const int nblocks = a.m.ntile[0] * a.m.ntile[1] * a.m.ntile[2];
    constexpr int threads = V == 1 ? (K + 1) * TX * TY * TZ : (V == 2 ? 2 : 1) * TX * TY * TZ;
    hipLaunchKernelGGL((kernel_ptr<K, T, V, TX, TY, TZ, HV, DOT, MASS>()), dim3(nblocks), dim3(threads), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || a.tiles_only) return e;
    const int tile[3] = {TX, TY, TZ};
    AssembleArgs<T> b{a.m, shared_enum(a.m, K, tile), a.part, a.nshared, a.y, a.dot_part, nblocks, a.dot, a.done};
    return launch_assemble<T>(b, s);
}

template <int K, typename T, int V, int TX, int TY, int TZ, bool MASS = false>
inline hipError_t launch_one(const ApplyArgs<T>& a, hipStream_t s)
{
    // the x . (A x) partials are a separate instantiation, used inside CG only
    if (a.dot_part) {
        if (a.m.heaviside == 0) return launch_hv<K, T, V, TX, TY, TZ, 0, true, MASS>(a, s);
        return launch_hv<K, T, V, TX, TY, TZ, 1, true, MASS>(a, s);
    }
    if (a.m.heaviside == 0) return launch_hv<K, T, V, TX, TY, TZ, 0, false, MASS>(a, s);
    return launch_hv<K, T, V, TX, TY, TZ, 1, false, MASS>(a, s);
}

template <int K, typename T, int V, int TX, int TY, int TZ>
inline hipError_t launch_one_arith(const ApplyArgs<T>& a, hipStream_t s)
{
    if (a.dot_part) {
        if (a.m.heaviside == 2) return launch_hv<K, T, V, TX, TY, TZ, 2, true, false>(a, s);
        return launch_hv<K, T, V, TX, TY, TZ, 3, true, false>(a, s);
    }
    if (a.m.heaviside == 2) return launch_hv<K, T, V, TX, TY, TZ, 2, false, false>(a, s);
    return launch_hv<K, T, V, TX, TY, TZ, 3, false, false>(a, s);
}

// Launch of configuration c for the degree KS of the calling translation unit:
// only that degree's configurations are instantiated there, so the units of
// the three degrees compile in parallel.
template <typename T, int KS>
inline hipError_t launch_apply_t(const LaunchCfg& c, const ApplyArgs<T>& a, hipStream_t s)
{
    if (a.m.heaviside >= 2) {
        if (a.m.mass != 0.0) return hipErrorInvalidValue;
#define VPP_LAUNCH_ARITH(K, V, TX, TY, TZ)                                              \
    if constexpr (K == KS)                                                              \
        if (c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ)    \
            return launch_one_arith<K, T, V, TX, TY, TZ>(a, s);
        VPP_ARITH_CONFIGS(VPP_LAUNCH_ARITH)
#undef VPP_LAUNCH_ARITH
        return hipErrorInvalidValue;
    }
    if (a.m.mass != 0.0) {
#define VPP_LAUNCH_MASS(K, V, TX, TY, TZ)                                               \
    if constexpr (K == KS)                                                              \
        if (c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ)    \
            return launch_one<K, T, V, TX, TY, TZ, true>(a, s);
        VPP_MASS_CONFIGS(VPP_LAUNCH_MASS)
#undef VPP_LAUNCH_MASS
        return hipErrorInvalidValue;
    }
#define VPP_LAUNCH(K, V, TX, TY, TZ)                                                    \
    if constexpr (K == KS)                                                              \
        if (c.variant == V && c.tile[0] == TX && c.tile[1] == TY && c.tile[2] == TZ)    \
            return launch_one<K, T, V, TX, TY, TZ>(a, s);
    VPP_APPLY_CONFIGS(VPP_LAUNCH)
#undef VPP_LAUNCH
    return hipErrorInvalidValue;
}

}  // namespace vpp
