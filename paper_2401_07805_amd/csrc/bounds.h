// Bounds checks of the debug library (libvpp_debug.so, built with
// VPP_BOUNDS_CHECK); in the release library every macro below is the plain
// access.  An instrumented kernel first records the extent of each buffer it
// may touch (x, y, phi, the shared-node partials, the per-workgroup dot
// partials and its LDS exchange array) in a workgroup-shared table; every
// instrumented access then checks its address against the buffer it belongs
// to.  An access outside adds one to a device counter and is dropped (a load
// yields zero), so the kernel still completes normally and the host reads the
// count through vpp_debug_bounds_violations.  Instrumented: the tile kernels
// of every apply variant and the shared-node assembly.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vpp {

// Buffers of the table; BC_IN accepts x or phi (the gathers serve both), BC_OUT
// y or the partials (a write-out whose destination is chosen per node).
enum BcBuf { BC_X = 0, BC_Y, BC_PHI, BC_PART, BC_DOT, BC_SLOT, BC_NBUF, BC_IN = BC_NBUF, BC_OUT };

#ifdef VPP_BOUNDS_CHECK

struct BcTable {
    const char* lo[BC_NBUF];
    const char* hi[BC_NBUF];
};
static __shared__ BcTable bc_table;
static __device__ unsigned long long bc_violations;

__device__ __forceinline__ bool bc_in(const void* p, size_t bytes, int b)
{
    const char* c = static_cast<const char*>(p);
    return c >= bc_table.lo[b] && c + bytes <= bc_table.hi[b];
}

template <typename P>
__device__ __forceinline__ bool bc_ok(P* p, int b)
{
    const size_t nb = sizeof(*p);
    bool ok;
    if (b == BC_IN) ok = bc_in(p, nb, BC_X) || bc_in(p, nb, BC_PHI);
    else if (b == BC_OUT) ok = bc_in(p, nb, BC_Y) || bc_in(p, nb, BC_PART);
    else ok = bc_in(p, nb, b);
    if (!ok) atomicAdd(&bc_violations, 1ull);
    return ok;
}

// Every thread calls this first (before any early return): thread 0 fills the
// table (extents in elements of each buffer's type), then a barrier.
template <typename T, typename S>
__device__ __forceinline__ void bc_begin(const T* x, const T* y, const T* phi, const T* part, const double* dot,
                                         const S* slot, int64_t n, int64_t npart, int64_t ndot, int64_t nslot)
{
    if (threadIdx.x == 0) {
        auto put = [](int b, const void* p, int64_t bytes) {
            bc_table.lo[b] = static_cast<const char*>(p);
            bc_table.hi[b] = p ? static_cast<const char*>(p) + bytes : nullptr;
        };
        put(BC_X, x, n * (int64_t)sizeof(T));
        put(BC_Y, y, n * (int64_t)sizeof(T));
        put(BC_PHI, phi, n * (int64_t)sizeof(T));
        put(BC_PART, part, npart * (int64_t)sizeof(T));
        put(BC_DOT, dot, ndot * (int64_t)sizeof(double));
        put(BC_SLOT, slot, nslot * (int64_t)sizeof(S));
    }
    __syncthreads();
}

// Count of dropped accesses of this translation unit's kernels since the last
// call (the counter is reset).
static inline unsigned long long bc_take_count()
{
    unsigned long long v = 0, z = 0;
    if (hipMemcpyFromSymbol(&v, HIP_SYMBOL(bc_violations), sizeof v) != hipSuccess) return ~0ull;
    if (hipMemcpyToSymbol(HIP_SYMBOL(bc_violations), &z, sizeof z) != hipSuccess) return ~0ull;
    return v;
}

static inline unsigned long long bc_count_here() { return bc_take_count(); }

#define VPP_OK(p, b) (::vpp::bc_ok((p), (b)))
#define VPP_LD(p, b) \
    (::vpp::bc_ok((p), (b)) ? *(p) : std::remove_cv_t<std::remove_reference_t<decltype(*(p))>>{})
#define VPP_ST(p, b, v)                                   \
    do {                                                  \
        auto* vpp_bc_p_ = (p);                            \
        if (::vpp::bc_ok(vpp_bc_p_, (b))) *vpp_bc_p_ = (v); \
    } while (0)
#define VPP_BC_BEGIN(x, y, phi, part, dot, slot, n, npart, ndot, nslot) \
    ::vpp::bc_begin((x), (y), (phi), (part), (dot), (slot), (n), (npart), (ndot), (nslot))
#define VPP_BC_SYNC() __syncthreads()

#else

static inline unsigned long long bc_count_here() { return 0; }

#define VPP_OK(p, b) true
#define VPP_LD(p, b) (*(p))
#define VPP_ST(p, b, v) (*(p) = (v))
#define VPP_BC_BEGIN(x, y, phi, part, dot, slot, n, npart, ndot, nslot) ((void)0)
#define VPP_BC_SYNC() ((void)0)

#endif

}  // namespace vpp
