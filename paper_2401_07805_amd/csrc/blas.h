// CG state and vector-kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shared_nodes.h"

namespace vpp {

// Device-resident scalars of one PCG (FP64 for every precision).
struct CgState {
    double rz[2];     // r.D^-1 r at the start of the iteration of parity 0 / 1
    double pAp;       // p.Ap, written by the apply of the current iteration
    double rr[2];     // r.r of the new residual (by iteration parity)
    double rznew[2];  // r.D^-1 r of the new residual (by iteration parity)
    double tol2;      // convergence threshold on r.r
    double rr_last;   // r.r after the last completed iteration (initial r.r after init)
    int halt[2];      // stop flag read by the kernels of the iteration of parity 0 / 1
    int breakdown;    // p.Ap <= 0 or a non-finite scalar
    int iters;
    int max_iter;
};

// Reduction workspace: per-workgroup partial sums of two quantities, summed in
// a fixed order by the consumer (no atomics, bit-reproducible results).
constexpr int kMaxRedBlocks = 1024;
constexpr int kRedDoubles = 2 * kMaxRedBlocks;

template <typename T>
hipError_t launch_cg_init(CgState* st, double* red, const T* b, const T* q, T* r, T* p, const T* invd, int64_t n,
                          hipStream_t s);
// CG update after a tiles-only apply q = A p: p.Ap from the ndot per-workgroup
// partials dot_part; the values of q on shared nodes assembled from the partial
// array part (stride `stride`, enumeration e); alpha = rz / pAp, x += alpha p,
// r -= alpha q, and per-workgroup partials of r.r and r.(D^-1 r).
template <typename T>
hipError_t launch_cg_assemble_update(CgState* st, int par, double* red, const double* dot_part, int ndot,
                                     const MeshArgs& m, const SharedEnum& e, const T* part, int64_t stride, T* x,
                                     T* r, const T* p, const T* q, const T* invd, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_cg_pupdate(CgState* st, int par, const double* red, const T* r, T* p, const T* invd, int64_t n,
                             hipStream_t s);

// r = b - q in FP64 (r may be null) and *rr = r.r.
hipError_t launch_residual(const double* b, const double* q, double* r, int64_t n, double* red, double* rr,
                           hipStream_t s);
// Residual replacement of the FP32 inner PCG: r32 = (float)(scale r64),
// x32 = 0, and p32 = D^-1 r32 (pscale == 0: fresh start) or p32 *= pscale
// (search direction kept across the replacement); then the state restarts at
// parity 0 with rz[0] = r32.D^-1 r32, rr_last = r32.r32 and done = 0.
hipError_t launch_cg_replace32(CgState* st, double* red, const double* r64, double scale, double pscale,
                               float* r32, float* p32, float* x32, const float* invd, int64_t n, hipStream_t s);
hipError_t launch_convert(const double* a, float* b, int64_t n, hipStream_t s);
hipError_t launch_promote_add(double* x, const float* d, double scale, int64_t n, hipStream_t s);

}  // namespace vpp
