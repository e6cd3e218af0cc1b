// CG state and vector-kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vpp {

// Device-resident scalars of one PCG (FP64 for every precision).
struct CgState {
    double rz[2];     // r.D^-1 r at the start of the iteration of parity 0 / 1
    double pAp;       // p.Ap, written by the apply of the current iteration
    double rr[2];     // accumulated r.r of the new residual (by iteration parity)
    double rznew[2];  // accumulated r.D^-1 r of the new residual (by iteration parity)
    double tol2;      // convergence threshold on r.r
    double rr_last;   // r.r after the last completed iteration (initial r.r after init)
    int done;         // converged, broke down or hit max_iter
    int breakdown;
    int iters;
    int max_iter;
};

template <typename T>
hipError_t launch_cg_init(CgState* st, const T* b, const T* q, T* r, T* p, const T* invd, int64_t n,
                          hipStream_t s);
template <typename T>
hipError_t launch_cg_update(CgState* st, int par, T* x, T* r, const T* p, const T* q, const T* invd,
                            int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_cg_pupdate(CgState* st, int par, const T* r, T* p, T* q, const T* invd, int64_t n,
                             hipStream_t s);

hipError_t launch_residual(const double* b, const double* q, double* r, int64_t n, double* rr, hipStream_t s);
hipError_t launch_demote(const double* r, double scale, float* r32, float* x32, int64_t n, hipStream_t s);
hipError_t launch_convert(const double* a, float* b, int64_t n, hipStream_t s);
hipError_t launch_promote_add(double* x, const float* d, double scale, int64_t n, hipStream_t s);

}  // namespace vpp
