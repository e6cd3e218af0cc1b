// CG state and vector-kernel launchers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "shared_nodes.h"

namespace vpp {

// Device-resident scalars of one PCG (FP64 for every precision).
struct CgState {
    double rz[2];     // r.D^-1 r at the start of the iteration of parity 0 / 1
    double pAp;       // p.Ap of the current iteration, written by the update
    double rr[2];     // r.r of the new residual (by iteration parity)
    double rznew[2];  // r.D^-1 r of the new residual (by iteration parity)
    double tol2;      // convergence threshold on r.r
    double rr_last;   // r.r after the last completed iteration (initial r.r after init)
    int halt[2];      // stop flag read by the kernels of the iteration of parity 0 / 1
    int breakdown;    // p.Ap <= 0 or a non-finite scalar
    int iters;
    int max_iter;
    // Record of an FP32 phase (mixed-precision deflation; all zero = off): the
    // update of iteration it stores its residual r_it at hist + it * hist_stride
    // and the direction update stores alpha_{it-1}, beta_{it-1}, r_it.z_it at
    // coef[3 it .. 3 it + 2], for every it < hist_cap.
    float* hist;
    double* coef;
    int64_t hist_stride;
    int hist_cap;
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
// array part (stride `stride`, enumeration e); alpha = rz / pAp,
// r -= alpha q, and per-workgroup partials of r.r and r.(D^-1 r).
template <typename T>
hipError_t launch_cg_assemble_update(CgState* st, int par, double* red, const double* dot_part, int ndot,
                                     const MeshArgs& m, const SharedEnum& e, const T* part, int64_t stride, T* r,
                                     const T* q, const T* invd, int64_t n, hipStream_t s);
// Stop decision, x += alpha p (alpha as in the update) and p = D^-1 r + beta p.
template <typename T>
hipError_t launch_cg_pupdate(CgState* st, int par, const double* red, T* x, const T* r, T* p, const T* invd,
                             int64_t n, hipStream_t s);

// One system of a batched PCG (entry of a device table; one per (mesh, rhs)).
template <typename T>
struct CgSystem {
    CgState* st;
    double* red;              // kRedDoubles partials of this system's reductions
    SharedEnum e;             // shared-node enumeration of the batched apply's tiles
    int bcmask;
    const T* part;            // the batched apply's shared-node partials of this system
    int64_t stride;
    const double* dot_part;   // the batched apply's per-tile partials of p.Ap (ndot)
    int ndot;
    T* x;
    T* r;
    T* p;
    const T* q;
    const T* invd;
    int64_t n;
    int blk_begin;            // first workgroup of this system in the batched launches
    int nblk;                 // its workgroup count, cg_update_blocks(n)
};

// Workgroups of the single-system update and search-direction update.
int cg_update_blocks(int64_t n);
// The update and the search-direction update of every system of sys[0..nsys)
// (device table) as two launches of total_blocks workgroups; the first also
// resets the batched apply's work counter *queue (if not null).
hipError_t launch_cg_batch_step(const CgSystem<double>* sys, int nsys, int total_blocks, int par, int* queue,
                                hipStream_t s);

// r = b - q in FP64 (r may be null) and *rr = r.r.
// Deflation space of the mixed-precision solver: W[t] = D^-1 sum_j C[j k + t]
// hist[j] for t < k (k <= kMaxDefl), FP64 vectors of length n, W[t] at W + t n.
constexpr int kMaxDefl = 8;
hipError_t launch_ritz(const float* hist, int64_t stride, int m, const double* C, int k, const double* invd,
                       double* W, int64_t n, hipStream_t s);
// out[t] = V[t] . y for t < k (V[t] at V + t n), summed in a fixed order; red
// holds k * kMaxRedBlocks partials.
hipError_t launch_multi_dot(const double* V, int k, const double* y, int64_t n, double* red, double* out,
                            hipStream_t s);
struct DeflCoef {
    double c[kMaxDefl];
};
// x += sum_t c[t] W[t], r -= sum_t c[t] AW[t]; *rr = r.r afterwards.
hipError_t launch_defl_update(double* x, double* r, const double* W, const double* AW, DeflCoef c, int k, int64_t n,
                              double* red, double* rr, hipStream_t s);
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
