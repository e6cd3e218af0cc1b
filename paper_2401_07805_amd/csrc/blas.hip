// Vector kernels of the Jacobi-preconditioned CG (Krylov solvers of Sec.
// "Numerical framework", stopping rule of Table tab:solver_settings).
//
// All CG scalars live on the device in FP64 (CgState) so that a chunk of
// iterations can be recorded once in a hipGraph and replayed without host
// round trips.  One iteration is three kernels:
//   apply:    q = A p and pAp = p.q                         (apply kernels)
//   update:   alpha = rz/pAp; x += alpha p; r -= alpha q;
//             accumulate r.r and r.(D^-1 r)
//   pupdate:  beta = rz_new/rz; p = D^-1 r + beta p;
//             block 0 records the iteration and the convergence flag and
//             clears the accumulators of the next iteration.
// The accumulated scalars are double-buffered by iteration parity, so no
// kernel ever reads a scalar that the same kernel writes.  Once `done` is set, every
// kernel returns immediately, so replays past convergence change nothing.
#include "blas.h"

namespace vpp {

template <int NT>
__device__ __forceinline__ void block_sum2(double a, double b, double* outa, double* outb)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    __shared__ double pa[NT / 64], pb[NT / 64];
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        pa[w] = a;
        pb[w] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double sa = 0.0, sb = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            sa += pa[i];
            sb += pb[i];
        }
        if (outa) atomicAdd(outa, sa);
        if (outb) atomicAdd(outb, sb);
    }
}

constexpr int BT = 256;

// r = b - q (q may be null: zero initial guess), p = D^-1 r; the initial r.r is
// accumulated into rr_last and r.D^-1 r into rz[0] (both zeroed by the host).
template <typename T>
__global__ void __launch_bounds__(BT) cg_init_kernel(CgState* st, const T* __restrict__ b, const T* __restrict__ q,
                                                     T* __restrict__ r, T* __restrict__ p,
                                                     const T* __restrict__ invd, int64_t n)
{
    double rr = 0.0, rz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const T ri = q ? b[i] - q[i] : b[i];
        const T zi = ri * invd[i];
        r[i] = ri;
        p[i] = zi;
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)zi;
    }
    block_sum2<BT>(rr, rz, &st->rr_last, &st->rz[0]);
}

template <typename T>
__global__ void __launch_bounds__(BT) cg_update_kernel(CgState* st, int par, T* __restrict__ x, T* __restrict__ r,
                                                       const T* __restrict__ p, const T* __restrict__ q,
                                                       const T* __restrict__ invd, int64_t n)
{
    if (st->done) return;
    const double pAp = st->pAp;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        if (blockIdx.x == 0 && threadIdx.x == 0) {
            st->breakdown = 1;
            st->done = 1;
        }
        return;
    }
    const double alpha_d = st->rz[par] / pAp;
    const T alpha = T(alpha_d);
    double rr = 0.0, rz = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        x[i] = fma(alpha, p[i], x[i]);
        const T ri = fma(-alpha, q[i], r[i]);
        r[i] = ri;
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)(ri * invd[i]);
    }
    block_sum2<BT>(rr, rz, &st->rr[par], &st->rznew[par]);
}

template <typename T>
__global__ void __launch_bounds__(BT) cg_pupdate_kernel(CgState* st, int par, const T* __restrict__ r, T* __restrict__ p,
                                                        T* __restrict__ q, const T* __restrict__ invd, int64_t n)
{
    if (st->done) return;
    const double rznew = st->rznew[par];
    const double beta_d = rznew / st->rz[par];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        const double rr = st->rr[par];
        st->iters += 1;
        st->rr_last = rr;
        st->rz[1 - par] = rznew;
        st->rr[1 - par] = 0.0;
        st->rznew[1 - par] = 0.0;
        if (!isfinite(rr) || !isfinite(rznew)) {
            st->breakdown = 1;
            st->done = 1;
        } else if (rr < st->tol2 || st->iters >= st->max_iter) {
            st->done = 1;
        }
    }
    const T beta = T(beta_d);
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT)
        p[i] = fma(beta, p[i], r[i] * invd[i]);
}

// r = b - q in FP64 and its squared norm (outer residual of the mixed solver and
// the true residual at the end of every solve).
__global__ void __launch_bounds__(BT) residual_kernel(const double* __restrict__ b, const double* __restrict__ q,
                                                      double* __restrict__ r, int64_t n, double* rr)
{
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const double v = b[i] - q[i];
        if (r) r[i] = v;
        s += v * v;
    }
    block_sum2<BT>(s, 0.0, rr, nullptr);
}

// r32 = (float)(scale r64); the FP32 inner iterate starts at zero.
__global__ void __launch_bounds__(BT) demote_kernel(const double* __restrict__ r, double scale, float* __restrict__ r32,
                                                    float* __restrict__ x32, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        r32[i] = (float)(scale * r[i]);
        x32[i] = 0.0f;
    }
}

__global__ void __launch_bounds__(BT) convert_kernel(const double* __restrict__ a, float* __restrict__ b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) b[i] = (float)a[i];
}

// x += scale * d32, in FP64.
__global__ void __launch_bounds__(BT) promote_add_kernel(double* __restrict__ x, const float* __restrict__ d,
                                                         double scale, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT)
        x[i] = fma(scale, (double)d[i], x[i]);
}

static int grid_for(int64_t n)
{
    const int64_t want = (n + BT - 1) / BT;
    return (int)(want < 2048 ? (want < 1 ? 1 : want) : 2048);
}

template <typename T>
hipError_t launch_cg_init(CgState* st, const T* b, const T* q, T* r, T* p, const T* invd, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(cg_init_kernel<T>, dim3(grid_for(n)), dim3(BT), 0, s, st, b, q, r, p, invd, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_update(CgState* st, int par, T* x, T* r, const T* p, const T* q, const T* invd, int64_t n,
                            hipStream_t s)
{
    hipLaunchKernelGGL(cg_update_kernel<T>, dim3(grid_for(n)), dim3(BT), 0, s, st, par, x, r, p, q, invd, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_pupdate(CgState* st, int par, const T* r, T* p, T* q, const T* invd, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(cg_pupdate_kernel<T>, dim3(grid_for(n)), dim3(BT), 0, s, st, par, r, p, q, invd, n);
    return hipGetLastError();
}

#define VPP_INST(T)                                                                                       \
    template hipError_t launch_cg_init<T>(CgState*, const T*, const T*, T*, T*, const T*, int64_t,        \
                                          hipStream_t);                                                   \
    template hipError_t launch_cg_update<T>(CgState*, int, T*, T*, const T*, const T*, const T*, int64_t, \
                                            hipStream_t);                                                 \
    template hipError_t launch_cg_pupdate<T>(CgState*, int, const T*, T*, T*, const T*, int64_t, hipStream_t);
VPP_INST(double)
VPP_INST(float)
#undef VPP_INST

hipError_t launch_residual(const double* b, const double* q, double* r, int64_t n, double* rr, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(grid_for(n)), dim3(BT), 0, s, b, q, r, n, rr);
    return hipGetLastError();
}

hipError_t launch_demote(const double* r, double scale, float* r32, float* x32, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(demote_kernel, dim3(grid_for(n)), dim3(BT), 0, s, r, scale, r32, x32, n);
    return hipGetLastError();
}

hipError_t launch_convert(const double* a, float* b, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(convert_kernel, dim3(grid_for(n)), dim3(BT), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t launch_promote_add(double* x, const float* d, double scale, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(promote_add_kernel, dim3(grid_for(n)), dim3(BT), 0, s, x, d, scale, n);
    return hipGetLastError();
}

}  // namespace vpp
