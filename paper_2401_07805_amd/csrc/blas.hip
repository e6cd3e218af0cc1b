// Vector kernels of the Jacobi-preconditioned CG (Krylov solvers of Sec.
// "Numerical framework", stopping rule of Table tab:solver_settings).
//
// All CG scalars live on the device in FP64 (CgState) so that a chunk of
// iterations can be recorded once in a hipGraph and replayed without host
// round trips.  One iteration is three kernels:
//   apply:    the tile kernel of q = A p with per-workgroup partials of p.q
//             (apply kernels; the shared-node assembly is left to update)
//   update:   pAp from those partials; alpha = rz/pAp; q on shared nodes from
//             the apply's partials; r -= alpha q;
//             per-workgroup partial sums of r.r and r.(D^-1 r)
//   pupdate:  every workgroup sums the partials in the same fixed order,
//             beta = rz_new/rz; x += alpha p and p = D^-1 r + beta p in one
//             pass over p; workgroup 0 records the iteration and the stop
//             decision.
// The solution update sits in pupdate because that kernel reads p anyway:
// the iteration then moves 80 instead of 88 bytes per FP64 unknown.
// Reductions use no atomics: a producer writes one partial per workgroup and
// the consumer sums them in a fixed order, so every run gives the same bits.
//
// Stop flags are double-buffered by iteration parity: the kernels of the
// iteration of parity `par` test halt[par], and pupdate(par) writes only
// halt[1-par] (propagating a stop it sees), so no kernel reads a flag that the
// same kernel writes.  Once a stop is set every later kernel returns at once.
#include "blas.h"
#include "shared_nodes.h"

namespace vpp {

constexpr int BT = 256;

// 16-byte packet of T (two doubles or four floats): one dwordx4 access.
template <typename T>
struct alignas(16) Pack {
    static constexpr int W = 16 / (int)sizeof(T);
    T v[W];
};

// Workgroup sums of two doubles in a fixed order (butterfly inside each wave,
// then the waves in index order); every thread receives the totals.
template <int NT>
__device__ __forceinline__ void block_sum2(double& a, double& b)
{
    static_assert(NT % 64 == 0, "whole waves only");
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        a += __shfl_xor(a, o);
        b += __shfl_xor(b, o);
    }
    __shared__ double pa[NT / 64], pb[NT / 64];
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
        pa[threadIdx.x / 64] = a;
        pb[threadIdx.x / 64] = b;
    }
    __syncthreads();
    double sa = 0.0, sb = 0.0;
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) {
        sa += pa[i];
        sb += pb[i];
    }
    a = sa;
    b = sb;
}

// Totals of the ng partials of both quantities (every thread receives them).
__device__ __forceinline__ void sum_partials(const double* red, int ng, double& a, double& b)
{
    a = 0.0;
    b = 0.0;
    for (int i = threadIdx.x; i < ng; i += BT) {
        a += red[i];
        b += red[kMaxRedBlocks + i];
    }
    block_sum2<BT>(a, b);
}

__device__ __forceinline__ void write_partials(double* red, double a, double b, int bid)
{
    if (threadIdx.x == 0) {
        red[bid] = a;
        red[kMaxRedBlocks + bid] = b;
    }
}
__device__ __forceinline__ void write_partials(double* red, double a, double b)
{
    write_partials(red, a, b, blockIdx.x);
}

// Number of workgroups of the streaming kernels (about 4 packets per thread).
template <typename T>
static int grid_for(int64_t n)
{
    const int64_t packets = (n + Pack<T>::W - 1) / Pack<T>::W;
    const int64_t want = (packets + 4 * BT - 1) / (4 * BT);
    return (int)(want < 1 ? 1 : (want > kMaxRedBlocks ? kMaxRedBlocks : want));
}

// Number of workgroups of the fused update and of the search-direction update
// (which sums the former's partials): one packet per thread up to the
// partial-array capacity, since the shared-node lookups make the fused update
// latency-bound rather than bandwidth-bound.
template <typename T>
static int grid_update(int64_t n)
{
    const int64_t packets = (n + Pack<T>::W - 1) / Pack<T>::W;
    const int64_t want = (packets + BT - 1) / BT;
    return (int)(want < 1 ? 1 : (want > kMaxRedBlocks ? kMaxRedBlocks : want));
}

// r = b - q (q may be null: zero initial guess), p = D^-1 r; partials of r.r
// and r.D^-1 r.
template <typename T>
__global__ void __launch_bounds__(BT) cg_init_kernel(double* red, const T* __restrict__ b, const T* __restrict__ q,
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
    block_sum2<BT>(rr, rz);
    write_partials(red, rr, rz);
}

// One workgroup: rr_last = r.r, rz[0] = r.D^-1 r.
__global__ void __launch_bounds__(BT) cg_init_finish_kernel(CgState* st, const double* red, int ng)
{
    double rr, rz;
    sum_partials(red, ng, rr, rz);
    if (threadIdx.x == 0) {
        st->rr_last = rr;
        st->rz[0] = rz;
    }
}

// update fused with the assembly of the apply's shared-node partials: q holds
// A p on the nodes only one tile touches (and on Dirichlet rows); for a shared
// node the value is the sum of its partials in rank order, as the assembly
// kernel forms it.  p.Ap is summed from the apply's per-workgroup partials in
// the same fixed order by every workgroup.
template <typename T>
struct SharedParts {
    SharedEnum e;
    int bcmask;
    const T* part;
    int64_t stride;
    const double* dot_part;
    int ndot;
};

template <typename T>
__device__ __forceinline__ T node_value(const SharedParts<T>& sp, const T* __restrict__ q, int64_t g)
{
    int f, cnt;
    if (!shared_lookup(sp.e, sp.bcmask, (int)g, f, cnt)) return q[g];
    T v = sp.part[f] + sp.part[sp.stride + f];
    for (int c = 2; c < cnt; ++c) v += sp.part[c * sp.stride + f];
    return v;
}

// Body of the update for workgroup bid of nblk (one system); the workgroup
// returns at once when the system has stopped.
template <typename T>
__device__ __forceinline__ void assemble_update_body(int bid, int nblk, CgState* st, int par, double* red,
                                                     const SharedParts<T>& sp, T* __restrict__ r,
                                                     const T* __restrict__ q, const T* __restrict__ invd, int64_t n)
{
    // every state field this kernel needs, read at once (before the barrier of
    // the reduction, so the loads overlap it instead of following it)
    const int halt = st->halt[par];
    const double rz_par = st->rz[par];
    float* hist = nullptr;
    int hit = 0, hcap = 0;
    int64_t hstride = 0;
    if constexpr (sizeof(T) == 4) {
        // residual record of an FP32 phase (iterations counted by the previous
        // direction update, which has completed)
        hist = st->hist;
        hit = st->iters + 1;
        hcap = st->hist_cap;
        hstride = st->hist_stride;
    }
    if (halt) return;
    double pAp = 0.0, unused = 0.0;
    for (int i = threadIdx.x; i < sp.ndot; i += BT) pAp += sp.dot_part[i];
    block_sum2<BT>(pAp, unused);
    if (bid == 0 && threadIdx.x == 0) st->pAp = pAp;
    if (!(pAp > 0.0) || !isfinite(pAp)) {
        if (bid == 0 && threadIdx.x == 0) st->breakdown = 1;
        return;
    }
    const T alpha = T(rz_par / pAp);
    double rr = 0.0, rz = 0.0;
    using P = Pack<T>;
    const int64_t np = n / P::W;
    T* hrec = nullptr;
    if constexpr (sizeof(T) == 4)
        if (hist && hit < hcap) hrec = hist + (size_t)hit * (size_t)hstride;
    for (int64_t c = (int64_t)bid * BT + threadIdx.x; c < np; c += (int64_t)nblk * BT) {
        P rv = reinterpret_cast<const P*>(r)[c];
        const P dv = reinterpret_cast<const P*>(invd)[c];
        P qv = reinterpret_cast<const P*>(q)[c];
        // shared nodes of the packet: all partial loads issued before any use;
        // the row part of the lookup is shared unless the packet wraps a row
        int f[P::W], cnt[P::W];
        const int g0 = (int)(c * P::W);
        const int rw = qdiv(g0, sp.e.nn[0], sp.e.inv_nn[0]);
        const int i0 = g0 - rw * sp.e.nn[0];
        if (i0 + P::W <= sp.e.nn[0]) {
            const int l = qdiv(rw, sp.e.nn[1], sp.e.inv_nn[1]);
            const SharedRow w = shared_row(sp.e, sp.bcmask, rw - l * sp.e.nn[1], l);
#pragma unroll
            for (int j = 0; j < P::W; ++j)
                if (!shared_in_row(sp.e, sp.bcmask, w, i0 + j, f[j], cnt[j])) cnt[j] = 0;
        } else {
#pragma unroll
            for (int j = 0; j < P::W; ++j)
                if (!shared_lookup(sp.e, sp.bcmask, g0 + j, f[j], cnt[j])) cnt[j] = 0;
        }
        // (loaded into pv first, then summed in rank order as a plain loop would)
        T pv[P::W][8];
#pragma unroll
        for (int j = 0; j < P::W; ++j)
#pragma unroll
            for (int k = 0; k < 8; ++k) pv[j][k] = k < cnt[j] ? sp.part[k * sp.stride + f[j]] : T(0);
#pragma unroll
        for (int j = 0; j < P::W; ++j)
            if (cnt[j]) {
                T v = pv[j][0] + pv[j][1];
#pragma unroll
                for (int k = 2; k < 8; ++k)
                    if (k < cnt[j]) v += pv[j][k];
                qv.v[j] = v;
            }
#pragma unroll
        for (int j = 0; j < P::W; ++j) {
            const T ri = fma(-alpha, qv.v[j], rv.v[j]);
            rv.v[j] = ri;
            rr += (double)ri * (double)ri;
            rz += (double)ri * (double)(ri * dv.v[j]);
        }
        reinterpret_cast<P*>(r)[c] = rv;
        if (hrec) reinterpret_cast<P*>(hrec)[c] = rv;
    }
    if (bid == 0)
        for (int64_t i = np * P::W + threadIdx.x; i < n; i += BT) {
            const T ri = fma(-alpha, node_value(sp, q, i), r[i]);
            r[i] = ri;
            if (hrec) hrec[i] = ri;
            rr += (double)ri * (double)ri;
            rz += (double)ri * (double)(ri * invd[i]);
        }
    block_sum2<BT>(rr, rz);
    write_partials(red, rr, rz, bid);
}

template <typename T>
__global__ void __launch_bounds__(BT) cg_assemble_update_kernel(CgState* st, int par, double* red, SharedParts<T> sp,
                                                                T* __restrict__ r, const T* __restrict__ q,
                                                                const T* __restrict__ invd, int64_t n)
{
    assemble_update_body<T>(blockIdx.x, gridDim.x, st, par, red, sp, r, q, invd, n);
}

// Packets a thread handles per batch in the search-direction update.  A
// thread takes packets c, c + S, c + 2S, ... (S = threads of the system's
// grid) in that order, as a plain grid-stride loop would, but loads a whole
// batch before it uses any of it, and the first batch before the reduction
// that gives beta: each batch then costs one memory latency instead of one
// per packet.
constexpr int kBatch = 4;

// Body of the search-direction update for workgroup bid of nblk (one system;
// ng partials of the update to sum).
template <typename T>
__device__ __forceinline__ void pupdate_body(int bid, int nblk, CgState* st, int par, const double* red, int ng,
                                             T* __restrict__ x, const T* __restrict__ r, T* __restrict__ p,
                                             const T* __restrict__ invd, int64_t n)
{
    // every state field this kernel reads, at once (before the reduction's
    // barrier); thread 0 of workgroup 0 is the only writer, of other fields
    const int halt = st->halt[par], brk = st->breakdown;
    const double rz_par = st->rz[par], pAp_par = st->pAp, tol2 = st->tol2;
    const int iters0 = st->iters, max_iter = st->max_iter, hcap = st->hist_cap;
    double* const coef = st->coef;
    if (halt || brk) {
        if (bid == 0 && threadIdx.x == 0) st->halt[1 - par] = 1;
        return;
    }
    using P = Pack<T>;
    constexpr int W = P::W, U = kBatch;
    const int64_t np = n / W;
    const int64_t S = (int64_t)nblk * BT;
    const int64_t c0 = (int64_t)bid * BT + threadIdx.x;
    P rv[U], dv[U], pv[U], xv[U];
    auto load = [&](int64_t cb) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = cb + u * S;
            if (c < np) {
                rv[u] = reinterpret_cast<const P*>(r)[c];
                dv[u] = reinterpret_cast<const P*>(invd)[c];
                pv[u] = reinterpret_cast<const P*>(p)[c];
                xv[u] = reinterpret_cast<const P*>(x)[c];
            }
        }
    };
    load(c0);
    double rr, rzn;
    sum_partials(red, ng, rr, rzn);
    const double beta_d = rzn / rz_par;
    if (bid == 0 && threadIdx.x == 0) {
        const int it = iters0 + 1;
        st->iters = it;
        st->rr_last = rr;
        st->rr[par] = rr;
        st->rznew[par] = rzn;
        st->rz[1 - par] = rzn;
        if (!isfinite(rr) || !isfinite(rzn)) {
            st->breakdown = 1;
            st->halt[1 - par] = 1;
        } else if (rr < tol2 || it >= max_iter) {
            st->halt[1 - par] = 1;
        }
        if (coef && it < hcap) {
            coef[3 * it] = rz_par / pAp_par;
            coef[3 * it + 1] = beta_d;
            coef[3 * it + 2] = rzn;
        }
    }
    // the same alpha as the update's (same operands, same rounding)
    const T alpha = T(rz_par / pAp_par);
    const T beta = T(beta_d);
    for (int64_t cb = c0; cb < np; cb += U * S) {
        if (cb != c0) load(cb);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t c = cb + u * S;
            if (c >= np) break;
#pragma unroll
            for (int j = 0; j < W; ++j) {
                xv[u].v[j] = fma(alpha, pv[u].v[j], xv[u].v[j]);
                pv[u].v[j] = fma(beta, pv[u].v[j], rv[u].v[j] * dv[u].v[j]);
            }
            reinterpret_cast<P*>(x)[c] = xv[u];
            reinterpret_cast<P*>(p)[c] = pv[u];
        }
    }
    if (bid == 0)
        for (int64_t i = np * W + threadIdx.x; i < n; i += BT) {
            x[i] = fma(alpha, p[i], x[i]);
            p[i] = fma(beta, p[i], r[i] * invd[i]);
        }
}

template <typename T>
__global__ void __launch_bounds__(BT) cg_pupdate_kernel(CgState* st, int par, const double* red, int ng,
                                                        T* __restrict__ x, const T* __restrict__ r,
                                                        T* __restrict__ p, const T* __restrict__ invd, int64_t n)
{
    pupdate_body<T>(blockIdx.x, gridDim.x, st, par, red, ng, x, r, p, invd, n);
}

// ---------------------------------------------------------------------------
// Batched PCG: the update and the search-direction update of every system of a
// batch in one launch each.  System i owns workgroups [blk_begin, blk_begin +
// nblk) of the grid, nblk being what the single-system launch would use, so
// each system's reductions are summed in the same order as in a single solve.

template <typename T>
__device__ __forceinline__ int system_of_block(const CgSystem<T>* sys, int nsys)
{
    int s = 0;
    for (int i = 1; i < nsys; ++i)
        if (sys[i].blk_begin <= (int)blockIdx.x) s = i;
    return s;
}

template <typename T>
__global__ void __launch_bounds__(BT) cg_batch_update_kernel(const CgSystem<T>* sys, int nsys, int par, int* queue)
{
    // the batched apply that precedes this launch pulls work items from queue
    if (queue && blockIdx.x == 0 && threadIdx.x == 0) *queue = 0;
    const CgSystem<T>& y = sys[system_of_block(sys, nsys)];
    const SharedParts<T> sp{y.e, y.bcmask, y.part, y.stride, y.dot_part, y.ndot};
    assemble_update_body<T>((int)blockIdx.x - y.blk_begin, y.nblk, y.st, par, y.red, sp, y.r, y.q, y.invd, y.n);
}

template <typename T>
__global__ void __launch_bounds__(BT) cg_batch_pupdate_kernel(const CgSystem<T>* sys, int nsys, int par)
{
    const CgSystem<T>& y = sys[system_of_block(sys, nsys)];
    pupdate_body<T>((int)blockIdx.x - y.blk_begin, y.nblk, y.st, par, y.red, y.nblk, y.x, y.r, y.p, y.invd, y.n);
}

// r = b - q in FP64 and partials of r.r (outer residual of the mixed solver and
// the true residual at the end of every solve).
__global__ void __launch_bounds__(BT) residual_kernel(const double* __restrict__ b, const double* __restrict__ q,
                                                      double* __restrict__ r, int64_t n, double* red)
{
    double s = 0.0, unused = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const double v = b[i] - q[i];
        if (r) r[i] = v;
        s += v * v;
    }
    block_sum2<BT>(s, unused);
    write_partials(red, s, 0.0);
}

__global__ void __launch_bounds__(BT) sum_finish_kernel(const double* red, int ng, double* out)
{
    double a, b;
    sum_partials(red, ng, a, b);
    if (threadIdx.x == 0) *out = a;
}

__global__ void __launch_bounds__(BT) cg_replace32_kernel(const double* __restrict__ r64, double scale,
                                                          double pscale, float* __restrict__ r32,
                                                          float* __restrict__ p32, float* __restrict__ x32,
                                                          const float* __restrict__ invd, int64_t n, double* red)
{
    double rr = 0.0, rz = 0.0;
    const float ps = (float)pscale;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const float ri = (float)(scale * r64[i]);
        const float zi = ri * invd[i];
        r32[i] = ri;
        x32[i] = 0.0f;
        p32[i] = pscale == 0.0 ? zi : ps * p32[i];
        rr += (double)ri * (double)ri;
        rz += (double)ri * (double)zi;
    }
    block_sum2<BT>(rr, rz);
    write_partials(red, rr, rz);
}

// One workgroup: restart the inner state at parity 0 after a replacement.
__global__ void __launch_bounds__(BT) cg_resume_kernel(CgState* st, const double* red, int ng)
{
    double rr, rz;
    sum_partials(red, ng, rr, rz);
    if (threadIdx.x == 0) {
        st->rz[0] = rz;
        st->rr_last = rr;
        st->halt[0] = 0;
        st->halt[1] = 0;
        st->breakdown = 0;
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

template <typename T>
hipError_t launch_cg_init(CgState* st, double* red, const T* b, const T* q, T* r, T* p, const T* invd, int64_t n,
                          hipStream_t s)
{
    const int g = grid_for<T>(n);
    hipLaunchKernelGGL(cg_init_kernel<T>, dim3(g), dim3(BT), 0, s, red, b, q, r, p, invd, n);
    hipLaunchKernelGGL(cg_init_finish_kernel, dim3(1), dim3(BT), 0, s, st, red, g);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_assemble_update(CgState* st, int par, double* red, const double* dot_part, int ndot,
                                     const MeshArgs& m, const SharedEnum& e, const T* part, int64_t stride, T* r,
                                     const T* q, const T* invd, int64_t n, hipStream_t s)
{
    SharedParts<T> sp{e, m.bcmask, part, stride, dot_part, ndot};
    hipLaunchKernelGGL(cg_assemble_update_kernel<T>, dim3(grid_update<T>(n)), dim3(BT), 0, s, st, par, red, sp, r,
                       q, invd, n);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_cg_pupdate(CgState* st, int par, const double* red, T* x, const T* r, T* p, const T* invd,
                             int64_t n, hipStream_t s)
{
    const int g = grid_update<T>(n);   // also the number of partials the update wrote
    hipLaunchKernelGGL(cg_pupdate_kernel<T>, dim3(g), dim3(BT), 0, s, st, par, red, g, x, r, p, invd, n);
    return hipGetLastError();
}

int cg_update_blocks(int64_t n) { return grid_update<double>(n); }

hipError_t launch_cg_batch_step(const CgSystem<double>* sys, int nsys, int total_blocks, int par, int* queue,
                                hipStream_t s)
{
    hipLaunchKernelGGL(cg_batch_update_kernel<double>, dim3(total_blocks), dim3(BT), 0, s, sys, nsys, par, queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(cg_batch_pupdate_kernel<double>, dim3(total_blocks), dim3(BT), 0, s, sys, nsys, par);
    return hipGetLastError();
}

#define VPP_INST(T)                                                                                          \
    template hipError_t launch_cg_init<T>(CgState*, double*, const T*, const T*, T*, T*, const T*, int64_t,  \
                                          hipStream_t);                                                      \
    template hipError_t launch_cg_pupdate<T>(CgState*, int, const double*, T*, const T*, T*, const T*, int64_t, \
                                             hipStream_t);                                                       \
    template hipError_t launch_cg_assemble_update<T>(CgState*, int, double*, const double*, int, const MeshArgs&, \
                                                     const SharedEnum&, const T*, int64_t, T*, const T*,          \
                                                     const T*, int64_t, hipStream_t);
VPP_INST(double)
VPP_INST(float)
#undef VPP_INST

// ---------------------------------------------------------------------------
// Deflation space of the mixed-precision solver (Ritz vectors of the first
// FP32 phase and the Galerkin correction in their span).

// One unknown per thread; the recorded residuals are read eight at a time
// (all loads of a group issued before their use).
__global__ void __launch_bounds__(BT) ritz_kernel(const float* __restrict__ hist, int64_t stride, int m,
                                                  const double* __restrict__ C, int k,
                                                  const double* __restrict__ invd, double* __restrict__ W, int64_t n)
{
    constexpr int G = 8;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        double acc[kMaxDefl];
#pragma unroll
        for (int t = 0; t < kMaxDefl; ++t) acc[t] = 0.0;
        const float* col = hist + (size_t)i;
        for (int j0 = 0; j0 < m; j0 += G) {
            float h[G];
#pragma unroll
            for (int u = 0; u < G; ++u) h[u] = (j0 + u < m) ? col[(size_t)(j0 + u) * (size_t)stride] : 0.0f;
#pragma unroll
            for (int u = 0; u < G; ++u) {
                if (j0 + u >= m) break;
#pragma unroll
                for (int t = 0; t < kMaxDefl; ++t)
                    if (t < k) acc[t] = fma(C[(j0 + u) * k + t], (double)h[u], acc[t]);
            }
        }
        const double di = invd[i];
#pragma unroll
        for (int t = 0; t < kMaxDefl; ++t)
            if (t < k) W[(size_t)t * (size_t)n + (size_t)i] = acc[t] * di;
    }
}

__global__ void __launch_bounds__(BT) multi_dot_kernel(const double* __restrict__ V, int k,
                                                       const double* __restrict__ y, int64_t n, double* red)
{
    double acc[kMaxDefl];
#pragma unroll
    for (int t = 0; t < kMaxDefl; ++t) acc[t] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        const double yi = y[i];
#pragma unroll
        for (int t = 0; t < kMaxDefl; ++t)
            if (t < k) acc[t] = fma(V[(size_t)t * (size_t)n + (size_t)i], yi, acc[t]);
    }
#pragma unroll
    for (int t = 0; t < kMaxDefl; t += 2) {
        double a = acc[t], b = acc[t + 1];
        block_sum2<BT>(a, b);
        if (threadIdx.x == 0) {
            if (t < k) red[(size_t)t * kMaxRedBlocks + blockIdx.x] = a;
            if (t + 1 < k) red[(size_t)(t + 1) * kMaxRedBlocks + blockIdx.x] = b;
        }
    }
}

__global__ void __launch_bounds__(BT) multi_dot_finish_kernel(const double* red, int k, int ng, double* out)
{
    for (int t = 0; t < k; t += 2) {
        double a = 0.0, b = 0.0;
        for (int i = threadIdx.x; i < ng; i += BT) {
            a += red[(size_t)t * kMaxRedBlocks + i];
            if (t + 1 < k) b += red[(size_t)(t + 1) * kMaxRedBlocks + i];
        }
        block_sum2<BT>(a, b);
        if (threadIdx.x == 0) {
            out[t] = a;
            if (t + 1 < k) out[t + 1] = b;
        }
    }
}

__global__ void __launch_bounds__(BT) defl_update_kernel(double* __restrict__ x, double* __restrict__ r,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ AW, DeflCoef c, int k,
                                                         int64_t n, double* red)
{
    double s2 = 0.0, unused = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * BT + threadIdx.x; i < n; i += (int64_t)gridDim.x * BT) {
        double xi = x[i], ri = r[i];
#pragma unroll
        for (int t = 0; t < kMaxDefl; ++t)
            if (t < k) {
                xi = fma(c.c[t], W[(size_t)t * (size_t)n + (size_t)i], xi);
                ri = fma(-c.c[t], AW[(size_t)t * (size_t)n + (size_t)i], ri);
            }
        x[i] = xi;
        r[i] = ri;
        s2 += ri * ri;
    }
    block_sum2<BT>(s2, unused);
    write_partials(red, s2, 0.0);
}

hipError_t launch_ritz(const float* hist, int64_t stride, int m, const double* C, int k, const double* invd,
                       double* W, int64_t n, hipStream_t s)
{
    if (k < 1 || k > kMaxDefl) return hipErrorInvalidValue;
    const int64_t want = (n + BT - 1) / BT;
    const int g = (int)(want < 1 ? 1 : (want > 65536 ? 65536 : want));
    hipLaunchKernelGGL(ritz_kernel, dim3(g), dim3(BT), 0, s, hist, stride, m, C, k, invd, W, n);
    return hipGetLastError();
}

hipError_t launch_multi_dot(const double* V, int k, const double* y, int64_t n, double* red, double* out,
                            hipStream_t s)
{
    if (k < 1 || k > kMaxDefl) return hipErrorInvalidValue;
    const int g = grid_for<double>(n);
    hipLaunchKernelGGL(multi_dot_kernel, dim3(g), dim3(BT), 0, s, V, k, y, n, red);
    hipLaunchKernelGGL(multi_dot_finish_kernel, dim3(1), dim3(BT), 0, s, red, k, g, out);
    return hipGetLastError();
}

hipError_t launch_defl_update(double* x, double* r, const double* W, const double* AW, DeflCoef c, int k, int64_t n,
                              double* red, double* rr, hipStream_t s)
{
    if (k < 1 || k > kMaxDefl) return hipErrorInvalidValue;
    const int g = grid_for<double>(n);
    hipLaunchKernelGGL(defl_update_kernel, dim3(g), dim3(BT), 0, s, x, r, W, AW, c, k, n, red);
    hipLaunchKernelGGL(sum_finish_kernel, dim3(1), dim3(BT), 0, s, red, g, rr);
    return hipGetLastError();
}

hipError_t launch_residual(const double* b, const double* q, double* r, int64_t n, double* red, double* rr,
                           hipStream_t s)
{
    const int g = grid_for<double>(n);
    hipLaunchKernelGGL(residual_kernel, dim3(g), dim3(BT), 0, s, b, q, r, n, red);
    hipLaunchKernelGGL(sum_finish_kernel, dim3(1), dim3(BT), 0, s, red, g, rr);
    return hipGetLastError();
}

hipError_t launch_cg_replace32(CgState* st, double* red, const double* r64, double scale, double pscale,
                               float* r32, float* p32, float* x32, const float* invd, int64_t n, hipStream_t s)
{
    const int g = grid_for<float>(n);
    hipLaunchKernelGGL(cg_replace32_kernel, dim3(g), dim3(BT), 0, s, r64, scale, pscale, r32, p32, x32, invd, n,
                       red);
    hipLaunchKernelGGL(cg_resume_kernel, dim3(1), dim3(BT), 0, s, st, red, g);
    return hipGetLastError();
}

static int grid_plain(int64_t n)
{
    const int64_t want = (n + BT - 1) / BT;
    return (int)(want < 2048 ? (want < 1 ? 1 : want) : 2048);
}

hipError_t launch_convert(const double* a, float* b, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(convert_kernel, dim3(grid_plain(n)), dim3(BT), 0, s, a, b, n);
    return hipGetLastError();
}

hipError_t launch_promote_add(double* x, const float* d, double scale, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(promote_add_kernel, dim3(grid_plain(n)), dim3(BT), 0, s, x, d, scale, n);
    return hipGetLastError();
}

}  // namespace vpp
