// Pressure operator on a once-refined mesh with hanging nodes (adaptive
// refinement of Sec. "Numerical framework", one level): kernels.
//
// The unknowns of the two lattices sit in one vector: the coarse lattice
// (entries [0, nc)) and the fine lattice over the whole box (entries [nc, n)).
// Each active cell (an unrefined coarse cell, or one of the eight fine cells of
// a refined one) is one thread: it gathers its (k+1)^3 values, applies the
// cell operator by sum factorisation (the same building blocks as the uniform
// apply, with the cell size of its lattice) and stores its results in a
// cell-major scratch; a second launch sums every entry of y over the cell
// results that reach it, through a list built on the host, in a fixed order
// (the diagonal likewise).  A fine node on the boundary of an unrefined coarse cell is
// constrained: its value is sum_p w_p x[src_p] over the coarse cell's nodes
// (the Q_k interpolant there), and its result goes back to those nodes with
// the same weights (C^T).  Entries that are not free unknowns (unused nodes of
// either lattice, constrained fine nodes) and free unknowns on Dirichlet faces
// are identity rows: gathers read them as zero, and a last pass sets y = x.
#include "amr.h"
#include "apply_impl.h"

namespace vpp {

template <int K>
__device__ __forceinline__ int64_t amr_local(const MeshArgs& m, int64_t base, int a)
{
    constexpr int N = K + 1;
    const int a0 = a % N, a1 = (a / N) % N, a2 = a / (N * N);
    return base + a0 + (int64_t)m.nn[0] * (a1 + (int64_t)m.nn[1] * a2);
}

// Lattice index of local node 0 of cell idx of lattice m.
template <int K>
__device__ __forceinline__ int64_t amr_base(const MeshArgs& m, int idx)
{
    const int cx = idx % m.nc[0], cy = (idx / m.nc[0]) % m.nc[1], cz = idx / (m.nc[0] * m.nc[1]);
    return node_index(m, (int64_t)K * cx, (int64_t)K * cy, (int64_t)K * cz);
}

// Value of the unknown at vector entry g as a gather sees it: zero for
// identity rows.
__device__ __forceinline__ double amr_read(const AmrArgs& a, const double* __restrict__ x, int64_t g)
{
    return a.ident[g] ? 0.0 : x[g];
}

// Constraint list of local node gl of a cell of lattice FINE (-1: none).
template <bool FINE>
__device__ __forceinline__ int amr_kind(const AmrArgs& a, int64_t gl)
{
    if constexpr (FINE) return a.fkind[gl];
    else return -1;
}

template <int K, int HV>
__device__ __forceinline__ void amr_coefficient(const MeshArgs& m, int64_t base, int64_t off,
                                                const double* __restrict__ phi,
                                                double (&cw)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
#pragma unroll
    for (int q = 0; q < N3; ++q) cw[q] = phi[off + amr_local<K>(m, base, q)];
    sweep3<K, MS, false, 0>(cw);
    sweep3<K, MS, false, 1>(cw);
    sweep3<K, MS, false, 2>(cw);
    coef_weights3<K, HV>(m, cw);
}

// One active cell of lattice m (FINE: the fine lattice, whose nodes may be
// constrained).
template <int K, int HV, bool FINE>
__device__ __forceinline__ void amr_apply_cell(const AmrArgs& a, const MeshArgs& m, int idx, int e,
                                               const double* __restrict__ phi, const double* __restrict__ x)
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
    const int64_t base = amr_base<K>(m, idx), off = FINE ? a.nc : 0;
    double cw[N3], u[N3];
    amr_coefficient<K, HV>(m, base, off, phi, cw);
    // gather in stages, each stage's loads issued together: the constraint
    // kinds of the cell's nodes, then x and the identity flag of every free
    // node, then the constrained nodes' terms
    int kind[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) kind[q] = amr_kind<FINE>(a, amr_local<K>(m, base, q));
    unsigned char idb[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q)
        if (kind[q] < 0) {
            const int64_t g = off + amr_local<K>(m, base, q);
            u[q] = x[g];
            idb[q] = a.ident[g];
        }
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        if (kind[q] < 0) {
            if (idb[q]) u[q] = 0.0;
        } else {
            double s = 0.0;
            for (int p = a.cptr[kind[q]]; p < a.cptr[kind[q] + 1]; ++p)
                s = fma(a.cw[p], amr_read(a, x, a.ccol[p]), s);
            u[q] = s;
        }
    }
    cell_operator<K, double>(m, cw, u);
#pragma unroll
    for (int q = 0; q < N3; ++q) a.scratch[(size_t)q * (size_t)a.ncells + (size_t)e] = u[q];
}

template <int K, int HV>
__global__ void __launch_bounds__(64) amr_apply_kernel(AmrArgs a, const double* __restrict__ phi,
                                                       const double* __restrict__ x)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.ncells) return;
    const int code = a.cells[e];
    if (code >= 0) amr_apply_cell<K, HV, false>(a, a.mc, code, e, phi, x);
    else amr_apply_cell<K, HV, true>(a, a.mf, -(code + 1), e, phi, x);
}

// y[g] = x[g] on identity rows, else the sum of the cell results reaching g.
__global__ void amr_node_sum_kernel(AmrArgs a, const double* __restrict__ x, double* __restrict__ y)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        if (a.ident[g]) {
            y[g] = x[g];
            continue;
        }
        double v = 0.0;
        for (int j = a.nptr[g]; j < a.nptr[g + 1]; ++j) v = fma(a.nw[j], a.scratch[a.nidx[j]], v);
        y[g] = v;
    }
}

// Diagonal of C^T K_e C for one cell: K_aa from the squared 1D tables for the
// free nodes; for the coarse nodes that constrained nodes of the cell draw on,
// e_i^T K_e e_i with e_i the cell vector of node i's weights, K_e applied by
// the cell operator (each such coarse node once per cell).
template <int K, int HV, bool FINE>
__device__ __forceinline__ void amr_diag_cell(const AmrArgs& a, const MeshArgs& m, int idx, int e,
                                              const double* __restrict__ phi)
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
    const int64_t base = amr_base<K>(m, idx), off = FINE ? a.nc : 0;
    double cw[N3];
    amr_coefficient<K, HV>(m, base, off, phi, cw);
    {
        double A[N3], Z[N3], Y[N3], out[N3];
#pragma unroll
        for (int q = 0; q < N3; ++q) A[q] = cw[q];
#pragma unroll
        for (int q = 0; q < N3; ++q) Z[q] = A[q];
        sweep3<K, MS2, true, 2>(Z);
#pragma unroll
        for (int q = 0; q < N3; ++q) Y[q] = Z[q];
        sweep3<K, MS2, true, 1>(Y);
        sweep3<K, MD2, true, 0>(Y);
#pragma unroll
        for (int q = 0; q < N3; ++q) out[q] = m.rd[0] * Y[q];
#pragma unroll
        for (int q = 0; q < N3; ++q) Y[q] = Z[q];
        sweep3<K, MD2, true, 1>(Y);
        sweep3<K, MS2, true, 0>(Y);
#pragma unroll
        for (int q = 0; q < N3; ++q) out[q] = fma(m.rd[1], Y[q], out[q]);
        sweep3<K, MD2, true, 2>(A);
        sweep3<K, MS2, true, 1>(A);
        sweep3<K, MS2, true, 0>(A);
#pragma unroll
        for (int q = 0; q < N3; ++q) out[q] = fma(m.rd[2], A[q], out[q]);
#pragma unroll
        for (int q = 0; q < N3; ++q) {
            const int64_t gl = amr_local<K>(m, base, q);
            if (amr_kind<FINE>(a, gl) < 0) a.scratch[(size_t)q * (size_t)a.ncells + (size_t)e] = out[q];
        }
    }
    if constexpr (FINE) {
        // coarse nodes reached through constraints: visit each (node q, term p)
        // pair and handle its coarse node at its first occurrence in that order
        // (the host numbers the slots in the same order)
        int64_t slot = a.nfree_slots + a.soff[e];
        for (int q = 0; q < N3; ++q) {
            const int kq = a.fkind[amr_local<K>(m, base, q)];
            if (kq < 0) continue;
            for (int p = a.cptr[kq]; p < a.cptr[kq + 1]; ++p) {
                const int src = a.ccol[p];
                bool seen = false;
                for (int q2 = 0; q2 <= q && !seen; ++q2) {
                    const int k2 = a.fkind[amr_local<K>(m, base, q2)];
                    if (k2 < 0) continue;
                    const int pend = (q2 == q) ? p : a.cptr[k2 + 1];
                    for (int p2 = a.cptr[k2]; p2 < pend; ++p2)
                        if (a.ccol[p2] == src) seen = true;
                }
                if (seen) continue;
                double ev[N3], kv[N3];
                for (int r = 0; r < N3; ++r) {
                    double w = 0.0;
                    const int kr = a.fkind[amr_local<K>(m, base, r)];
                    if (kr >= 0)
                        for (int p2 = a.cptr[kr]; p2 < a.cptr[kr + 1]; ++p2)
                            if (a.ccol[p2] == src) w += a.cw[p2];
                    ev[r] = w;
                    kv[r] = w;
                }
                cell_operator<K, double>(m, cw, kv);
                double d = 0.0;
                for (int r = 0; r < N3; ++r) d = fma(ev[r], kv[r], d);
                a.scratch[slot++] = d;
            }
        }
    }
}

template <int K, int HV>
__global__ void __launch_bounds__(64) amr_diag_kernel(AmrArgs a, const double* __restrict__ phi)
{
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= a.ncells) return;
    const int code = a.cells[e];
    if (code >= 0) amr_diag_cell<K, HV, false>(a, a.mc, code, e, phi);
    else amr_diag_cell<K, HV, true>(a, a.mf, -(code + 1), e, phi);
}

// diag = 1 on identity rows, else the sum of its cell slots; then the FP64
// and FP32 inverses.
__global__ void amr_fix_diag_kernel(AmrArgs a, double* __restrict__ diag, double* __restrict__ inv64,
                                    float* __restrict__ inv32)
{
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < a.n; g += (int64_t)gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int j = a.dptr[g]; j < a.dptr[g + 1]; ++j) s += a.scratch[a.didx[j]];
        const double d = a.ident[g] ? 1.0 : s;
        diag[g] = d;
        inv64[g] = 1.0 / d;
        inv32[g] = (float)(1.0 / d);
    }
}

static int stream_blocks(int64_t n)
{
    const int64_t want = (n + 255) / 256;
    return (int)(want < 8192 ? (want < 1 ? 1 : want) : 8192);
}

#define VPP_AMR_SWITCH(KERNEL, ...)                                                                       \
    switch (k * 4 + a.mc.heaviside) {                                                                     \
    case 8: hipLaunchKernelGGL((KERNEL<2, 0>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;    \
    case 9: hipLaunchKernelGGL((KERNEL<2, 1>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;    \
    case 10: hipLaunchKernelGGL((KERNEL<2, 2>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 11: hipLaunchKernelGGL((KERNEL<2, 3>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 12: hipLaunchKernelGGL((KERNEL<3, 0>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 13: hipLaunchKernelGGL((KERNEL<3, 1>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 14: hipLaunchKernelGGL((KERNEL<3, 2>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 15: hipLaunchKernelGGL((KERNEL<3, 3>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 16: hipLaunchKernelGGL((KERNEL<4, 0>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 17: hipLaunchKernelGGL((KERNEL<4, 1>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 18: hipLaunchKernelGGL((KERNEL<4, 2>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    case 19: hipLaunchKernelGGL((KERNEL<4, 3>), dim3(blocks), dim3(64), 0, s, a, __VA_ARGS__); break;   \
    default: return hipErrorInvalidValue;                                                                 \
    }

hipError_t launch_amr_apply(int k, const AmrArgs& a, const double* phi, const double* x, double* y, hipStream_t s)
{
    hipError_t e;
    if (a.ncells > 0) {
        const int blocks = (a.ncells + 63) / 64;
        VPP_AMR_SWITCH(amr_apply_kernel, phi, x)
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(amr_node_sum_kernel, dim3(stream_blocks(a.n)), dim3(256), 0, s, a, x, y);
    return hipGetLastError();
}

hipError_t launch_amr_diag(int k, const AmrArgs& a, const double* phi, double* diag, double* inv64, float* inv32,
                           hipStream_t s)
{
    hipError_t e;
    if (a.ncells > 0) {
        const int blocks = (a.ncells + 63) / 64;
        VPP_AMR_SWITCH(amr_diag_kernel, phi)
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(amr_fix_diag_kernel, dim3(stream_blocks(a.n)), dim3(256), 0, s, a, diag, inv64, inv32);
    return hipGetLastError();
}

#undef VPP_AMR_SWITCH

}  // namespace vpp
