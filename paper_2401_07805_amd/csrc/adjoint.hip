// Adjoint of the operator with respect to its coefficient and to nodal phi.
//
// With A_D(c) p = b (b independent of phi) and J(p), the adjoint lam solves
// A_D lam = dJ/dp (A_D is symmetric), and for every Gauss point
//   dJ/dc_q = -lam^T (dA_D/dc_q) p = -W_q grad(lam_h) . grad(p_h),
// where dA_D/dc_q only touches free rows and columns, so Dirichlet entries of p
// and lam are taken as zero.  The chain rule through Eq. rhoEff, the Heaviside
// and the clamp of the interpolated level set gives
//   dJ/dphi_j = sum_q dJ/dc_q (1/rho_l - 1/rho_g) H'(phi_h(x_q)) [|phi_h(x_q)| < 1] N_j(x_q).
// Both are evaluated by sum factorisation on one cell per thread.
#include "kernels.h"

namespace vpp {

template <int K>
__device__ __forceinline__ void load_cell(const MeshArgs& m, const double* __restrict__ v, int cx, int cy, int cz,
                                          bool mask, double (&u)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N = K + 1;
    const int64_t nx = m.nn[0], nxy = (int64_t)m.nn[0] * m.nn[1];
    const int64_t base = node_index(m, (int64_t)K * cx, (int64_t)K * cy, (int64_t)K * cz);
#pragma unroll
    for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
        for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) {
                double x = v[base + a0 + nx * a1 + nxy * a2];
                if (mask && is_dirichlet(m, K * cx + a0, K * cy + a1, K * cz + a2)) x = 0.0;
                u[a0 + N * (a1 + N * a2)] = x;
            }
}

template <int K>
__global__ void __launch_bounds__(64) grad_coef_kernel(MeshArgs m, const double* __restrict__ p,
                                                       const double* __restrict__ lam, double* __restrict__ g)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    if (cell >= ncell) return;
    const int cx = (int)(cell % m.nc[0]), cy = (int)((cell / m.nc[0]) % m.nc[1]),
              cz = (int)(cell / ((int64_t)m.nc[0] * m.nc[1]));
    double pq[N3], lq[N3], acc[N3];
    load_cell<K>(m, p, cx, cy, cz, true, pq);
    load_cell<K>(m, lam, cx, cy, cz, true, lq);
    sweep3<K, MS, false, 0>(pq);
    sweep3<K, MS, false, 1>(pq);
    sweep3<K, MS, false, 2>(pq);
    sweep3<K, MS, false, 0>(lq);
    sweep3<K, MS, false, 1>(lq);
    sweep3<K, MS, false, 2>(lq);
#pragma unroll
    for (int q = 0; q < N3; ++q) acc[q] = 0.0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int st = d == 0 ? 1 : (d == 1 ? N : N * N);
        const int s1 = d == 0 ? N : 1;
        const int s2 = d == 2 ? N : N * N;
#pragma unroll
        for (int i2 = 0; i2 < N; ++i2)
#pragma unroll
            for (int i1 = 0; i1 < N; ++i1) {
                const int base = i1 * s1 + i2 * s2;
                double a[N], b[N], ga[N], gb[N];
#pragma unroll
                for (int t = 0; t < N; ++t) {
                    a[t] = pq[base + t * st];
                    b[t] = lq[base + t * st];
                }
                line<K, MDC, false>(a, ga);
                line<K, MDC, false>(b, gb);
#pragma unroll
                for (int t = 0; t < N; ++t) acc[base + t * st] = fma(m.rd[d] * ga[t], gb[t], acc[base + t * st]);
            }
    }
#pragma unroll
    for (int q = 0; q < N3; ++q)
        g[cell * N3 + q] = -m.r0 * wref<K>(q % N, (q / N) % N, q / (N * N)) * acc[q];
}

template <int K>
__global__ void __launch_bounds__(64) grad_phi_kernel(MeshArgs m, const double* __restrict__ phi,
                                                      const double* __restrict__ g, double* __restrict__ cv)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int cx, cy, cz;
    if (!cell_of(m, cell, cx, cy, cz)) return;
    double s[N3];
    load_cell<K>(m, phi, cx, cy, cz, false, s);
    sweep3<K, MS, false, 0>(s);
    sweep3<K, MS, false, 1>(s);
    sweep3<K, MS, false, 2>(s);
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        const double ph = s[q];
        const double dH = (m.heaviside == 0) ? 0.5 : sine_ramp_deriv(ph);
        s[q] = (fabs(ph) < 1.0) ? g[cell * N3 + q] * m.dcdphi * dH : 0.0;
    }
    sweep3<K, MS, true, 2>(s);
    sweep3<K, MS, true, 1>(s);
    sweep3<K, MS, true, 0>(s);
    // the cell's values, cell-major (the node sum adds them into the nodes)
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
#pragma unroll
    for (int q = 0; q < N3; ++q) cv[q * ncell + cell] = s[q];
}

hipError_t launch_grad_coef(int k, const MeshArgs& m, const double* p, const double* lam, double* g, hipStream_t s)
{
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    const int blocks = (int)((ncell + 63) / 64);
    switch (k) {
    case 2: hipLaunchKernelGGL(grad_coef_kernel<2>, dim3(blocks), dim3(64), 0, s, m, p, lam, g); break;
    case 3: hipLaunchKernelGGL(grad_coef_kernel<3>, dim3(blocks), dim3(64), 0, s, m, p, lam, g); break;
    case 4: hipLaunchKernelGGL(grad_coef_kernel<4>, dim3(blocks), dim3(64), 0, s, m, p, lam, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_grad_phi(int k, const MeshArgs& m, const double* phi, const double* g, double* out, double* cv,
                           hipStream_t s)
{
    // the cells' contributions into a cell-major buffer, then the node sum
    // (fixed order per node, no atomics)
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    const int blocks = (int)((ncell + 63) / 64);
    switch (k) {
    case 2: hipLaunchKernelGGL(grad_phi_kernel<2>, dim3(blocks), dim3(64), 0, s, m, phi, g, cv); break;
    case 3: hipLaunchKernelGGL(grad_phi_kernel<3>, dim3(blocks), dim3(64), 0, s, m, phi, g, cv); break;
    case 4: hipLaunchKernelGGL(grad_phi_kernel<4>, dim3(blocks), dim3(64), 0, s, m, phi, g, cv); break;
    default: return hipErrorInvalidValue;
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_node_sum(k, m, cv, out, s);
}

}  // namespace vpp
