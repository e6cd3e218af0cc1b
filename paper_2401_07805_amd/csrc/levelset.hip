// Right-hand sides of the level-set filter systems (Eqs. normal_vector and
// normal_vector_regularized, curvature and curvature_regularized):
//   normal:    b_d = (n_bar_d, v) with n_bar = grad phi_h / |grad phi_h| at every
//              Gauss point (zero where the gradient vanishes), d = x, y, z;
//   curvature: b = (kappa_bar, v) with kappa_bar = -div n_h at every Gauss point,
//              n_h the (filtered) nodal normal components.
// One cell per thread: values at the Gauss points by the interpolation
// sweeps, derivatives by the collocation derivative along each direction,
// the weights W_q, the transposed interpolation sweeps, and an atomic
// scatter-add into the nodes (all rows assembled, no constraint applied).
#include "kernels.h"

namespace vpp {

namespace {

template <int K>
__device__ __forceinline__ void load_nodes(const MeshArgs& m, const double* __restrict__ v, int cx, int cy, int cz,
                                           double (&u)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N = K + 1;
    const int64_t nx = m.nn[0], nxy = (int64_t)m.nn[0] * m.nn[1];
    const int64_t base = node_index(m, (int64_t)K * cx, (int64_t)K * cy, (int64_t)K * cz);
#pragma unroll
    for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
        for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) u[a0 + N * (a1 + N * a2)] = v[base + a0 + nx * a1 + nxy * a2];
}

template <int K>
__device__ __forceinline__ void scatter_add(const MeshArgs& m, int cx, int cy, int cz,
                                            const double (&s)[(K + 1) * (K + 1) * (K + 1)], double* __restrict__ b)
{
    constexpr int N = K + 1;
    const int64_t nx = m.nn[0], nxy = (int64_t)m.nn[0] * m.nn[1];
    const int64_t base = node_index(m, (int64_t)K * cx, (int64_t)K * cy, (int64_t)K * cz);
#pragma unroll
    for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
        for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) atomicAdd(&b[base + a0 + nx * a1 + nxy * a2], s[a0 + N * (a1 + N * a2)]);
}

template <int K>
__device__ __forceinline__ void transpose_interp(double (&s)[(K + 1) * (K + 1) * (K + 1)])
{
    sweep3<K, MS, true, 2>(s);
    sweep3<K, MS, true, 1>(s);
    sweep3<K, MS, true, 0>(s);
}

template <int K>
__global__ void __launch_bounds__(64) normal_rhs_kernel(RhsGeo g, const double* __restrict__ phi,
                                                        double* __restrict__ b0, double* __restrict__ b1,
                                                        double* __restrict__ b2)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = g.m;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    if (cell >= ncell) return;
    const int cx = (int)(cell % m.nc[0]), cy = (int)((cell / m.nc[0]) % m.nc[1]),
              cz = (int)(cell / ((int64_t)m.nc[0] * m.nc[1]));
    double gx[N3], gy[N3], gz[N3];
    load_nodes<K>(m, phi, cx, cy, cz, gx);
    sweep3<K, MS, false, 0>(gx);
    sweep3<K, MS, false, 1>(gx);
    sweep3<K, MS, false, 2>(gx);
#pragma unroll
    for (int q = 0; q < N3; ++q) gy[q] = gz[q] = gx[q];
    sweep3<K, MDC, false, 0>(gx);
    sweep3<K, MDC, false, 1>(gy);
    sweep3<K, MDC, false, 2>(gz);
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        const double a = gx[q] * g.ih[0], b = gy[q] * g.ih[1], c = gz[q] * g.ih[2];
        const double nrm = sqrt(a * a + b * b + c * c);
        const double w = nrm > 0.0 ? g.vol * wref<K>(q % N, (q / N) % N, q / (N * N)) / nrm : 0.0;
        gx[q] = w * a;
        gy[q] = w * b;
        gz[q] = w * c;
    }
    transpose_interp<K>(gx);
    scatter_add<K>(m, cx, cy, cz, gx, b0);
    transpose_interp<K>(gy);
    scatter_add<K>(m, cx, cy, cz, gy, b1);
    transpose_interp<K>(gz);
    scatter_add<K>(m, cx, cy, cz, gz, b2);
}

template <int K, int D>
__device__ __forceinline__ void add_derivative(const MeshArgs& m, const double* __restrict__ f, double ih, int cx,
                                               int cy, int cz, double (&div)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N = K + 1, N3 = N * N * N;
    double u[N3];
    load_nodes<K>(m, f, cx, cy, cz, u);
    sweep3<K, MS, false, 0>(u);
    sweep3<K, MS, false, 1>(u);
    sweep3<K, MS, false, 2>(u);
    sweep3<K, MDC, false, D>(u);
#pragma unroll
    for (int q = 0; q < N3; ++q) div[q] = fma(ih, u[q], div[q]);
}

template <int K>
__global__ void __launch_bounds__(64) curvature_rhs_kernel(RhsGeo g, const double* __restrict__ n0,
                                                           const double* __restrict__ n1,
                                                           const double* __restrict__ n2, double* __restrict__ b)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = g.m;
    const int64_t cell = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    if (cell >= ncell) return;
    const int cx = (int)(cell % m.nc[0]), cy = (int)((cell / m.nc[0]) % m.nc[1]),
              cz = (int)(cell / ((int64_t)m.nc[0] * m.nc[1]));
    double div[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) div[q] = 0.0;
    add_derivative<K, 0>(m, n0, g.ih[0], cx, cy, cz, div);
    add_derivative<K, 1>(m, n1, g.ih[1], cx, cy, cz, div);
    add_derivative<K, 2>(m, n2, g.ih[2], cx, cy, cz, div);
#pragma unroll
    for (int q = 0; q < N3; ++q) div[q] *= -g.vol * wref<K>(q % N, (q / N) % N, q / (N * N));
    transpose_interp<K>(div);
    scatter_add<K>(m, cx, cy, cz, div, b);
}

}  // namespace

hipError_t launch_normal_rhs(int k, const RhsGeo& g, const double* phi, double* b0, double* b1, double* b2,
                             hipStream_t s)
{
    const int64_t n = (int64_t)g.m.nn[0] * g.m.nn[1] * g.m.nn[2];
    hipError_t e;
    if ((e = launch_fill<double>(b0, n, 0.0, s)) != hipSuccess || (e = launch_fill<double>(b1, n, 0.0, s)) != hipSuccess ||
        (e = launch_fill<double>(b2, n, 0.0, s)) != hipSuccess)
        return e;
    const int64_t ncell = (int64_t)g.m.nc[0] * g.m.nc[1] * g.m.nc[2];
    const int blocks = (int)((ncell + 63) / 64);
    switch (k) {
    case 2: hipLaunchKernelGGL(normal_rhs_kernel<2>, dim3(blocks), dim3(64), 0, s, g, phi, b0, b1, b2); break;
    case 3: hipLaunchKernelGGL(normal_rhs_kernel<3>, dim3(blocks), dim3(64), 0, s, g, phi, b0, b1, b2); break;
    case 4: hipLaunchKernelGGL(normal_rhs_kernel<4>, dim3(blocks), dim3(64), 0, s, g, phi, b0, b1, b2); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_curvature_rhs(int k, const RhsGeo& g, const double* n0, const double* n1, const double* n2,
                                double* b, hipStream_t s)
{
    const int64_t n = (int64_t)g.m.nn[0] * g.m.nn[1] * g.m.nn[2];
    hipError_t e = launch_fill<double>(b, n, 0.0, s);
    if (e != hipSuccess) return e;
    const int64_t ncell = (int64_t)g.m.nc[0] * g.m.nc[1] * g.m.nc[2];
    const int blocks = (int)((ncell + 63) / 64);
    switch (k) {
    case 2: hipLaunchKernelGGL(curvature_rhs_kernel<2>, dim3(blocks), dim3(64), 0, s, g, n0, n1, n2, b); break;
    case 3: hipLaunchKernelGGL(curvature_rhs_kernel<3>, dim3(blocks), dim3(64), 0, s, g, n0, n1, n2, b); break;
    case 4: hipLaunchKernelGGL(curvature_rhs_kernel<4>, dim3(blocks), dim3(64), 0, s, g, n0, n1, n2, b); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vpp
