// Right-hand sides of the level-set filter systems (Eqs. normal_vector and
// normal_vector_regularized, curvature and curvature_regularized), and the
// operator, diagonal and right-hand side of one semi-implicit step of
// Eq. reinitialization (further below):
//   normal:    b_d = (n_bar_d, v) with n_bar = grad phi_h / |grad phi_h| at every
//              Gauss point (zero where the gradient vanishes), d = x, y, z;
//   curvature: b = (kappa_bar, v) with kappa_bar = -div n_h at every Gauss point,
//              n_h the (filtered) nodal normal components.
// One cell per thread: values at the Gauss points by the interpolation
// sweeps, derivatives by the collocation derivative along each direction,
// the weights W_q, the transposed interpolation sweeps, and a scatter-add into
// the nodes (all rows assembled, no constraint applied) without atomics: one
// launch per cell colour (cell_color), so every node sum has a fixed order.
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
            for (int a0 = 0; a0 < N; ++a0) b[base + a0 + nx * a1 + nxy * a2] += s[a0 + N * (a1 + N * a2)];
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
                                                        double* __restrict__ b2, CellColor cc)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = g.m;
    int cx, cy, cz;
    if (!color_cell(cc, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
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
                                                           const double* __restrict__ n2, double* __restrict__ b,
                                                           CellColor cc)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = g.m;
    int cx, cy, cz;
    if (!color_cell(cc, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
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

// ---------------------------------------------------------------------------
// Reinitialization step (Eq. reinitialization, semi-implicit Euler in pseudo-
// time with the compressive flux explicit):
//   (psi', v)/dtau + eps ((grad psi' . n)(grad v . n)) = (psi, v)/dtau + ((1 - psi^2)/2 n, grad v),
// boundary terms of the integrations by parts dropped, n the nodal normal
// interpolated at the Gauss points as it is.  One cell per thread, one launch
// per cell colour, scatter-add without atomics (the output is zeroed first).

// The nodal normal components at the Gauss points of a cell.
template <int K>
__device__ __forceinline__ void normal_at_gauss(const ReinitArgs& r, int cx, int cy, int cz,
                                                double (&nq)[3][(K + 1) * (K + 1) * (K + 1)])
{
    const double* f[3] = {r.n0, r.n1, r.n2};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        load_nodes<K>(r.g.m, f[d], cx, cy, cz, nq[d]);
        sweep3<K, MS, false, 0>(nq[d]);
        sweep3<K, MS, false, 1>(nq[d]);
        sweep3<K, MS, false, 2>(nq[d]);
    }
}

// One nodal normal component at the Gauss points of a cell.
template <int K, int D>
__device__ __forceinline__ void normal_comp_at_gauss(const ReinitArgs& r, int cx, int cy, int cz,
                                                     double (&nd)[(K + 1) * (K + 1) * (K + 1)])
{
    load_nodes<K>(r.g.m, D == 0 ? r.n0 : (D == 1 ? r.n1 : r.n2), cx, cy, cz, nd);
    sweep3<K, MS, false, 0>(nd);
    sweep3<K, MS, false, 1>(nd);
    sweep3<K, MS, false, 2>(nd);
}

template <int K, int D>
__device__ __forceinline__ void add_directional(const double (&u)[(K + 1) * (K + 1) * (K + 1)],
                                                const double (&n)[(K + 1) * (K + 1) * (K + 1)], double ih,
                                                double (&s)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
    double g[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) g[q] = u[q];
    sweep3<K, MDC, false, D>(g);
#pragma unroll
    for (int q = 0; q < N3; ++q) s[q] = fma(n[q] * ih, g[q], s[q]);
}

// out += Dc_D^T (w n ih) at the Gauss points.
template <int K, int D>
__device__ __forceinline__ void add_flux(const double (&w)[(K + 1) * (K + 1) * (K + 1)],
                                         const double (&n)[(K + 1) * (K + 1) * (K + 1)], double ih,
                                         double (&out)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
    double g[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) g[q] = w[q] * n[q] * ih;
    sweep3<K, MDC, true, D>(g);
#pragma unroll
    for (int q = 0; q < N3; ++q) out[q] += g[q];
}

template <int K>
__global__ void __launch_bounds__(64) reinit_apply_kernel(ReinitArgs r, const double* __restrict__ x,
                                                          double* __restrict__ y, CellColor cc)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = r.g.m;
    int cx, cy, cz;
    if (!color_cell(cc, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
    // One normal component is live at a time (interpolated again for the
    // flux pass): holding all three at the Gauss points left one wave per SIMD.
    double u[N3], s[N3], out[N3], nd[N3];
    load_nodes<K>(m, x, cx, cy, cz, u);
    sweep3<K, MS, false, 0>(u);
    sweep3<K, MS, false, 1>(u);
    sweep3<K, MS, false, 2>(u);
#pragma unroll
    for (int q = 0; q < N3; ++q) s[q] = 0.0;
    normal_comp_at_gauss<K, 0>(r, cx, cy, cz, nd);
    add_directional<K, 0>(u, nd, r.g.ih[0], s);
    normal_comp_at_gauss<K, 1>(r, cx, cy, cz, nd);
    add_directional<K, 1>(u, nd, r.g.ih[1], s);
    normal_comp_at_gauss<K, 2>(r, cx, cy, cz, nd);
    add_directional<K, 2>(u, nd, r.g.ih[2], s);
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        const double w = r.g.vol * wref<K>(q % N, (q / N) % N, q / (N * N));
        out[q] = r.idtau * w * u[q];
        s[q] *= r.eps * w;
    }
    normal_comp_at_gauss<K, 0>(r, cx, cy, cz, nd);
    add_flux<K, 0>(s, nd, r.g.ih[0], out);
    normal_comp_at_gauss<K, 1>(r, cx, cy, cz, nd);
    add_flux<K, 1>(s, nd, r.g.ih[1], out);
    normal_comp_at_gauss<K, 2>(r, cx, cy, cz, nd);
    add_flux<K, 2>(s, nd, r.g.ih[2], out);
    transpose_interp<K>(out);
    scatter_add<K>(m, cx, cy, cz, out, y);
}

// Transposed sweep along DIR with the product table T0(q,a) T1(q,a) of the
// basis values (S) or derivatives (D) at the Gauss points: 0 S S, 1 D D, 2 S D.
template <int K, int TAB, int DIR>
__device__ __forceinline__ void sweep_sq(double (&v)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N = K + 1;
    constexpr int st = DIR == 0 ? 1 : (DIR == 1 ? N : N * N);
    constexpr int s1 = DIR == 0 ? N : 1;
    constexpr int s2 = DIR == 2 ? N : N * N;
#pragma unroll
    for (int i2 = 0; i2 < N; ++i2)
#pragma unroll
        for (int i1 = 0; i1 < N; ++i1) {
            const int base = i1 * s1 + i2 * s2;
            double in[N], out[N];
#pragma unroll
            for (int q = 0; q < N; ++q) in[q] = v[base + q * st];
#pragma unroll
            for (int a = 0; a < N; ++a) {
                double acc = 0.0;
#pragma unroll
                for (int q = 0; q < N; ++q) {
                    const double Sv = Tab<K>::t.S[q][a], Dv = Tab<K>::t.D[q][a];
                    const double c = TAB == 0 ? Sv * Sv : (TAB == 1 ? Dv * Dv : Sv * Dv);
                    acc = fma(c, in[q], acc);
                }
                out[a] = acc;
            }
#pragma unroll
            for (int a = 0; a < N; ++a) v[base + a * st] = out[a];
        }
}

// sum_q c_q dN_a/dx_D dN_a/dx_E (values N_a where the direction is neither D nor E).
template <int K, int D, int E>
__device__ __forceinline__ void add_diag_pair(const double (&c)[(K + 1) * (K + 1) * (K + 1)],
                                              double (&out)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
    constexpr int T0 = (D == 0 && E == 0) ? 1 : ((D == 0 || E == 0) ? 2 : 0);
    constexpr int T1 = (D == 1 && E == 1) ? 1 : ((D == 1 || E == 1) ? 2 : 0);
    constexpr int T2 = (D == 2 && E == 2) ? 1 : ((D == 2 || E == 2) ? 2 : 0);
    double v[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) v[q] = c[q];
    sweep_sq<K, T2, 2>(v);
    sweep_sq<K, T1, 1>(v);
    sweep_sq<K, T0, 0>(v);
#pragma unroll
    for (int q = 0; q < N3; ++q) out[q] += v[q];
}

template <int K, int D, int E>
__device__ __forceinline__ void diag_pair(const ReinitArgs& r, const double (&nq)[3][(K + 1) * (K + 1) * (K + 1)],
                                          double (&out)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N = K + 1, N3 = N * N * N;
    double c[N3];
    const double f = r.eps * r.g.ih[D] * r.g.ih[E] * (D == E ? 1.0 : 2.0);
#pragma unroll
    for (int q = 0; q < N3; ++q)
        c[q] = f * r.g.vol * wref<K>(q % N, (q / N) % N, q / (N * N)) * nq[D][q] * nq[E][q];
    add_diag_pair<K, D, E>(c, out);
}

template <int K>
__global__ void __launch_bounds__(64) reinit_diag_kernel(ReinitArgs r, double* __restrict__ diag, CellColor cc)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = r.g.m;
    int cx, cy, cz;
    if (!color_cell(cc, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
    double nq[3][N3], out[N3], c[N3];
    normal_at_gauss<K>(r, cx, cy, cz, nq);
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        out[q] = 0.0;
        c[q] = r.idtau * r.g.vol * wref<K>(q % N, (q / N) % N, q / (N * N));
    }
    add_diag_pair<K, 3, 3>(c, out);   // no derivative direction: the mass term
    diag_pair<K, 0, 0>(r, nq, out);
    diag_pair<K, 1, 1>(r, nq, out);
    diag_pair<K, 2, 2>(r, nq, out);
    diag_pair<K, 0, 1>(r, nq, out);
    diag_pair<K, 0, 2>(r, nq, out);
    diag_pair<K, 1, 2>(r, nq, out);
    scatter_add<K>(m, cx, cy, cz, out, diag);
}

template <int K>
__global__ void __launch_bounds__(64) reinit_rhs_kernel(ReinitArgs r, const double* __restrict__ psi,
                                                        double* __restrict__ b, CellColor cc)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = r.g.m;
    int cx, cy, cz;
    if (!color_cell(cc, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
    double nq[3][N3], u[N3], w[N3], out[N3];
    normal_at_gauss<K>(r, cx, cy, cz, nq);
    load_nodes<K>(m, psi, cx, cy, cz, u);
    sweep3<K, MS, false, 0>(u);
    sweep3<K, MS, false, 1>(u);
    sweep3<K, MS, false, 2>(u);
#pragma unroll
    for (int q = 0; q < N3; ++q) {
        const double wq = r.g.vol * wref<K>(q % N, (q / N) % N, q / (N * N));
        out[q] = r.idtau * wq * u[q];
        w[q] = wq * 0.5 * (1.0 - u[q] * u[q]);
    }
    add_flux<K, 0>(w, nq[0], r.g.ih[0], out);
    add_flux<K, 1>(w, nq[1], r.g.ih[1], out);
    add_flux<K, 2>(w, nq[2], r.g.ih[2], out);
    transpose_interp<K>(out);
    scatter_add<K>(m, cx, cy, cz, out, b);
}

// Per-workgroup partials of x . y (fixed order inside the workgroup).
__global__ void __launch_bounds__(256) dot_partials_kernel(const double* __restrict__ x, const double* __restrict__ y,
                                                           int64_t n, double* __restrict__ part)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
        s = fma(x[i], y[i], s);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

}  // namespace

// One launch of KERNEL<k> per cell colour (the scatter-adds need no atomics).
#define VPP_COLORED(KERNEL, ...)                                                                               \
    switch (k) {                                                                                                \
    case 2:                                                                                                     \
        return for_each_color(m, 64, [&](const CellColor& cc, int blocks) {                                    \
            hipLaunchKernelGGL(KERNEL<2>, dim3(blocks), dim3(64), 0, s, __VA_ARGS__, cc);                     \
        });                                                                                                     \
    case 3:                                                                                                     \
        return for_each_color(m, 64, [&](const CellColor& cc, int blocks) {                                    \
            hipLaunchKernelGGL(KERNEL<3>, dim3(blocks), dim3(64), 0, s, __VA_ARGS__, cc);                     \
        });                                                                                                     \
    case 4:                                                                                                     \
        return for_each_color(m, 64, [&](const CellColor& cc, int blocks) {                                    \
            hipLaunchKernelGGL(KERNEL<4>, dim3(blocks), dim3(64), 0, s, __VA_ARGS__, cc);                     \
        });                                                                                                     \
    default: return hipErrorInvalidValue;                                                                       \
    }

hipError_t launch_normal_rhs(int k, const RhsGeo& g, const double* phi, double* b0, double* b1, double* b2,
                             hipStream_t s)
{
    const MeshArgs& m = g.m;
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    hipError_t e;
    if ((e = launch_fill<double>(b0, n, 0.0, s)) != hipSuccess || (e = launch_fill<double>(b1, n, 0.0, s)) != hipSuccess ||
        (e = launch_fill<double>(b2, n, 0.0, s)) != hipSuccess)
        return e;
    VPP_COLORED(normal_rhs_kernel, g, phi, b0, b1, b2)
}

hipError_t launch_curvature_rhs(int k, const RhsGeo& g, const double* n0, const double* n1, const double* n2,
                                double* b, hipStream_t s)
{
    const MeshArgs& m = g.m;
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    hipError_t e = launch_fill<double>(b, n, 0.0, s);
    if (e != hipSuccess) return e;
    VPP_COLORED(curvature_rhs_kernel, g, n0, n1, n2, b)
}

hipError_t launch_reinit_apply(int k, const ReinitArgs& r, const double* x, double* y, hipStream_t s)
{
    const MeshArgs& m = r.g.m;
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    hipError_t e = launch_fill<double>(y, n, 0.0, s);
    if (e != hipSuccess) return e;
    VPP_COLORED(reinit_apply_kernel, r, x, y)
}

hipError_t launch_reinit_diag(int k, const ReinitArgs& r, double* diag, hipStream_t s)
{
    const MeshArgs& m = r.g.m;
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    hipError_t e = launch_fill<double>(diag, n, 0.0, s);
    if (e != hipSuccess) return e;
    VPP_COLORED(reinit_diag_kernel, r, diag)
}

hipError_t launch_reinit_rhs(int k, const ReinitArgs& r, const double* psi, double* b, hipStream_t s)
{
    const MeshArgs& m = r.g.m;
    const int64_t n = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    hipError_t e = launch_fill<double>(b, n, 0.0, s);
    if (e != hipSuccess) return e;
    VPP_COLORED(reinit_rhs_kernel, r, psi, b)
}
#undef VPP_COLORED

hipError_t launch_dot_partials(const double* x, const double* y, int64_t n, double* part, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(dot_partials_kernel, dim3(nblocks), dim3(256), 0, s, x, y, n, part);
    return hipGetLastError();
}

}  // namespace vpp
