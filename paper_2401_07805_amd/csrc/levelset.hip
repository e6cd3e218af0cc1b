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
// the weights W_q and the transposed interpolation sweeps, stored per cell in
// a cell-major buffer; a second launch adds them into the nodes (all rows
// assembled, no constraint applied), each node summing its cells in a fixed
// order, so no atomics are needed and every run gives the same bits.
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

// The (k+1)^3 local results of cell (cx, cy, cz) into the cell-major buffer
// cv (position q of cell c at cv[q * ncell + c]: a wave's stores are
// consecutive); launch_node_sum then adds them into the nodes.
template <int K>
__device__ __forceinline__ void store_cell(const MeshArgs& m, int cx, int cy, int cz,
                                           const double (&s)[(K + 1) * (K + 1) * (K + 1)], double* __restrict__ cv)
{
    constexpr int N3 = (K + 1) * (K + 1) * (K + 1);
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    const int64_t c = cx + (int64_t)m.nc[0] * (cy + (int64_t)m.nc[1] * cz);
#pragma unroll
    for (int q = 0; q < N3; ++q) cv[q * ncell + c] = s[q];
}

template <int K>
__device__ __forceinline__ void transpose_interp(double (&s)[(K + 1) * (K + 1) * (K + 1)])
{
    sweep3<K, MS, true, 2>(s);
    sweep3<K, MS, true, 1>(s);
    sweep3<K, MS, true, 0>(s);
}

// out[g] = sum of the cell-major values cv[q * ncell + c] of the cells c holding
// node g (q: the node's position in c), cells taken in increasing index.
template <int K>
__global__ void __launch_bounds__(256) node_sum_kernel(MeshArgs m, const double* __restrict__ cv,
                                                       double* __restrict__ out)
{
    constexpr int N = K + 1;
    const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];
    const int64_t nn = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    for (int64_t g = (int64_t)blockIdx.x * 256 + threadIdx.x; g < nn; g += (int64_t)gridDim.x * 256) {
        const int64_t r = g / m.nn[0];
        const int idx[3] = {(int)(g - r * m.nn[0]), (int)(r % m.nn[1]), (int)(r / m.nn[1])};
        int cell[3][2], loc[3][2], cnt[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int q = idx[d] / K, rem = idx[d] - q * K;
            if (rem != 0) {
                cell[d][0] = q;
                loc[d][0] = rem;
                cnt[d] = 1;
            } else {
                int c = 0;
                if (q > 0) {
                    cell[d][c] = q - 1;
                    loc[d][c] = K;
                    ++c;
                }
                if (q < m.nc[d]) {
                    cell[d][c] = q;
                    loc[d][c] = 0;
                    ++c;
                }
                cnt[d] = c;
            }
        }
        // every contribution loaded before any is added; added in increasing
        // cell order (b2, b1, b0 nested) as before
        double t[8];
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
            for (int b1 = 0; b1 < 2; ++b1)
#pragma unroll
                for (int b0 = 0; b0 < 2; ++b0)
                    if (b0 < cnt[0] && b1 < cnt[1] && b2 < cnt[2]) {
                        const int64_t c =
                            cell[0][b0] + (int64_t)m.nc[0] * (cell[1][b1] + (int64_t)m.nc[1] * cell[2][b2]);
                        const int q = loc[0][b0] + N * (loc[1][b1] + N * loc[2][b2]);
                        t[b0 + 2 * (b1 + 2 * b2)] = cv[q * ncell + c];
                    }
        double v = 0.0;
#pragma unroll
        for (int b2 = 0; b2 < 2; ++b2)
#pragma unroll
            for (int b1 = 0; b1 < 2; ++b1)
#pragma unroll
                for (int b0 = 0; b0 < 2; ++b0)
                    if (b0 < cnt[0] && b1 < cnt[1] && b2 < cnt[2]) v += t[b0 + 2 * (b1 + 2 * b2)];
        out[g] = v;
    }
}

template <int K>
__global__ void __launch_bounds__(64) normal_rhs_kernel(RhsGeo g, const double* __restrict__ phi,
                                                        double* __restrict__ cv0, double* __restrict__ cv1,
                                                        double* __restrict__ cv2)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = g.m;
    int cx, cy, cz;
    if (!cell_of(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
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
    store_cell<K>(m, cx, cy, cz, gx, cv0);
    transpose_interp<K>(gy);
    store_cell<K>(m, cx, cy, cz, gy, cv1);
    transpose_interp<K>(gz);
    store_cell<K>(m, cx, cy, cz, gz, cv2);
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
                                                           const double* __restrict__ n2, double* __restrict__ cv)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = g.m;
    int cx, cy, cz;
    if (!cell_of(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
    double div[N3];
#pragma unroll
    for (int q = 0; q < N3; ++q) div[q] = 0.0;
    add_derivative<K, 0>(m, n0, g.ih[0], cx, cy, cz, div);
    add_derivative<K, 1>(m, n1, g.ih[1], cx, cy, cz, div);
    add_derivative<K, 2>(m, n2, g.ih[2], cx, cy, cz, div);
#pragma unroll
    for (int q = 0; q < N3; ++q) div[q] *= -g.vol * wref<K>(q % N, (q / N) % N, q / (N * N));
    transpose_interp<K>(div);
    store_cell<K>(m, cx, cy, cz, div, cv);
}

// ---------------------------------------------------------------------------
// Reinitialization step (Eq. reinitialization, semi-implicit Euler in pseudo-
// time with the compressive flux explicit):
//   (psi', v)/dtau + eps ((grad psi' . n)(grad v . n)) = (psi, v)/dtau + ((1 - psi^2)/2 n, grad v),
// boundary terms of the integrations by parts dropped, n the nodal normal
// interpolated at the Gauss points as it is.  One cell per thread into the
// cell-major buffer, then the node sum (launch_node_sum).

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
                                                          double* __restrict__ cv)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = r.g.m;
    int cx, cy, cz;
    if (!cell_of(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
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
    store_cell<K>(m, cx, cy, cz, out, cv);
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
__global__ void __launch_bounds__(64) reinit_diag_kernel(ReinitArgs r, double* __restrict__ cv)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = r.g.m;
    int cx, cy, cz;
    if (!cell_of(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
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
    store_cell<K>(m, cx, cy, cz, out, cv);
}

template <int K>
__global__ void __launch_bounds__(64) reinit_rhs_kernel(ReinitArgs r, const double* __restrict__ psi,
                                                        double* __restrict__ cv)
{
    constexpr int N = K + 1, N3 = N * N * N;
    const MeshArgs& m = r.g.m;
    int cx, cy, cz;
    if (!cell_of(m, (int64_t)blockIdx.x * blockDim.x + threadIdx.x, cx, cy, cz)) return;
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
    store_cell<K>(m, cx, cy, cz, out, cv);
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

// The cell kernel KERNEL<k> over all cells (64-thread workgroups), writing the
// cell-major buffer(s) that the node sums then read.
#define VPP_CELLS(KERNEL, ...)                                                                                  \
    {                                                                                                           \
        const int64_t ncell = (int64_t)m.nc[0] * m.nc[1] * m.nc[2];                                             \
        const int blocks = (int)((ncell + 63) / 64);                                                            \
        switch (k) {                                                                                            \
        case 2: hipLaunchKernelGGL(KERNEL<2>, dim3(blocks), dim3(64), 0, s, __VA_ARGS__); break;              \
        case 3: hipLaunchKernelGGL(KERNEL<3>, dim3(blocks), dim3(64), 0, s, __VA_ARGS__); break;              \
        case 4: hipLaunchKernelGGL(KERNEL<4>, dim3(blocks), dim3(64), 0, s, __VA_ARGS__); break;              \
        default: return hipErrorInvalidValue;                                                                   \
        }                                                                                                       \
        const hipError_t e = hipGetLastError();                                                                 \
        if (e != hipSuccess) return e;                                                                          \
    }

hipError_t launch_node_sum(int k, const MeshArgs& m, const double* cv, double* out, hipStream_t s)
{
    const int64_t nn = (int64_t)m.nn[0] * m.nn[1] * m.nn[2];
    const int64_t want = (nn + 255) / 256;
    const int blocks = (int)(want < 16384 ? want : 16384);
    switch (k) {
    case 2: hipLaunchKernelGGL(node_sum_kernel<2>, dim3(blocks), dim3(256), 0, s, m, cv, out); break;
    case 3: hipLaunchKernelGGL(node_sum_kernel<3>, dim3(blocks), dim3(256), 0, s, m, cv, out); break;
    case 4: hipLaunchKernelGGL(node_sum_kernel<4>, dim3(blocks), dim3(256), 0, s, m, cv, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int64_t cell_values(int k, const MeshArgs& m)
{
    return (int64_t)(k + 1) * (k + 1) * (k + 1) * m.nc[0] * m.nc[1] * m.nc[2];
}

hipError_t launch_normal_rhs(int k, const RhsGeo& g, const double* phi, double* b0, double* b1, double* b2,
                             double* cv, hipStream_t s)
{
    const MeshArgs& m = g.m;
    const int64_t nv = cell_values(k, m);
    VPP_CELLS(normal_rhs_kernel, g, phi, cv, cv + nv, cv + 2 * nv)
    hipError_t e;
    if ((e = launch_node_sum(k, m, cv, b0, s)) != hipSuccess || (e = launch_node_sum(k, m, cv + nv, b1, s)) != hipSuccess)
        return e;
    return launch_node_sum(k, m, cv + 2 * nv, b2, s);
}

hipError_t launch_curvature_rhs(int k, const RhsGeo& g, const double* n0, const double* n1, const double* n2,
                                double* b, double* cv, hipStream_t s)
{
    const MeshArgs& m = g.m;
    VPP_CELLS(curvature_rhs_kernel, g, n0, n1, n2, cv)
    return launch_node_sum(k, m, cv, b, s);
}

hipError_t launch_reinit_apply(int k, const ReinitArgs& r, const double* x, double* y, double* cv, hipStream_t s)
{
    const MeshArgs& m = r.g.m;
    VPP_CELLS(reinit_apply_kernel, r, x, cv)
    return launch_node_sum(k, m, cv, y, s);
}

hipError_t launch_reinit_diag(int k, const ReinitArgs& r, double* diag, double* cv, hipStream_t s)
{
    const MeshArgs& m = r.g.m;
    VPP_CELLS(reinit_diag_kernel, r, cv)
    return launch_node_sum(k, m, cv, diag, s);
}

hipError_t launch_reinit_rhs(int k, const ReinitArgs& r, const double* psi, double* b, double* cv, hipStream_t s)
{
    const MeshArgs& m = r.g.m;
    VPP_CELLS(reinit_rhs_kernel, r, psi, cv)
    return launch_node_sum(k, m, cv, b, s);
}
#undef VPP_CELLS

hipError_t launch_dot_partials(const double* x, const double* y, int64_t n, double* part, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(dot_partials_kernel, dim3(nblocks), dim3(256), 0, s, x, y, n, part);
    return hipGetLastError();
}

}  // namespace vpp
