// Closest-point projection onto the zero isosurface of the FE level set phi_h
// (appendix "Extension of solution quantities from a level-set isosurface
// using closest point projection", Eq. cpp), one thread per point.
//
// From y = x, every outer step takes `normal_steps` corrections along the
// normal, y <- y - d(y) n(y) with the signed distance d = eps log((1+phi)/(1-phi))
// of Eq. distance and n = grad phi_h / |grad phi_h|, then one tangential
// correction y <- y - sum_j ((y - x).t_j) t_j over the unit tangents
// t_0 = (v - (v.n) n)/|.| and t_1 = n x t_0 (v = e_x, or e_y when |n_x| > 0.9),
// until |y^(k+1) - y^(k)| < tol or max_iter outer steps.  y is clipped to the
// domain box after every correction, phi_h to +-(1 - 1e-12) inside the
// logarithm, and a step whose gradient vanishes leaves y unchanged.
//
// phi_h and its gradient at y come from the Q_k Lagrange basis on the GLL
// support points of the cell holding y (values and derivatives by the product
// formula at the point's reference coordinates; (k+1)^3 nodal loads).  Every
// cell index is clamped into the mesh (NaN-safe), so no load leaves phi.
#include "common.h"
#include "kernels.h"

namespace vpp {

namespace {

constexpr double kPhiClip = 1.0 - 1e-12;

// Lagrange values V[a] and derivatives D[a] (reference coordinate) at t.
template <int K>
__device__ __forceinline__ void lagrange_at(double t, double (&V)[K + 1], double (&D)[K + 1])
{
    constexpr int N = K + 1;
    const double* x = Tab<K>::t.gll;
#pragma unroll
    for (int a = 0; a < N; ++a) {
        double v = 1.0, d = 0.0;
#pragma unroll
        for (int b = 0; b < N; ++b)
            if (b != a) {
                const double q = 1.0 / (x[a] - x[b]);
                d = d * ((t - x[b]) * q) + v * q;   // product rule, one factor at a time
                v *= (t - x[b]) * q;
            }
        V[a] = v;
        D[a] = d;
    }
}

// Value and gradient at y of the nodal field f (phi or any Q_k field of the mesh).
template <int K>
__device__ __forceinline__ void eval_field(const CpArgs& a, const double* __restrict__ f, const double (&y)[3],
                                           double& val, double (&g)[3])
{
    constexpr int N = K + 1;
    double V[3][N], D[3][N];
    int c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double s = (y[d] - a.lo[d]) / a.h[d];
        if (!(s >= 0.0)) s = 0.0;                 // also catches NaN
        if (!(s <= (double)a.m.nc[d])) s = (double)a.m.nc[d];
        int cd = (int)s;
        if (cd > a.m.nc[d] - 1) cd = a.m.nc[d] - 1;
        c[d] = cd;
        lagrange_at<K>(s - cd, V[d], D[d]);
#pragma unroll
        for (int i = 0; i < N; ++i) D[d][i] /= a.h[d];
    }
    const int64_t nx = a.m.nn[0], nxy = (int64_t)a.m.nn[0] * a.m.nn[1];
    const double* p = f + node_index(a.m, (int64_t)K * c[0], (int64_t)K * c[1], (int64_t)K * c[2]);
    val = 0.0;
    g[0] = g[1] = g[2] = 0.0;
#pragma unroll
    for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
        for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
            for (int a0 = 0; a0 < N; ++a0) {
                const double fv = p[a0 + nx * a1 + nxy * a2];
                val += V[0][a0] * V[1][a1] * V[2][a2] * fv;
                g[0] += D[0][a0] * V[1][a1] * V[2][a2] * fv;
                g[1] += V[0][a0] * D[1][a1] * V[2][a2] * fv;
                g[2] += V[0][a0] * V[1][a1] * D[2][a2] * fv;
            }
}

__device__ __forceinline__ void clip_box(const CpArgs& a, double (&y)[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fmin(fmax(y[d], a.lo[d]), a.hi[d]);
}

template <int K>
__global__ void __launch_bounds__(256) closest_point_kernel(CpArgs a)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    double x[3];
    if (a.pts) {
#pragma unroll
        for (int d = 0; d < 3; ++d) x[d] = a.pts[3 * i + d];
    } else {
        // support point i of the mesh: in the band only if |phi_i| < phi_lim
        const int64_t ij[3] = {i % a.m.nn[0], (i / a.m.nn[0]) % a.m.nn[1], i / ((int64_t)a.m.nn[0] * a.m.nn[1])};
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            int cd = (int)(ij[d] / K);
            if (cd > a.m.nc[d] - 1) cd = a.m.nc[d] - 1;
            const int al = (int)(ij[d] - (int64_t)K * cd);
            double xi = 0.0;
#pragma unroll
            for (int q = 0; q <= K; ++q)
                if (q == al) xi = Tab<K>::t.gll[q];   // compile-time table entries only
            x[d] = a.lo[d] + (cd + xi) * a.h[d];
        }
        if (!(fabs(a.phi[i]) < a.phi_lim)) {
#pragma unroll
            for (int d = 0; d < 3; ++d) a.y[3 * i + d] = x[d];
            a.info[i] = -1;
            return;
        }
    }
    double y[3] = {x[0], x[1], x[2]};
    int info = 0;
    for (int it = 1; it <= a.max_iter; ++it) {
        const double prev[3] = {y[0], y[1], y[2]};
        double val, g[3];
        for (int s = 0; s < a.normal_steps; ++s) {
            eval_field<K>(a, a.phi, y, val, g);
            const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
            if (gn > 0.0) {
                const double pc = fmin(fmax(val, -kPhiClip), kPhiClip);
                const double dist = a.eps * log((1.0 + pc) / (1.0 - pc));
#pragma unroll
                for (int d = 0; d < 3; ++d) y[d] -= dist * (g[d] / gn);
                clip_box(a, y);
            }
        }
        eval_field<K>(a, a.phi, y, val, g);
        const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        if (gn > 0.0) {
            const double n[3] = {g[0] / gn, g[1] / gn, g[2] / gn};
            const bool use_y = fabs(n[0]) > 0.9;
            const double v[3] = {use_y ? 0.0 : 1.0, use_y ? 1.0 : 0.0, 0.0};
            const double vn = v[0] * n[0] + v[1] * n[1] + v[2] * n[2];
            double t0[3] = {v[0] - vn * n[0], v[1] - vn * n[1], v[2] - vn * n[2]};
            const double tl = sqrt(t0[0] * t0[0] + t0[1] * t0[1] + t0[2] * t0[2]);
#pragma unroll
            for (int d = 0; d < 3; ++d) t0[d] /= tl;
            const double t1[3] = {n[1] * t0[2] - n[2] * t0[1], n[2] * t0[0] - n[0] * t0[2],
                                  n[0] * t0[1] - n[1] * t0[0]};
            const double r[3] = {y[0] - x[0], y[1] - x[1], y[2] - x[2]};
            const double r0 = r[0] * t0[0] + r[1] * t0[1] + r[2] * t0[2];
            const double r1 = r[0] * t1[0] + r[1] * t1[1] + r[2] * t1[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) y[d] -= r0 * t0[d] + r1 * t1[d];
            clip_box(a, y);
        }
        const double dy[3] = {y[0] - prev[0], y[1] - prev[1], y[2] - prev[2]};
        if (sqrt(dy[0] * dy[0] + dy[1] * dy[1] + dy[2] * dy[2]) < a.tol) {
            info = it;
            break;
        }
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) a.y[3 * i + d] = y[d];
    a.info[i] = info;
}

// Extension from the closest points: out[g] = f_h(y_g) for a node in the band
// (info[g] >= 0), f[g] elsewhere.
template <int K>
__global__ void __launch_bounds__(256) extend_kernel(CpArgs a, const double* __restrict__ f,
                                                     double* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= a.n) return;
    if (a.info[i] < 0) {
        out[i] = f[i];
        return;
    }
    const double y[3] = {a.y[3 * i], a.y[3 * i + 1], a.y[3 * i + 2]};
    double val, g[3];
    eval_field<K>(a, f, y, val, g);
    out[i] = val;
}

}  // namespace

hipError_t launch_extend(int k, const CpArgs& a, const double* f, double* out, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t blocks = (a.n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    switch (k) {
    case 2: hipLaunchKernelGGL(extend_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, a, f, out); break;
    case 3: hipLaunchKernelGGL(extend_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, a, f, out); break;
    case 4: hipLaunchKernelGGL(extend_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, s, a, f, out); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_closest_points(int k, const CpArgs& a, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    const int64_t blocks = (a.n + 255) / 256;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
    switch (k) {
    case 2: hipLaunchKernelGGL(closest_point_kernel<2>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    case 3: hipLaunchKernelGGL(closest_point_kernel<3>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    case 4: hipLaunchKernelGGL(closest_point_kernel<4>, dim3((unsigned)blocks), dim3(256), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace vpp
