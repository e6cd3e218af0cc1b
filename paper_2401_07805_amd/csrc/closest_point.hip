// Closest-point projection onto the zero isosurface of the FE level set phi_h
// (appendix "Extension of solution quantities from a level-set isosurface
// using closest point projection", Eq. cpp), one lane per point at a time:
// a persistent grid works through a queue of points (the compacted narrow
// band of the mesh nodes, or the caller's points), and the extension of nodal
// fields from the closest points.
//
// From y = x, every outer step takes `normal_steps` corrections along the
// normal, y <- y - d(y) n(y) with the signed distance d = eps log((1+phi)/(1-phi))
// of Eq. distance and n = grad phi_h / |grad phi_h|, then one tangential
// correction y <- y - sum_j ((y - x).t_j) t_j over the unit tangents
// t_0 = (v - (v.n) n)/|.| and t_1 = n x t_0 (v = e_x, or e_y when |n_x| > 0.9),
// until |y^(k+1) - y^(k)| < tol or max_iter outer steps.  y is clipped to the
// domain box after every correction, phi_h to +-(1 - 1e-12) inside the
// logarithm, and a step whose normal vanishes leaves y unchanged.  With a
// nodal normal field given (the filtered interface normal of Eq.
// normal_vector_regularized, which is the n of Eq. cpp), n = n_h(y)/|n_h(y)|
// replaces the normalised gradient: n_h is continuous across cell faces,
// where the gradient of phi_h jumps.
//
// phi_h, its gradient and n_h at y come from the Q_k Lagrange basis on the GLL
// support points of the cell holding y (values and derivatives by the product
// formula at the point's reference coordinates; (k+1)^3 nodal loads per
// field).  Every cell index is clamped into the mesh (NaN-safe), so no load
// leaves the nodal arrays.
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

// Cell of y (clamped into the mesh), Lagrange values V and physical
// derivatives D at y's reference coordinates; returns the cell's first node.
template <int K>
__device__ __forceinline__ int64_t locate(const CpArgs& a, const double (&y)[3], double (&V)[3][K + 1],
                                          double (&D)[3][K + 1])
{
    constexpr int N = K + 1;
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
        const double ih = 1.0 / a.h[d];
#pragma unroll
        for (int i = 0; i < N; ++i) D[d][i] *= ih;
    }
    return node_index(a.m, (int64_t)K * c[0], (int64_t)K * c[1], (int64_t)K * c[2]);
}

// Value and gradient at y of the nodal field f (phi or any Q_k field of the mesh).
template <int K>
__device__ __forceinline__ void eval_field(const CpArgs& a, const double* __restrict__ f, const double (&y)[3],
                                           double& val, double (&g)[3])
{
    constexpr int N = K + 1;
    double V[3][N], D[3][N];
    const int64_t nx = a.m.nn[0], nxy = (int64_t)a.m.nn[0] * a.m.nn[1];
    const double* p = f + locate<K>(a, y, V, D);
    // (loads left where they are used: this evaluation's time is its
    // dependent arithmetic, and gathering first only raised its registers)
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

// Values at y of phi_h and of the nodal normal field's three components.
template <int K>
__device__ __forceinline__ void eval_phi_normal(const CpArgs& a, const double (&y)[3], double& val,
                                                double (&nv)[3])
{
    constexpr int N = K + 1;
    double V[3][N], D[3][N];
    const int64_t nx = a.m.nn[0], nxy = (int64_t)a.m.nn[0] * a.m.nn[1];
    const int64_t base = locate<K>(a, y, V, D);
    // one field at a time, its nodal values loaded before any is used (four
    // memory latencies per evaluation instead of one per few loads: 950 -> 805
    // us for the 64^3 band)
    const double* fields[4] = {a.phi, a.nrm[0], a.nrm[1], a.nrm[2]};
    double out[4];
#pragma unroll
    for (int fi = 0; fi < 4; ++fi) {
        const double* __restrict__ f = fields[fi];
        double fc[N * N * N];
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
            for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
                for (int a0 = 0; a0 < N; ++a0) fc[a0 + N * (a1 + N * a2)] = f[base + a0 + nx * a1 + nxy * a2];
        double s = 0.0;
#pragma unroll
        for (int a2 = 0; a2 < N; ++a2)
#pragma unroll
            for (int a1 = 0; a1 < N; ++a1)
#pragma unroll
                for (int a0 = 0; a0 < N; ++a0) s += V[0][a0] * V[1][a1] * V[2][a2] * fc[a0 + N * (a1 + N * a2)];
        out[fi] = s;
    }
    val = out[0];
    nv[0] = out[1];
    nv[1] = out[2];
    nv[2] = out[3];
}

// phi_h(y) and the unit normal at y (the normalised gradient of phi_h, or of
// the nodal normal field when one is given); false where that vector vanishes.
template <int K>
__device__ __forceinline__ bool normal_at(const CpArgs& a, const double (&y)[3], double& val, double (&n)[3])
{
    double g[3];
    if (a.nrm[0]) eval_phi_normal<K>(a, y, val, g);
    else eval_field<K>(a, a.phi, y, val, g);
    const double gn = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    if (!(gn > 0.0)) return false;
#pragma unroll
    for (int d = 0; d < 3; ++d) n[d] = g[d] / gn;
    return true;
}

__device__ __forceinline__ void clip_box(const CpArgs& a, double (&y)[3])
{
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = fmin(fmax(y[d], a.lo[d]), a.hi[d]);
}

// Coordinates of support point i of the mesh.
template <int K>
__device__ __forceinline__ void node_coords(const CpArgs& a, int64_t i, double (&x)[3])
{
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
}

// One outer step from y towards the closest point of x; true once the step
// moved y by less than tol.
template <int K>
__device__ __forceinline__ bool outer_step(const CpArgs& a, const double (&x)[3], double (&y)[3])
{
    const double prev[3] = {y[0], y[1], y[2]};
    double val, n[3];
    for (int s = 0; s < a.normal_steps; ++s) {
        if (normal_at<K>(a, y, val, n)) {
            const double pc = fmin(fmax(val, -kPhiClip), kPhiClip);
            const double dist = a.eps * log((1.0 + pc) / (1.0 - pc));
#pragma unroll
            for (int d = 0; d < 3; ++d) y[d] -= dist * n[d];
            clip_box(a, y);
        }
    }
    if (normal_at<K>(a, y, val, n)) {
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
    return sqrt(dy[0] * dy[0] + dy[1] * dy[1] + dy[2] * dy[2]) < a.tol;
}

__device__ __forceinline__ unsigned long long lanes_below()
{
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Node mode, first pass: the band nodes |phi_g| < phi_lim are appended to list
// with one atomic per 1024-thread workgroup (the waves' counts are summed in
// LDS; same-address atomics serialise, so one per wave took 130 us at 64^3);
// their order does not matter, each point's result is written to its own node.
// Every other node gets y = x and info = -1.
constexpr int kListThreads = 1024;

template <int K>
__global__ void __launch_bounds__(kListThreads) band_list_kernel(CpArgs a, int* __restrict__ list,
                                                                  int* __restrict__ count)
{
    constexpr int NW = kListThreads / 64;
    __shared__ int wcount[NW], wbase[NW], bbase;
    const int64_t i = (int64_t)blockIdx.x * kListThreads + threadIdx.x;
    const int wave = threadIdx.x / 64;
    const bool in_mesh = i < a.n;
    const bool band = in_mesh && fabs(a.phi[i]) < a.phi_lim;
    const unsigned long long mask = __ballot(band);
    if (__lane_id() == 0) wcount[wave] = __popcll(mask);
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < NW; ++w) {
            wbase[w] = t;
            t += wcount[w];
        }
        bbase = t ? atomicAdd(count, t) : 0;
    }
    __syncthreads();
    if (band) list[bbase + wbase[wave] + __popcll(mask & lanes_below())] = (int)i;
    if (in_mesh && !band) {
        double x[3];
        node_coords<K>(a, i, x);
#pragma unroll
        for (int d = 0; d < 3; ++d) a.y[3 * i + d] = x[d];
        a.info[i] = -1;
    }
}

// Persistent projection over a queue of points (the band list, or the caller's
// points 0..n-1): a lane whose point has converged or used max_iter outer steps
// writes it and takes the next one (one atomic per wave and refill), so a
// point that needs many steps does not hold its wave's other lanes idle.
// Every lane leaves once the queue is empty and its point is done; each point
// takes at most max_iter steps, so every wave finishes.
template <int K>
__global__ void __launch_bounds__(256) closest_point_queue_kernel(CpArgs a, const int* __restrict__ list,
                                                                  const int* __restrict__ count,
                                                                  int* __restrict__ next)
{
    const int64_t total = a.pts ? a.n : (int64_t)*count;
    bool have = false, live = true;
    int64_t g = 0;
    int it = 0;
    double x[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
    for (;;) {
        const unsigned long long need = __ballot(live && !have);
        if (need) {
            const int leader = __ffsll((long long)need) - 1;
            int base = 0;
            if (__lane_id() == leader) base = atomicAdd(next, __popcll(need));
            base = __shfl(base, leader);
            if (live && !have) {
                const int64_t q = (int64_t)base + __popcll(need & lanes_below());
                if (q < total) {
                    if (a.pts) {
                        g = q;
#pragma unroll
                        for (int d = 0; d < 3; ++d) x[d] = a.pts[3 * q + d];
                    } else {
                        g = list[q];
                        node_coords<K>(a, g, x);
                    }
#pragma unroll
                    for (int d = 0; d < 3; ++d) y[d] = x[d];
                    it = 0;
                    have = true;
                } else {
                    live = false;
                }
            }
        }
        if (!__ballot(have)) break;   // queue empty and every point written
        if (have) {
            ++it;
            const bool conv = outer_step<K>(a, x, y);
            if (conv || it >= a.max_iter) {
#pragma unroll
                for (int d = 0; d < 3; ++d) a.y[3 * g + d] = y[d];
                a.info[g] = conv ? it : 0;
                have = false;
            }
        }
    }
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

hipError_t launch_closest_points(int k, const CpArgs& a, int* list, int* ctr, int nblocks, hipStream_t s)
{
    if (a.n <= 0) return hipSuccess;
    hipError_t e = launch_fill<int>(ctr, 2, 0, s);   // ctr[0]: band count, ctr[1]: queue head
    if (e != hipSuccess) return e;
    const int64_t blocks = (a.n + kListThreads - 1) / kListThreads;
    if (blocks > INT32_MAX) return hipErrorInvalidValue;
#define VPP_CP(K)                                                                                          \
    if (!a.pts)                                                                                             \
        hipLaunchKernelGGL(band_list_kernel<K>, dim3((unsigned)blocks), dim3(kListThreads), 0, s, a, list, ctr); \
    hipLaunchKernelGGL(closest_point_queue_kernel<K>, dim3(nblocks), dim3(256), 0, s, a, list, ctr, ctr + 1);
    switch (k) {
    case 2: VPP_CP(2) break;
    case 3: VPP_CP(3) break;
    case 4: VPP_CP(4) break;
    default: return hipErrorInvalidValue;
    }
#undef VPP_CP
    return hipGetLastError();
}

// Persistent workgroups of the projection: two per CU (two waves per SIMD), so
// that the lanes are fewer than the points of a typical band and refill from
// the queue, while the loads of one wave still overlap the other's arithmetic.
constexpr int kCpBlocksPerCu = 2;

int closest_point_blocks(int k)
{
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
    switch (k) {
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, closest_point_queue_kernel<2>, 256, 0); break;
    case 3: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, closest_point_queue_kernel<3>, 256, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, closest_point_queue_kernel<4>, 256, 0); break;
    default: break;
    }
    if (e != hipSuccess || per_cu < 1) per_cu = 1;
    if (per_cu > kCpBlocksPerCu) per_cu = kCpBlocksPerCu;
    return per_cu * device_cu_count();
}

}  // namespace vpp
