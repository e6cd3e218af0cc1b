// Device-side building blocks shared by the kernels: argument blocks, the
// coefficient law, 1D sum-factorisation sweeps and the tile geometry.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tables.h"

namespace vpp {

// ---------------------------------------------------------------------------
// Geometry and material law of one problem, as the kernels see it.
//
// The element matrix of cell e is sum_q W_q c_q sum_d h_d^-2 (dN/dxi_d)(dN/dxi_d)^T
// with W_q = w_q0 w_q1 w_q2 hx hy hz (Gauss weights on [0,1]).  We write the
// Gauss-point factor as  c'(phi_q) * wref_q * rd[d]  with
//   c'(phi) = r0 * c(phi),  r0 = hx hy hz / hx^2,  rd = (1, hx^2/hy^2, hx^2/hz^2),
//   wref_q  = w_q0 w_q1 w_q2.
// c(phi) = 1/rho_g + H(clamp(phi)) (1/rho_l - 1/rho_g)        (Eq. rhoEff)
//   linear H:  c' = ca + cb * phi
//   sine ramp: c' = cg + cd * H(phi), H from Eq. heaviside written in phi.
// The arithmetic density mean rho = H rho_l + (1 - H) rho_g, the law App. D
// contrasts with Eq. rhoEff, gives c = 1/rho:
//   linear H:  c' = 1 / (qa + qb * phi)
//   sine ramp: c' = 1 / (qs + qd * H(phi))   (all scaled by 1/r0)
struct MeshArgs {
    int nc[3];        // cells per direction
    int nn[3];        // nodes per direction (k nc + 1)
    int ntile[3];     // workgroup tiles per direction
    int bcmask;       // bit f set: face f (x-,x+,y-,y+,z-,z+) is Dirichlet
    int heaviside;    // 0 linear, 1 sine ramp; 2, 3 the same with the arithmetic density mean
    double ca, cb;    // linear law (scaled by r0)
    double cg, cd;    // sine-ramp law (scaled by r0)
    double qa, qb;    // arithmetic mean, linear H (density scaled by 1/r0)
    double qs, qd;    // arithmetic mean, sine ramp
    double rd[3];
    double dcdphi;    // r0-free (1/rho_l - 1/rho_g), used by the adjoint
    double rho_l, rho_g;
    double r0;
    double mass;      // mass shift mu scaled as the Gauss-point factors: mu hx hy hz (0: no mass term)
};

__host__ __device__ inline int64_t node_index(const MeshArgs& m, int64_t i, int64_t j, int64_t l)
{
    return i + (int64_t)m.nn[0] * (j + (int64_t)m.nn[1] * l);
}

__host__ __device__ inline bool is_dirichlet(const MeshArgs& m, int i, int j, int l)
{
    return ((m.bcmask & 1) && i == 0) || ((m.bcmask & 2) && i == m.nn[0] - 1) ||
           ((m.bcmask & 4) && j == 0) || ((m.bcmask & 8) && j == m.nn[1] - 1) ||
           ((m.bcmask & 16) && l == 0) || ((m.bcmask & 32) && l == m.nn[2] - 1);
}

// Cell (cx, cy, cz) of linear index i (x fastest); false past the last cell.
__host__ __device__ inline bool cell_of(const MeshArgs& m, int64_t i, int& cx, int& cy, int& cz)
{
    if (i >= (int64_t)m.nc[0] * m.nc[1] * m.nc[2]) return false;
    cx = (int)(i % m.nc[0]);
    const int64_t r = i / m.nc[0];
    cy = (int)(r % m.nc[1]);
    cz = (int)(r / m.nc[1]);
    return true;
}

// Parity colouring of the cells for node scatter-adds without atomics: colour
// c holds the cells whose indices have the parities (c & 1, (c >> 1) & 1,
// (c >> 2) & 1).  Two cells of one colour are two or more cells apart along
// some direction, so they share no node and their threads may add into the
// nodes with plain loads and stores; the colours run one launch after another
// in a fixed order, so every node sum is formed in the same order on every
// run.
struct CellColor {
    int c[3];     // parity per direction
    int n[3];     // cells of the colour per direction
};

__host__ __device__ inline CellColor cell_color(const MeshArgs& m, int color)
{
    CellColor cc;
    for (int d = 0; d < 3; ++d) {
        cc.c[d] = (color >> d) & 1;
        cc.n[d] = m.nc[d] > cc.c[d] ? (m.nc[d] - cc.c[d] + 1) / 2 : 0;
    }
    return cc;
}

__host__ __device__ inline int64_t color_count(const CellColor& cc)
{
    return (int64_t)cc.n[0] * cc.n[1] * cc.n[2];
}

// Cell of position i in colour cc; false past the colour's last cell.
__host__ __device__ inline bool color_cell(const CellColor& cc, int64_t i, int& cx, int& cy, int& cz)
{
    if (i >= color_count(cc)) return false;
    const int a = (int)(i % cc.n[0]);
    const int64_t r = i / cc.n[0];
    const int b = (int)(r % cc.n[1]), e = (int)(r / cc.n[1]);
    cx = 2 * a + cc.c[0];
    cy = 2 * b + cc.c[1];
    cz = 2 * e + cc.c[2];
    return true;
}

// Launches launch(colour, blocks) for the eight colours in order, with
// enough blocks of bt threads for one thread per cell of the colour.
template <typename F>
inline hipError_t for_each_color(const MeshArgs& m, int bt, F&& launch)
{
    for (int c = 0; c < 8; ++c) {
        const CellColor cc = cell_color(m, c);
        const int64_t n = color_count(cc);
        if (n == 0) continue;
        launch(cc, (int)((n + bt - 1) / bt));
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Sine-ramp Heaviside of Eq. heaviside written in phi through Eq. distance:
// with a = artanh(phi) = d/(2 eps), H = 1/2 + a/3 + sin(2 pi a/3)/(2 pi) for
// |a| < 3/2, and 0 / 1 beyond.  eps cancels.
template <typename T>
__device__ __forceinline__ T sine_ramp(T phi)
{
    const T lim = T(0.90514825364486640);   // tanh(3/2)
    if (phi >= lim) return T(1);
    if (phi <= -lim) return T(0);
    const T a = T(0.5) * log((T(1) + phi) / (T(1) - phi));
    return T(0.5) + a * T(1.0 / 3.0) + sin(a * T(2.0943951023931955)) * T(0.15915494309189535);
}

template <typename T>
__device__ __forceinline__ T sine_ramp_deriv(T phi)
{
    const T lim = T(0.90514825364486640);
    if (phi >= lim || phi <= -lim) return T(0);
    const T a = T(0.5) * log((T(1) + phi) / (T(1) - phi));
    return (T(1) + cos(a * T(2.0943951023931955))) / (T(3) * (T(1) - phi * phi));
}

template <typename T>
__device__ __forceinline__ T clamp1(T v)
{
    return fmin(fmax(v, T(-1)), T(1));
}

// ---------------------------------------------------------------------------
// Multiply-accumulate with a compile-time coefficient: zero coefficients are
// skipped and unit ones become plain adds (the loops are fully unrolled, so all
// of this folds away).
template <typename T>
struct Acc {
    T s;
    bool init;
    __device__ __forceinline__ Acc() : s(T(0)), init(false) {}
    __device__ __forceinline__ void add(double c, T x)
    {
        if (c == 0.0) return;
        if (!init) {
            s = (c == 1.0) ? x : (c == -1.0 ? -x : T(c) * x);
            init = true;
        } else {
            s = (c == 1.0) ? s + x : (c == -1.0 ? s - x : fma(T(c), x, s));
        }
    }
    __device__ __forceinline__ T get() const { return init ? s : T(0); }
};

enum Mat { MS = 0, MD = 1, MDC = 2, MS2 = 3, MD2 = 4 };

template <int K, Mat M>
__device__ __forceinline__ constexpr double mat(int q, int a)
{
    return M == MS    ? Tab<K>::t.S[q][a]
           : M == MD  ? Tab<K>::t.D[q][a]
           : M == MDC ? Tab<K>::t.Dc[q][a]
           : M == MS2 ? Tab<K>::t.S[q][a] * Tab<K>::t.S[q][a]
                      : Tab<K>::t.D[q][a] * Tab<K>::t.D[q][a];
}

// out[q] = sum_a M[q][a] in[a]   (TR=false)   or   out[a] = sum_q M[q][a] in[q]  (TR=true)
template <int K, Mat M, bool TR, typename T>
__device__ __forceinline__ void line(const T (&in)[K + 1], T (&out)[K + 1])
{
    constexpr int N = K + 1;
#pragma unroll
    for (int o = 0; o < N; ++o) {
        Acc<T> acc;
#pragma unroll
        for (int i = 0; i < N; ++i) acc.add(TR ? mat<K, M>(i, o) : mat<K, M>(o, i), in[i]);
        out[o] = acc.get();
    }
}

// Same, accumulating into out.
template <int K, Mat M, bool TR, typename T>
__device__ __forceinline__ void line_acc(const T (&in)[K + 1], T (&out)[K + 1])
{
    constexpr int N = K + 1;
#pragma unroll
    for (int o = 0; o < N; ++o) {
        T s = out[o];
#pragma unroll
        for (int i = 0; i < N; ++i) {
            const double c = TR ? mat<K, M>(i, o) : mat<K, M>(o, i);
            if (c == 0.0) continue;
            s = (c == 1.0) ? s + in[i] : fma(T(c), in[i], s);
        }
        out[o] = s;
    }
}

// In-place sweep of a 1D matrix along direction DIR of an N^3 array
// (index a0 + N a1 + N^2 a2).
template <int K, Mat M, bool TR, int DIR, typename T>
__device__ __forceinline__ void sweep3(T (&v)[(K + 1) * (K + 1) * (K + 1)])
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
            T in[N], out[N];
#pragma unroll
            for (int a = 0; a < N; ++a) in[a] = v[base + a * st];
            line<K, M, TR>(in, out);
#pragma unroll
            for (int a = 0; a < N; ++a) v[base + a * st] = out[a];
        }
}

// Same on an N^2 plane (index b0 + N b1), direction 0 or 1 of the plane.
template <int K, Mat M, bool TR, int DIR, typename T>
__device__ __forceinline__ void sweep2(T (&v)[(K + 1) * (K + 1)])
{
    constexpr int N = K + 1;
    constexpr int st = DIR == 0 ? 1 : N;
    constexpr int so = DIR == 0 ? N : 1;
#pragma unroll
    for (int i1 = 0; i1 < N; ++i1) {
        const int base = i1 * so;
        T in[N], out[N];
#pragma unroll
        for (int a = 0; a < N; ++a) in[a] = v[base + a * st];
        line<K, M, TR>(in, out);
#pragma unroll
        for (int a = 0; a < N; ++a) v[base + a * st] = out[a];
    }
}

template <int K>
__device__ __forceinline__ constexpr double wref(int q0, int q1, int q2)
{
    return Tab<K>::t.w[q0] * Tab<K>::t.w[q1] * Tab<K>::t.w[q2];
}

// Scaled coefficient c'(phi) at one Gauss point; HV selects the law at
// compile time so that each kernel carries one: the reciprocal mean of
// Eq. rhoEff with H linear (0) or the sine ramp (1), or the arithmetic density
// mean with H linear (2) or the sine ramp (3).
template <int HV, typename T>
__device__ __forceinline__ T coef_scaled(const MeshArgs& m, T phi)
{
    if constexpr (HV == 0) return fma(T(m.cb), clamp1(phi), T(m.ca));
    else if constexpr (HV == 1) return fma(T(m.cd), sine_ramp(clamp1(phi)), T(m.cg));
    else if constexpr (HV == 2) return T(1) / fma(T(m.qb), clamp1(phi), T(m.qa));
    else return T(1) / fma(T(m.qd), sine_ramp(clamp1(phi)), T(m.qs));
}

// Scaled coefficient c'(phi) * wref at every Gauss point of a cell, in place
// (phi values at the Gauss points in, factors out).
template <int K, int HV, typename T>
__device__ __forceinline__ void coef_weights3(const MeshArgs& m, T (&v)[(K + 1) * (K + 1) * (K + 1)])
{
    constexpr int N = K + 1;
#pragma unroll
    for (int q = 0; q < N * N * N; ++q)
        v[q] = coef_scaled<HV>(m, v[q]) * T(wref<K>(q % N, (q / N) % N, q / (N * N)));
}

// ---------------------------------------------------------------------------
// Tile geometry.  A workgroup owns TX x TY x TZ cells; tiles are numbered
// x-fastest.  Workgroups are dispatched round-robin over the 8 XCDs, so block b
// runs on XCD b % 8; remapping b -> (b % 8) * chunk + b / 8 gives every XCD a
// contiguous run of tiles, whose shared faces then meet in the same L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks)
{
    const int chunk = (nblocks + 7) / 8;
    const int x = b % 8, r = b / 8;
    const int full = nblocks - 8 * (chunk - 1);   // XCDs that get `chunk` tiles
    int t;
    if (x < full) t = x * chunk + r;
    else t = full * chunk + (x - full) * (chunk - 1) + r;
    return t;
}

}  // namespace vpp
