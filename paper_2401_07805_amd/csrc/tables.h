// Compile-time 1D tables of the Q_k tensor-product element on [0,1].
//
// Support points: Gauss-Lobatto-Legendre points (reading of "Lagrange
// polynomials", Sec. "Numerical framework"); quadrature: (k+1)-point Gauss rule
// per direction (same section).  All values are derived at compile time from
// closed forms of the points and the product formula of Lagrange polynomials,
// so the sweep loops below fold them into immediates.
//
//   S[q][a]  = L_a(g_q)        GLL Lagrange basis at Gauss point q
//   D[q][a]  = L_a'(g_q)       its derivative
//   Dc[q][p] = l_p'(g_q)       derivative of the Lagrange basis through the Gauss
//                              points (collocation derivative at the Gauss points)
//   w[q]                       Gauss weights on [0,1]
#pragma once

namespace vpp {

constexpr double c_sqrt(double a)
{
    double x = a > 1.0 ? a : 1.0;
    for (int i = 0; i < 200; ++i) x = 0.5 * (x + a / x);
    return x;
}

template <int K>
struct Tables {
    static constexpr int N = K + 1;
    double gll[N] = {};
    double gx[N] = {};
    double w[N] = {};
    double S[N][N] = {};
    double D[N][N] = {};
    double Dc[N][N] = {};
};

template <int K>
constexpr Tables<K> make_tables()
{
    constexpr int N = K + 1;
    Tables<K> t{};
    // Gauss-Legendre rule on [-1,1] (closed forms), mapped to [0,1].
    double x[N] = {}, w[N] = {};
    if constexpr (N == 3) {
        const double r = c_sqrt(3.0 / 5.0);
        x[0] = -r; x[1] = 0.0; x[2] = r;
        w[0] = 5.0 / 9.0; w[1] = 8.0 / 9.0; w[2] = 5.0 / 9.0;
    } else if constexpr (N == 4) {
        const double s = c_sqrt(6.0 / 5.0);
        const double a = c_sqrt(3.0 / 7.0 - 2.0 / 7.0 * s);
        const double b = c_sqrt(3.0 / 7.0 + 2.0 / 7.0 * s);
        const double s30 = c_sqrt(30.0);
        x[0] = -b; x[1] = -a; x[2] = a; x[3] = b;
        w[0] = (18.0 - s30) / 36.0; w[1] = (18.0 + s30) / 36.0;
        w[2] = w[1]; w[3] = w[0];
    } else {
        static_assert(N == 5, "degree 2..4");
        const double s = c_sqrt(10.0 / 7.0);
        const double a = c_sqrt(5.0 - 2.0 * s) / 3.0;
        const double b = c_sqrt(5.0 + 2.0 * s) / 3.0;
        const double s70 = c_sqrt(70.0);
        x[0] = -b; x[1] = -a; x[2] = 0.0; x[3] = a; x[4] = b;
        w[0] = (322.0 - 13.0 * s70) / 900.0; w[1] = (322.0 + 13.0 * s70) / 900.0;
        w[2] = 128.0 / 225.0; w[3] = w[1]; w[4] = w[0];
    }
    for (int i = 0; i < N; ++i) {
        t.gx[i] = 0.5 * (x[i] + 1.0);
        t.w[i] = 0.5 * w[i];
    }
    // GLL points on [-1,1]: ends and the roots of P_k'.
    double g[N] = {};
    g[0] = -1.0; g[N - 1] = 1.0;
    if constexpr (K == 2) {
        g[1] = 0.0;
    } else if constexpr (K == 3) {
        g[1] = -1.0 / c_sqrt(5.0); g[2] = 1.0 / c_sqrt(5.0);
    } else {
        g[1] = -c_sqrt(3.0 / 7.0); g[2] = 0.0; g[3] = c_sqrt(3.0 / 7.0);
    }
    for (int i = 0; i < N; ++i) t.gll[i] = 0.5 * (g[i] + 1.0);
    // Lagrange values / derivatives by the product formula.
    for (int q = 0; q < N; ++q)
        for (int a = 0; a < N; ++a) {
            double v = 1.0;
            for (int b = 0; b < N; ++b)
                if (b != a) v *= (t.gx[q] - t.gll[b]) / (t.gll[a] - t.gll[b]);
            t.S[q][a] = v;
            double d = 0.0;
            for (int m = 0; m < N; ++m) {
                if (m == a) continue;
                double p = 1.0 / (t.gll[a] - t.gll[m]);
                for (int b = 0; b < N; ++b)
                    if (b != a && b != m) p *= (t.gx[q] - t.gll[b]) / (t.gll[a] - t.gll[b]);
                d += p;
            }
            t.D[q][a] = d;
            double dc = 0.0;
            for (int m = 0; m < N; ++m) {
                if (m == a) continue;
                double p = 1.0 / (t.gx[a] - t.gx[m]);
                for (int b = 0; b < N; ++b)
                    if (b != a && b != m) p *= (t.gx[q] - t.gx[b]) / (t.gx[a] - t.gx[b]);
                dc += p;
            }
            t.Dc[q][a] = dc;
        }
    // Exact structural zeros/ones: for odd N the middle Gauss point is the middle
    // GLL node, so that row of S is a unit vector.
    if constexpr (N % 2 == 1) {
        for (int a = 0; a < N; ++a) t.S[N / 2][a] = (a == N / 2) ? 1.0 : 0.0;
        t.Dc[N / 2][N / 2] = 0.0;
        t.D[N / 2][N / 2] = 0.0;
    }
    return t;
}

template <int K>
struct Tab {
    static constexpr Tables<K> t = make_tables<K>();
};

}  // namespace vpp
