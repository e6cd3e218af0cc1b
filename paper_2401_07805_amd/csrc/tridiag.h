// Smallest eigenpairs of a real symmetric tridiagonal matrix (host code, no
// HIP): the Lanczos matrix that the CG coefficients of the first FP32 phase of
// a mixed-precision solve define.  Eigenvalues by bisection on Sturm sequence
// counts, eigenvectors by inverse iteration with a partially pivoted
// tridiagonal factorization, re-orthogonalized against the vectors of nearby
// eigenvalues.
#pragma once
#include <algorithm>
#include <cmath>
#include <vector>

namespace vpp {

// Number of eigenvalues of T (diagonal d[0..m), off-diagonal e[0..m-1)) below x.
inline int tridiag_count_below(int m, const double* d, const double* e, double x, double tiny)
{
    // a (near-)zero pivot is replaced by -tiny and counted as negative in the
    // same step, so that the count stays consistent with the shifted factorization
    int c = 0;
    double q = d[0] - x;
    if (std::fabs(q) < tiny) q = -tiny;
    if (q < 0) ++c;
    for (int i = 1; i < m; ++i) {
        q = d[i] - x - e[i - 1] * e[i - 1] / q;
        if (std::fabs(q) < tiny) q = -tiny;
        if (q < 0) ++c;
    }
    return c;
}

// Solve (T - s I) y = b in place (b -> y) by Gaussian elimination with
// partial pivoting on the tridiagonal band; zero pivots are replaced by `tiny`.
inline void tridiag_shift_solve(int m, const double* d, const double* e, double s, double tiny, double* b)
{
    std::vector<double> a(m), c(m), u1(m), u2(m);
    // row i: sub a[i] (column i-1), diag c[i], super u1[i] (column i+1), second super u2[i]
    for (int i = 0; i < m; ++i) {
        c[i] = d[i] - s;
        a[i] = i > 0 ? e[i - 1] : 0.0;
        u1[i] = i + 1 < m ? e[i] : 0.0;
        u2[i] = 0.0;
    }
    for (int i = 0; i + 1 < m; ++i) {
        // candidates for the pivot of column i: row i (c[i]) and row i+1 (a[i+1])
        if (std::fabs(a[i + 1]) > std::fabs(c[i])) {
            std::swap(c[i], a[i + 1]);
            std::swap(u1[i], c[i + 1]);
            std::swap(u2[i], u1[i + 1]);
            std::swap(b[i], b[i + 1]);
        }
        if (std::fabs(c[i]) < tiny) c[i] = tiny;
        const double f = a[i + 1] / c[i];
        a[i + 1] = 0.0;
        c[i + 1] -= f * u1[i];
        u1[i + 1] -= f * u2[i];
        b[i + 1] -= f * b[i];
    }
    if (std::fabs(c[m - 1]) < tiny) c[m - 1] = tiny;
    for (int i = m - 1; i >= 0; --i) {
        double v = b[i];
        if (i + 1 < m) v -= u1[i] * b[i + 1];
        if (i + 2 < m) v -= u2[i] * b[i + 2];
        b[i] = v / c[i];
    }
}

// Gershgorin bounds and the largest absolute row sum of T.
inline void tridiag_bounds(int m, const double* d, const double* e, double* lo, double* hi, double* scale)
{
    *lo = d[0];
    *hi = d[0];
    *scale = 0.0;
    for (int i = 0; i < m; ++i) {
        const double r = (i > 0 ? std::fabs(e[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(e[i]) : 0.0);
        *lo = std::min(*lo, d[i] - r);
        *hi = std::max(*hi, d[i] + r);
        *scale = std::max(*scale, std::fabs(d[i]) + r);
    }
    if (*scale == 0.0) *scale = 1.0;
}

// The k smallest eigenvalues (ascending, vals[0..k)).  Returns k (at most m).
inline int tridiag_smallest_values(int m, const double* d, const double* e, int k, double* vals)
{
    k = std::min(k, m);
    if (k <= 0) return 0;
    double lo, hi, scale;
    tridiag_bounds(m, d, e, &lo, &hi, &scale);
    const double tiny = 1e-300 + 1e-17 * scale;
    for (int t = 0; t < k; ++t) {
        // bisection for the (t+1)-th smallest eigenvalue: count_below(x) >= t+1 <=> lambda_t < x
        double a = lo, b = hi;
        for (int it = 0; it < 200 && b - a > 4e-16 * std::max(std::fabs(a), std::fabs(b)) + 1e-300; ++it) {
            const double mid = 0.5 * (a + b);
            if (tridiag_count_below(m, d, e, mid, tiny) >= t + 1) b = mid;
            else a = mid;
        }
        vals[t] = 0.5 * (a + b);
    }
    return k;
}

// Unit eigenvectors (vecs[t * m + j], component j of vector t) of the k
// eigenvalues vals[0..k) (ascending, from tridiag_smallest_values).
inline void tridiag_vectors(int m, const double* d, const double* e, int k, const double* vals, double* vecs)
{
    double lo, hi, scale;
    tridiag_bounds(m, d, e, &lo, &hi, &scale);
    const double tiny = 1e-300 + 1e-17 * scale;
    for (int t = 0; t < k; ++t) {
        double* y = vecs + (size_t)t * m;
        for (int j = 0; j < m; ++j) y[j] = 1.0 + 0.01 * ((j * 7 + t * 13) % 17);   // generic start
        const double shift = vals[t] - 1e-14 * scale;
        for (int pass = 0; pass < 4; ++pass) {
            tridiag_shift_solve(m, d, e, shift, tiny, y);
            // keep the vectors of (nearly) repeated eigenvalues apart
            for (int s = 0; s < t; ++s)
                if (std::fabs(vals[s] - vals[t]) < 1e-7 * scale) {
                    const double* z = vecs + (size_t)s * m;
                    double dot = 0.0;
                    for (int j = 0; j < m; ++j) dot += z[j] * y[j];
                    for (int j = 0; j < m; ++j) y[j] -= dot * z[j];
                }
            double nrm = 0.0;
            for (int j = 0; j < m; ++j) nrm += y[j] * y[j];
            nrm = std::sqrt(nrm);
            if (!(nrm > 0.0) || !std::isfinite(nrm)) {
                for (int j = 0; j < m; ++j) y[j] = (j == t) ? 1.0 : 0.0;
                nrm = 1.0;
            }
            for (int j = 0; j < m; ++j) y[j] /= nrm;
        }
    }
}

// The k smallest eigenvalues (ascending, vals[0..k)) and unit eigenvectors
// (vecs[t * m + j], component j of vector t).  Returns k.
inline int tridiag_smallest(int m, const double* d, const double* e, int k, double* vals, double* vecs)
{
    k = tridiag_smallest_values(m, d, e, k, vals);
    tridiag_vectors(m, d, e, k, vals, vecs);
    return k;
}

}  // namespace vpp
