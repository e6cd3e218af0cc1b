/* Drives every entry point of the C oracle on small meshes, for a build with
 * -fsanitize=address,undefined (tests/test_host_logic.py compiles and runs it
 * on the CPU).  Any out-of-bounds access, use after free, leak or undefined
 * behaviour aborts the run; the few value checks below (operator symmetry,
 * selected rows against the assembled matrix, PCG convergence) make sure the
 * calls did real work.  Exit status: number of failed checks. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/oracle.h"

static int fails = 0;
#define CHECK(c, ...)                        \
    do {                                     \
        if (!(c)) {                          \
            if (fails < 20) printf(__VA_ARGS__); \
            ++fails;                         \
        }                                    \
    } while (0)

static unsigned long long rng = 88172645463325252ULL;
static double urand(double lo, double hi)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return lo + (hi - lo) * (double)(rng >> 11) / 9007199254740992.0;
}

static double* vec(int64_t n, double lo, double hi)
{
    double* v = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) v[i] = urand(lo, hi);
    return v;
}

static void one_mesh(int k, const int nc[3], const double ext[3], const int bc[6], int heav, double mass)
{
    orc_desc d;
    memset(&d, 0, sizeof d);
    for (int i = 0; i < 3; ++i) {
        d.ncells[i] = nc[i];
        d.origin[i] = 0.25 * i;
        d.extent[i] = ext[i];
    }
    for (int f = 0; f < 6; ++f) d.bc[f] = bc[f];
    d.degree = k;
    d.rho_l = 1000.0;
    d.rho_g = 1.0;
    d.heaviside = heav;
    d.eps = 0.3;
    d.mass = mass;
    const int64_t n = orc_num_dofs(&d), nq = orc_num_qpoints(&d);
    /* nodal phi beyond [-1, 1] so that the clamp and the indicator are reached */
    double* phi = vec(n, -1.3, 1.3);
    double* x = vec(n, -1.0, 1.0);
    double* lam = vec(n, -1.0, 1.0);
    double* cq = malloc(sizeof(double) * (size_t)nq);
    orc_coef_qp(&d, phi, cq);
    for (int constrained = 0; constrained < 2; ++constrained) {
        orc_csr* A = orc_assemble(&d, phi, constrained);
        orc_csr* B = orc_assemble_cq(&d, cq, constrained);
        CHECK(orc_rows(A) == n && orc_rows(B) == n, "k=%d rows\n", k);
        const int64_t nnz = orc_nnz(A);
        int64_t* rp = malloc(sizeof(int64_t) * (size_t)(n + 1));
        int64_t* col = malloc(sizeof(int64_t) * (size_t)nnz);
        double* val = malloc(sizeof(double) * (size_t)nnz);
        orc_export(A, rp, col, val);
        CHECK(rp[n] == nnz, "k=%d nnz\n", k);
        /* symmetry of the exported matrix (entry-by-entry search) */
        double asym = 0.0, amax = 0.0;
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
                const int64_t j = col[e];
                double t = 0.0;
                for (int64_t f = rp[j]; f < rp[j + 1]; ++f)
                    if (col[f] == i) t = val[f];
                asym = fmax(asym, fabs(val[e] - t));
                amax = fmax(amax, fabs(val[e]));
            }
        CHECK(asym <= 1e-12 * amax, "k=%d constrained=%d asymmetry %g\n", k, constrained, asym);
        double* y = malloc(sizeof(double) * (size_t)n);
        double* y2 = malloc(sizeof(double) * (size_t)n);
        double* dg = malloc(sizeof(double) * (size_t)n);
        orc_spmv(A, x, y);
        orc_spmv(B, x, y2);
        orc_diag(A, dg);
        double dmax = 0.0, ymax = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            dmax = fmax(dmax, fabs(y[i] - y2[i]));
            ymax = fmax(ymax, fabs(y[i]));
        }
        CHECK(dmax <= 1e-12 * (ymax + 1e-300), "k=%d assemble vs assemble_cq %g\n", k, dmax);
        if (constrained) {
            int64_t* rows = malloc(sizeof(int64_t) * (size_t)n);
            for (int64_t i = 0; i < n; ++i) rows[i] = n - 1 - i;
            double* yr = malloc(sizeof(double) * (size_t)n);
            orc_apply_rows(&d, phi, x, rows, n, yr);
            double rmax = 0.0;
            for (int64_t i = 0; i < n; ++i) rmax = fmax(rmax, fabs(yr[i] - y[rows[i]]));
            CHECK(rmax <= 1e-12 * (ymax + 1e-300), "k=%d apply_rows %g\n", k, rmax);
            /* PCG on an SPD system: Dirichlet faces present or a mass shift */
            const int spd = mass > 0.0 || bc[0] == 0 || bc[1] == 0 || bc[2] == 0 || bc[3] == 0 || bc[4] == 0 ||
                            bc[5] == 0;
            if (spd) {
                double* sol = calloc((size_t)n, sizeof(double));
                int iters = 0;
                double rel = 1.0;
                const int st = orc_pcg(A, y, sol, 1e-12, 0.0, 10000, &iters, &rel);
                CHECK(st == 0 && rel < 1e-12, "k=%d pcg status %d rel %g\n", k, st, rel);
                free(sol);
            }
            free(rows);
            free(yr);
        }
        free(rp);
        free(col);
        free(val);
        free(y);
        free(y2);
        free(dg);
        orc_free(A);
        orc_free(B);
    }
    /* load vectors, point evaluations and the adjoint pieces */
    double* fq = vec(nq, -1.0, 1.0);
    double* fy = vec(nq, -1.0, 1.0);
    double* fz = vec(nq, -1.0, 1.0);
    double* b = malloc(sizeof(double) * (size_t)n);
    orc_rhs_qp(&d, fq, b);
    orc_rhs_flux(&d, fq, fy, fz, b);
    for (int m = 1; m <= 8; ++m) {
        const int64_t ncell = (int64_t)nc[0] * nc[1] * nc[2];
        const int64_t np = ncell * m * m * m;
        double* qx = malloc(sizeof(double) * (size_t)np);
        double* qy = malloc(sizeof(double) * (size_t)np);
        double* qz = malloc(sizeof(double) * (size_t)np);
        double* qw = malloc(sizeof(double) * (size_t)np);
        double* qv = malloc(sizeof(double) * (size_t)np);
        orc_qp_coords(&d, m, qx, qy, qz, qw);
        orc_eval_qp(&d, m, x, qv);
        double vol = 0.0;
        for (int64_t i = 0; i < np; ++i) vol += qw[i];
        CHECK(fabs(vol - ext[0] * ext[1] * ext[2]) < 1e-12, "k=%d nq=%d volume %g\n", k, m, vol);
        free(qx);
        free(qy);
        free(qz);
        free(qw);
        free(qv);
    }
    double* gq = malloc(sizeof(double) * (size_t)nq);
    double* gphi = malloc(sizeof(double) * (size_t)n);
    orc_grad_coef(&d, x, lam, gq);
    orc_grad_phi(&d, phi, gq, gphi);
    free(fq);
    free(fy);
    free(fz);
    free(b);
    free(gq);
    free(gphi);
    free(phi);
    free(x);
    free(lam);
    free(cq);
}

int main(void)
{
    /* 1D tables and the coefficient law */
    double pts[8], w[8];
    for (int k = 1; k <= 4; ++k) {
        orc_gll_points(k, pts);
        for (int a = 0; a <= k; ++a) {
            (void)orc_lagrange(k, pts, a, 0.3);
            (void)orc_lagrange_deriv(k, pts, a, 0.7);
        }
    }
    for (int m = 1; m <= 8; ++m) orc_gauss_rule(m, pts, w);
    orc_desc law;
    memset(&law, 0, sizeof law);
    law.rho_l = 1000.0;
    law.rho_g = 1.0;
    law.eps = 0.1;
    for (int h = 0; h < 2; ++h) {
        law.heaviside = h;
        for (double p = -1.5; p <= 1.5; p += 0.125) {
            (void)orc_heaviside(&law, p);
            (void)orc_heaviside_deriv(&law, p);
            const double c = orc_coefficient(&law, p);
            CHECK(c >= 1.0 / 1000.0 - 1e-15 && c <= 1.0 + 1e-15, "coefficient %g at %g\n", c, p);
        }
    }
    const int meshes[3][3] = {{3, 2, 2}, {2, 3, 1}, {1, 1, 1}};
    const double exts[3][3] = {{1.0, 0.5, 0.75}, {0.6, 1.2, 0.4}, {1.0, 1.0, 1.0}};
    const int bcs[3][6] = {{0, 0, 0, 0, 0, 0}, {0, 1, 1, 0, 1, 1}, {1, 1, 1, 1, 1, 1}};
    for (int k = 1; k <= 4; ++k)
        for (int mi = 0; mi < 3; ++mi)
            for (int bi = 0; bi < 3; ++bi)
                for (int h = 0; h < 2; ++h) one_mesh(k, meshes[mi], exts[mi], bcs[bi], h, bi == 2 ? 1.0 : 0.0);
    orc_set_num_threads(2);
    (void)orc_num_threads();
    one_mesh(2, meshes[0], exts[0], bcs[1], 1, 0.0);
    printf("%d failures\n", fails);
    return fails;
}
