/*
 * FP64 CPU oracle for the variable-coefficient pressure-Poisson operator.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark; never by the product path.  No code is shared
 * with the HIP library.
 *
 * Each function cites the part of the paper it follows; the operator is the
 * plain definition (assembled matrix, full quadrature), written for checking by
 * eye rather than for speed.  Parallelism is OpenMP over independent cells
 * (8-colour parity classes, so every matrix entry is summed in a fixed order).
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXN 5           /* up to k = 4 */
#define MAXQ 8           /* Gauss rules used for error integration */

/* ------------------------------------------------------------------------ */
/* 1D Legendre polynomial P_n and its derivative at x in [-1,1] (three-term
 * recurrence).                                                              */
static void legendre(int n, double x, double* P, double* dP)
{
    double p0 = 1.0, p1 = x;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int m = 1; m < n; ++m) {
        double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
        p0 = p1; p1 = p2;
    }
    *P = p1;
    /* (x^2-1) P_n' = n (x P_n - P_{n-1}) */
    *dP = n * (x * p1 - p0) / (x * x - 1.0);
}

/* n-point Gauss-Legendre rule on [0,1] (Sec. "Numerical framework": (k+1)^dim
 * Gauss points).  Newton iteration on the roots of P_n. */
void orc_gauss_rule(int n, double* xi, double* w)
{
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(n, x, &P, &dP);
            double dx = P / dP;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        double P, dP;
        legendre(n, x, &P, &dP);
        /* root x is in descending order for ascending i; map to [0,1] ascending */
        xi[i] = 0.5 * (1.0 - x);
        w[i] = 1.0 / ((1.0 - x * x) * dP * dP);   /* (2/((1-x^2)P'^2)) / 2 */
    }
}

/* Gauss-Lobatto-Legendre points on [0,1]: the end points and the roots of P_k'.
 * (The paper only says "Lagrange polynomials"; the GLL placement is a reading.) */
void orc_gll_points(int k, double* xi)
{
    xi[0] = 0.0;
    xi[k] = 1.0;
    for (int j = 1; j < k; ++j) {
        double x = -cos(M_PI * j / k);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre(k, x, &P, &dP);
            /* Legendre equation: (1-x^2) P'' = 2x P' - k(k+1) P */
            double d2P = (2.0 * x * dP - k * (k + 1.0) * P) / (1.0 - x * x);
            double dx = dP / d2P;
            x -= dx;
            if (fabs(dx) < 1e-17) break;
        }
        xi[j] = 0.5 * (1.0 + x);
    }
}

/* Lagrange polynomial N_a of the nodes x_0..x_k, by the product formula. */
double orc_lagrange(int k, const double* nodes, int a, double x)
{
    double v = 1.0;
    for (int b = 0; b <= k; ++b)
        if (b != a) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
    return v;
}

/* Its derivative: sum over the dropped factor m of the remaining product. */
double orc_lagrange_deriv(int k, const double* nodes, int a, double x)
{
    double s = 0.0;
    for (int m = 0; m <= k; ++m) {
        if (m == a) continue;
        double v = 1.0 / (nodes[a] - nodes[m]);
        for (int b = 0; b <= k; ++b)
            if (b != a && b != m) v *= (x - nodes[b]) / (nodes[a] - nodes[b]);
        s += v;
    }
    return s;
}

/* ------------------------------------------------------------------------ */
/* Coefficient law.                                                          */

/* Smoothed Heaviside.  Linear: H = (phi+1)/2.  Sine ramp: Eq. heaviside with
 * the signed distance recovered from phi by Eq. distance. */
double orc_heaviside(const orc_desc* d, double phi)
{
    if (d->heaviside == 0) return 0.5 * (phi + 1.0);
    if (phi >= 1.0) return 1.0;
    if (phi <= -1.0) return 0.0;
    const double eps = d->eps;
    const double dist = eps * log((1.0 + phi) / (1.0 - phi));
    if (dist <= -3.0 * eps) return 0.0;
    if (dist >= 3.0 * eps) return 1.0;
    return 0.5 + dist / (6.0 * eps) + sin(M_PI * dist / (3.0 * eps)) / (2.0 * M_PI);
}

/* dH/dphi = dH/dd * dd/dphi with dd/dphi = 2 eps / (1 - phi^2). */
double orc_heaviside_deriv(const orc_desc* d, double phi)
{
    if (d->heaviside == 0) return 0.5;
    if (phi >= 1.0 || phi <= -1.0) return 0.0;
    const double eps = d->eps;
    const double dist = eps * log((1.0 + phi) / (1.0 - phi));
    if (dist <= -3.0 * eps || dist >= 3.0 * eps) return 0.0;
    const double dH_dd = 1.0 / (6.0 * eps) + cos(M_PI * dist / (3.0 * eps)) / (6.0 * eps);
    const double dd_dphi = 2.0 * eps / (1.0 - phi * phi);
    return dH_dd * dd_dphi;
}

/* Reciprocal density, Eq. rhoEff, of the level set clamped to [-1,1]. */
double orc_coefficient(const orc_desc* d, double phi)
{
    if (phi > 1.0) phi = 1.0;
    if (phi < -1.0) phi = -1.0;
    const double H = orc_heaviside(d, phi);
    return H / d->rho_l + (1.0 - H) / d->rho_g;
}

/* ------------------------------------------------------------------------ */
/* Lattice helpers.                                                          */

typedef struct {
    int k, n1;                 /* degree, points per direction */
    int nc[3];                 /* cells */
    int64_t N[3];              /* nodes per direction */
    double h[3];
    double W3;                 /* hx*hy*hz */
    double gll[MAXN];
    double gx[MAXN], gw[MAXN]; /* (k+1)-point Gauss rule on [0,1] */
    double V[MAXN][MAXN];      /* V[q][a] = N_a(gx_q) */
    double D[MAXN][MAXN];      /* D[q][a] = N_a'(gx_q) */
} lattice;

static void make_lattice(const orc_desc* d, lattice* L)
{
    L->k = d->degree;
    L->n1 = d->degree + 1;
    for (int i = 0; i < 3; ++i) {
        L->nc[i] = d->ncells[i];
        L->N[i] = (int64_t)d->degree * d->ncells[i] + 1;
        L->h[i] = d->extent[i] / d->ncells[i];
    }
    L->W3 = L->h[0] * L->h[1] * L->h[2];
    orc_gll_points(L->k, L->gll);
    orc_gauss_rule(L->n1, L->gx, L->gw);
    for (int q = 0; q < L->n1; ++q)
        for (int a = 0; a < L->n1; ++a) {
            L->V[q][a] = orc_lagrange(L->k, L->gll, a, L->gx[q]);
            L->D[q][a] = orc_lagrange_deriv(L->k, L->gll, a, L->gx[q]);
        }
}

int64_t orc_num_dofs(const orc_desc* d)
{
    int64_t n = 1;
    for (int i = 0; i < 3; ++i) n *= (int64_t)d->degree * d->ncells[i] + 1;
    return n;
}

int64_t orc_num_qpoints(const orc_desc* d)
{
    int64_t n1 = d->degree + 1;
    return (int64_t)d->ncells[0] * d->ncells[1] * d->ncells[2] * n1 * n1 * n1;
}

static inline int64_t cell_index(const lattice* L, int cx, int cy, int cz)
{
    return cx + (int64_t)L->nc[0] * (cy + (int64_t)L->nc[1] * cz);
}

/* Global indices of the (k+1)^3 nodes of a cell, local index a0 fastest. */
static void cell_dofs(const lattice* L, int cx, int cy, int cz, int64_t* g)
{
    const int k = L->k, n1 = L->n1;
    int a = 0;
    for (int a2 = 0; a2 < n1; ++a2)
        for (int a1 = 0; a1 < n1; ++a1)
            for (int a0 = 0; a0 < n1; ++a0, ++a)
                g[a] = ((int64_t)k * cx + a0)
                     + L->N[0] * (((int64_t)k * cy + a1) + L->N[1] * ((int64_t)k * cz + a2));
}

static int is_dirichlet(const orc_desc* d, const lattice* L, int64_t g)
{
    int64_t i = g % L->N[0];
    int64_t j = (g / L->N[0]) % L->N[1];
    int64_t l = g / (L->N[0] * L->N[1]);
    if (d->bc[0] == 0 && i == 0) return 1;
    if (d->bc[1] == 0 && i == L->N[0] - 1) return 1;
    if (d->bc[2] == 0 && j == 0) return 1;
    if (d->bc[3] == 0 && j == L->N[1] - 1) return 1;
    if (d->bc[4] == 0 && l == 0) return 1;
    if (d->bc[5] == 0 && l == L->N[2] - 1) return 1;
    return 0;
}

/* Values and physical gradients of all 3D basis functions at Gauss point
 * (q0,q1,q2), each one a product of 1D Lagrange factors (tensor-product
 * Lagrange basis on an axis-aligned box cell). */
static void basis_at_qp(const lattice* L, int q0, int q1, int q2,
                        double* N, double* G0, double* G1, double* G2)
{
    const int n1 = L->n1;
    int a = 0;
    for (int a2 = 0; a2 < n1; ++a2)
        for (int a1 = 0; a1 < n1; ++a1)
            for (int a0 = 0; a0 < n1; ++a0, ++a) {
                N[a]  = L->V[q0][a0] * L->V[q1][a1] * L->V[q2][a2];
                G0[a] = L->D[q0][a0] * L->V[q1][a1] * L->V[q2][a2] / L->h[0];
                G1[a] = L->V[q0][a0] * L->D[q1][a1] * L->V[q2][a2] / L->h[1];
                G2[a] = L->V[q0][a0] * L->V[q1][a1] * L->D[q2][a2] / L->h[2];
            }
}

/* ------------------------------------------------------------------------ */
/* Coefficient at the Gauss points: phi_h(x_q) = sum_a N_a(x_q) phi_a, then the
 * clamp and Eq. rhoEff.                                                      */
void orc_coef_qp(const orc_desc* d, const double* phi, double* cq)
{
    lattice L;
    make_lattice(d, &L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    const int64_t ncell = (int64_t)L.nc[0] * L.nc[1] * L.nc[2];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        int cx = (int)(c % L.nc[0]), cy = (int)((c / L.nc[0]) % L.nc[1]),
            cz = (int)(c / ((int64_t)L.nc[0] * L.nc[1]));
        int64_t g[MAXN * MAXN * MAXN];
        double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
               G2[MAXN * MAXN * MAXN];
        cell_dofs(&L, cx, cy, cz, g);
        int q = 0;
        for (int q2 = 0; q2 < n1; ++q2)
            for (int q1 = 0; q1 < n1; ++q1)
                for (int q0 = 0; q0 < n1; ++q0, ++q) {
                    basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                    double ph = 0.0;
                    for (int a = 0; a < nb; ++a) ph += N[a] * phi[g[a]];
                    cq[c * nb + q] = orc_coefficient(d, ph);
                }
    }
}

/* ------------------------------------------------------------------------ */
/* CSR matrix with the lattice sparsity pattern (every node couples to all
 * nodes of the cells that contain it).                                       */
struct orc_csr {
    int64_t n;
    int64_t* rowptr;
    int64_t* col;
    double* val;
    /* per-row column ranges, used to locate entries during assembly */
    int64_t N[3];
    int k;
};

static void node_range(int64_t i, int k, int nc, int64_t* lo, int64_t* hi)
{
    int64_t cmin, cmax;
    if (i % k == 0) { cmin = i / k - 1; cmax = i / k; }
    else { cmin = cmax = i / k; }
    if (cmin < 0) cmin = 0;
    if (cmax > nc - 1) cmax = nc - 1;
    *lo = (int64_t)k * cmin;
    *hi = (int64_t)k * (cmax + 1);
}

static orc_csr* make_pattern(const lattice* L)
{
    orc_csr* A = (orc_csr*)calloc(1, sizeof(orc_csr));
    const int64_t Nx = L->N[0], Ny = L->N[1], Nz = L->N[2];
    A->n = Nx * Ny * Nz;
    A->k = L->k;
    A->N[0] = Nx; A->N[1] = Ny; A->N[2] = Nz;
    A->rowptr = (int64_t*)malloc((A->n + 1) * sizeof(int64_t));
    A->rowptr[0] = 0;
    for (int64_t g = 0; g < A->n; ++g) {
        int64_t i = g % Nx, j = (g / Nx) % Ny, l = g / (Nx * Ny);
        int64_t lx, hx, ly, hy, lz, hz;
        node_range(i, L->k, L->nc[0], &lx, &hx);
        node_range(j, L->k, L->nc[1], &ly, &hy);
        node_range(l, L->k, L->nc[2], &lz, &hz);
        A->rowptr[g + 1] = A->rowptr[g] + (hx - lx + 1) * (hy - ly + 1) * (hz - lz + 1);
    }
    const int64_t nnz = A->rowptr[A->n];
    A->col = (int64_t*)malloc(nnz * sizeof(int64_t));
    A->val = (double*)calloc(nnz, sizeof(double));
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < A->n; ++g) {
        int64_t i = g % Nx, j = (g / Nx) % Ny, l = g / (Nx * Ny);
        int64_t lx, hx, ly, hy, lz, hz;
        node_range(i, L->k, L->nc[0], &lx, &hx);
        node_range(j, L->k, L->nc[1], &ly, &hy);
        node_range(l, L->k, L->nc[2], &lz, &hz);
        int64_t p = A->rowptr[g];
        for (int64_t c = lz; c <= hz; ++c)
            for (int64_t b = ly; b <= hy; ++b)
                for (int64_t a = lx; a <= hx; ++a)
                    A->col[p++] = a + Nx * (b + Ny * c);
    }
    return A;
}

/* Position of column gc inside row gr (both lattice nodes of one cell). */
static inline int64_t entry_pos(const orc_csr* A, const lattice* L, int64_t gr, int64_t gc)
{
    const int64_t Nx = A->N[0], Ny = A->N[1];
    int64_t i = gr % Nx, j = (gr / Nx) % Ny, l = gr / (Nx * Ny);
    int64_t lx, hx, ly, hy, lz, hz;
    node_range(i, L->k, L->nc[0], &lx, &hx);
    node_range(j, L->k, L->nc[1], &ly, &hy);
    node_range(l, L->k, L->nc[2], &lz, &hz);
    int64_t ci = gc % Nx, cj = (gc / Nx) % Ny, cl = gc / (Nx * Ny);
    return A->rowptr[gr] + ((cl - lz) * (hy - ly + 1) + (cj - ly)) * (hx - lx + 1) + (ci - lx);
}

/* Assembly: K_e[a][b] = sum_q c_q W_q grad N_a . grad N_b, summed into the
 * global matrix (y = sum_i R_i^T A_i R_i x, Sec. "Numerical framework").
 * cq holds c at every Gauss point (cell-major). */
static orc_csr* assemble_from_cq(const orc_desc* d, const double* cq, int constrained)
{
    lattice L;
    make_lattice(d, &L);
    orc_csr* A = make_pattern(&L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
        const int mx = (L.nc[0] - px + 1) / 2, my = (L.nc[1] - py + 1) / 2,
                  mz = (L.nc[2] - pz + 1) / 2;
        const int64_t m = (int64_t)mx * my * mz;
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t t = 0; t < m; ++t) {
            const int cx = px + 2 * (int)(t % mx);
            const int cy = py + 2 * (int)((t / mx) % my);
            const int cz = pz + 2 * (int)(t / ((int64_t)mx * my));
            const int64_t c = cell_index(&L, cx, cy, cz);
            int64_t g[MAXN * MAXN * MAXN];
            double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
                   G2[MAXN * MAXN * MAXN];
            double* K = (double*)calloc((size_t)nb * nb, sizeof(double));
            cell_dofs(&L, cx, cy, cz, g);
            int q = 0;
            for (int q2 = 0; q2 < n1; ++q2)
                for (int q1 = 0; q1 < n1; ++q1)
                    for (int q0 = 0; q0 < n1; ++q0, ++q) {
                        basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                        const double W = L.gw[q0] * L.gw[q1] * L.gw[q2] * L.W3;
                        const double cw = cq[c * nb + q] * W;
                        const double mw = d->mass * W;
                        for (int a = 0; a < nb; ++a)
                            for (int b = 0; b < nb; ++b)
                                K[a * nb + b] += cw * (G0[a] * G0[b] + G1[a] * G1[b] + G2[a] * G2[b]) +
                                                 mw * N[a] * N[b];
                    }
            for (int a = 0; a < nb; ++a)
                for (int b = 0; b < nb; ++b)
                    A->val[entry_pos(A, &L, g[a], g[b])] += K[a * nb + b];
            free(K);
        }
    }
    if (constrained) {
        /* Dirichlet rows and columns replaced by the identity (A_D = [A_II 0; 0 I]). */
        char* bnd = (char*)malloc(A->n);
#pragma omp parallel for schedule(static)
        for (int64_t gi = 0; gi < A->n; ++gi) bnd[gi] = (char)is_dirichlet(d, &L, gi);
#pragma omp parallel for schedule(static)
        for (int64_t r = 0; r < A->n; ++r)
            for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; ++p) {
                const int64_t cc = A->col[p];
                if (bnd[r] || bnd[cc]) A->val[p] = (r == cc && bnd[r]) ? 1.0 : 0.0;
            }
        free(bnd);
    }
    return A;
}

orc_csr* orc_assemble(const orc_desc* d, const double* phi, int constrained)
{
    const int64_t nq = orc_num_qpoints(d);
    double* cq = (double*)malloc(nq * sizeof(double));
    orc_coef_qp(d, phi, cq);
    orc_csr* A = assemble_from_cq(d, cq, constrained);
    free(cq);
    return A;
}

orc_csr* orc_assemble_cq(const orc_desc* d, const double* cq, int constrained)
{
    return assemble_from_cq(d, cq, constrained);
}

void orc_free(orc_csr* A)
{
    if (!A) return;
    free(A->rowptr); free(A->col); free(A->val); free(A);
}

int64_t orc_rows(const orc_csr* A) { return A->n; }
int64_t orc_nnz(const orc_csr* A) { return A->rowptr[A->n]; }

void orc_export(const orc_csr* A, int64_t* rowptr, int64_t* col, double* val)
{
    memcpy(rowptr, A->rowptr, (A->n + 1) * sizeof(int64_t));
    memcpy(col, A->col, orc_nnz(A) * sizeof(int64_t));
    memcpy(val, A->val, orc_nnz(A) * sizeof(double));
}

void orc_spmv(const orc_csr* A, const double* x, double* y)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < A->n; ++r) {
        double s = 0.0;
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; ++p) s += A->val[p] * x[A->col[p]];
        y[r] = s;
    }
}

void orc_diag(const orc_csr* A, double* dg)
{
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < A->n; ++r) {
        double v = 0.0;
        for (int64_t p = A->rowptr[r]; p < A->rowptr[r + 1]; ++p)
            if (A->col[p] == r) v = A->val[p];
        dg[r] = v;
    }
}

static double dot(int64_t n, const double* a, const double* b)
{
    double s = 0.0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/* Jacobi-preconditioned CG (textbook form, Krylov solvers of Sec. "Numerical
 * framework"); stopping rule of Table tab:solver_settings. */
int orc_pcg(const orc_csr* A, const double* b, double* x, double rtol, double atol,
            int max_iter, int* iters, double* relres)
{
    const int64_t n = A->n;
    double* r = (double*)malloc(n * sizeof(double));
    double* z = (double*)malloc(n * sizeof(double));
    double* p = (double*)malloc(n * sizeof(double));
    double* q = (double*)malloc(n * sizeof(double));
    double* dinv = (double*)malloc(n * sizeof(double));
    orc_diag(A, dinv);
    for (int64_t i = 0; i < n; ++i) dinv[i] = 1.0 / dinv[i];
    orc_spmv(A, x, q);
    for (int64_t i = 0; i < n; ++i) r[i] = b[i] - q[i];
    const double r0 = sqrt(dot(n, r, r));
    int status = 1, it = 0;
    double rn = r0;
    if (r0 < atol || r0 == 0.0) {
        status = 0;
    } else {
        for (int64_t i = 0; i < n; ++i) { z[i] = dinv[i] * r[i]; p[i] = z[i]; }
        double rz = dot(n, r, z);
        for (it = 1; it <= max_iter; ++it) {
            orc_spmv(A, p, q);
            const double pq = dot(n, p, q);
            if (!(pq > 0.0) || !isfinite(pq) || !isfinite(rz)) { status = 2; break; }
            const double alpha = rz / pq;
            for (int64_t i = 0; i < n; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            rn = sqrt(dot(n, r, r));
            if (!isfinite(rn)) { status = 2; break; }
            if (rn < atol || rn / r0 < rtol) { status = 0; break; }
            for (int64_t i = 0; i < n; ++i) z[i] = dinv[i] * r[i];
            const double rz_new = dot(n, r, z);
            const double beta = rz_new / rz;
            rz = rz_new;
            for (int64_t i = 0; i < n; ++i) p[i] = z[i] + beta * p[i];
        }
        if (it > max_iter) it = max_iter;
    }
    if (iters) *iters = it;
    if (relres) *relres = (r0 > 0.0) ? rn / r0 : 0.0;
    free(r); free(z); free(p); free(q); free(dinv);
    return status;
}

/* ------------------------------------------------------------------------ */
/* Load vectors, evaluation, adjoint.                                        */

void orc_rhs_qp(const orc_desc* d, const double* fq, double* b)
{
    lattice L;
    make_lattice(d, &L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    const int64_t n = orc_num_dofs(d);
    memset(b, 0, n * sizeof(double));
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
        const int mx = (L.nc[0] - px + 1) / 2, my = (L.nc[1] - py + 1) / 2,
                  mz = (L.nc[2] - pz + 1) / 2;
        const int64_t m = (int64_t)mx * my * mz;
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < m; ++t) {
            const int cx = px + 2 * (int)(t % mx);
            const int cy = py + 2 * (int)((t / mx) % my);
            const int cz = pz + 2 * (int)(t / ((int64_t)mx * my));
            const int64_t c = cell_index(&L, cx, cy, cz);
            int64_t g[MAXN * MAXN * MAXN];
            double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
                   G2[MAXN * MAXN * MAXN];
            cell_dofs(&L, cx, cy, cz, g);
            int q = 0;
            for (int q2 = 0; q2 < n1; ++q2)
                for (int q1 = 0; q1 < n1; ++q1)
                    for (int q0 = 0; q0 < n1; ++q0, ++q) {
                        basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                        const double W = L.gw[q0] * L.gw[q1] * L.gw[q2] * L.W3;
                        for (int a = 0; a < nb; ++a) b[g[a]] += W * fq[c * nb + q] * N[a];
                    }
        }
    }
}

void orc_rhs_flux(const orc_desc* d, const double* fx, const double* fy, const double* fz,
                  double* b)
{
    lattice L;
    make_lattice(d, &L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    const int64_t n = orc_num_dofs(d);
    memset(b, 0, n * sizeof(double));
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
        const int mx = (L.nc[0] - px + 1) / 2, my = (L.nc[1] - py + 1) / 2,
                  mz = (L.nc[2] - pz + 1) / 2;
        const int64_t m = (int64_t)mx * my * mz;
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < m; ++t) {
            const int cx = px + 2 * (int)(t % mx);
            const int cy = py + 2 * (int)((t / mx) % my);
            const int cz = pz + 2 * (int)(t / ((int64_t)mx * my));
            const int64_t c = cell_index(&L, cx, cy, cz);
            int64_t g[MAXN * MAXN * MAXN];
            double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
                   G2[MAXN * MAXN * MAXN];
            cell_dofs(&L, cx, cy, cz, g);
            int q = 0;
            for (int q2 = 0; q2 < n1; ++q2)
                for (int q1 = 0; q1 < n1; ++q1)
                    for (int q0 = 0; q0 < n1; ++q0, ++q) {
                        basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                        const double W = L.gw[q0] * L.gw[q1] * L.gw[q2] * L.W3;
                        const int64_t iq = c * nb + q;
                        for (int a = 0; a < nb; ++a)
                            b[g[a]] += W * (fx[iq] * G0[a] + fy[iq] * G1[a] + fz[iq] * G2[a]);
                    }
        }
    }
}

void orc_qp_coords(const orc_desc* d, int nq, double* x, double* y, double* z, double* w)
{
    lattice L;
    make_lattice(d, &L);
    double gx[MAXQ], gw[MAXQ];
    orc_gauss_rule(nq, gx, gw);
    const int64_t ncell = (int64_t)L.nc[0] * L.nc[1] * L.nc[2];
    const int64_t nb = (int64_t)nq * nq * nq;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        int cx = (int)(c % L.nc[0]), cy = (int)((c / L.nc[0]) % L.nc[1]),
            cz = (int)(c / ((int64_t)L.nc[0] * L.nc[1]));
        int64_t q = c * nb;
        for (int q2 = 0; q2 < nq; ++q2)
            for (int q1 = 0; q1 < nq; ++q1)
                for (int q0 = 0; q0 < nq; ++q0, ++q) {
                    x[q] = d->origin[0] + (cx + gx[q0]) * L.h[0];
                    y[q] = d->origin[1] + (cy + gx[q1]) * L.h[1];
                    z[q] = d->origin[2] + (cz + gx[q2]) * L.h[2];
                    w[q] = gw[q0] * gw[q1] * gw[q2] * L.W3;
                }
    }
}

void orc_eval_qp(const orc_desc* d, int nq, const double* u, double* vals)
{
    lattice L;
    make_lattice(d, &L);
    double gx[MAXQ], gw[MAXQ];
    orc_gauss_rule(nq, gx, gw);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    double V[MAXQ][MAXN];
    for (int q = 0; q < nq; ++q)
        for (int a = 0; a < n1; ++a) V[q][a] = orc_lagrange(L.k, L.gll, a, gx[q]);
    const int64_t ncell = (int64_t)L.nc[0] * L.nc[1] * L.nc[2];
    const int64_t nqb = (int64_t)nq * nq * nq;
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        int cx = (int)(c % L.nc[0]), cy = (int)((c / L.nc[0]) % L.nc[1]),
            cz = (int)(c / ((int64_t)L.nc[0] * L.nc[1]));
        int64_t g[MAXN * MAXN * MAXN];
        cell_dofs(&L, cx, cy, cz, g);
        int64_t q = c * nqb;
        for (int q2 = 0; q2 < nq; ++q2)
            for (int q1 = 0; q1 < nq; ++q1)
                for (int q0 = 0; q0 < nq; ++q0, ++q) {
                    double s = 0.0;
                    int a = 0;
                    for (int a2 = 0; a2 < n1; ++a2)
                        for (int a1 = 0; a1 < n1; ++a1)
                            for (int a0 = 0; a0 < n1; ++a0, ++a)
                                s += V[q0][a0] * V[q1][a1] * V[q2][a2] * u[g[a]];
                    vals[q] = s;
                }
    }
}

/* dJ/dc_q = -lam^T (dA/dc_q) p, with dA/dc_q = W_q B_q^T B_q on the free rows
 * and columns (B_q: the 3 x (k+1)^3 matrix of basis gradients at x_q). */
void orc_grad_coef(const orc_desc* d, const double* p, const double* lam, double* gq)
{
    lattice L;
    make_lattice(d, &L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    const int64_t ncell = (int64_t)L.nc[0] * L.nc[1] * L.nc[2];
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < ncell; ++c) {
        int cx = (int)(c % L.nc[0]), cy = (int)((c / L.nc[0]) % L.nc[1]),
            cz = (int)(c / ((int64_t)L.nc[0] * L.nc[1]));
        int64_t g[MAXN * MAXN * MAXN];
        double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
               G2[MAXN * MAXN * MAXN], pe[MAXN * MAXN * MAXN], le[MAXN * MAXN * MAXN];
        cell_dofs(&L, cx, cy, cz, g);
        for (int a = 0; a < nb; ++a) {
            const int bnd = is_dirichlet(d, &L, g[a]);
            pe[a] = bnd ? 0.0 : p[g[a]];
            le[a] = bnd ? 0.0 : lam[g[a]];
        }
        int q = 0;
        for (int q2 = 0; q2 < n1; ++q2)
            for (int q1 = 0; q1 < n1; ++q1)
                for (int q0 = 0; q0 < n1; ++q0, ++q) {
                    basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                    const double W = L.gw[q0] * L.gw[q1] * L.gw[q2] * L.W3;
                    double Bp[3] = {0, 0, 0}, Bl[3] = {0, 0, 0};
                    for (int a = 0; a < nb; ++a) {
                        Bp[0] += G0[a] * pe[a]; Bp[1] += G1[a] * pe[a]; Bp[2] += G2[a] * pe[a];
                        Bl[0] += G0[a] * le[a]; Bl[1] += G1[a] * le[a]; Bl[2] += G2[a] * le[a];
                    }
                    gq[c * nb + q] = -W * (Bl[0] * Bp[0] + Bl[1] * Bp[1] + Bl[2] * Bp[2]);
                }
    }
}

/* Chain rule through the clamp, the Heaviside and Eq. rhoEff:
 * dc/dphi = (1/rho_l - 1/rho_g) H'(phi), zero where |phi_h| >= 1. */
void orc_grad_phi(const orc_desc* d, const double* phi, const double* gq, double* gphi)
{
    lattice L;
    make_lattice(d, &L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
    memset(gphi, 0, orc_num_dofs(d) * sizeof(double));
    const double dc = 1.0 / d->rho_l - 1.0 / d->rho_g;
    for (int color = 0; color < 8; ++color) {
        const int px = color & 1, py = (color >> 1) & 1, pz = (color >> 2) & 1;
        const int mx = (L.nc[0] - px + 1) / 2, my = (L.nc[1] - py + 1) / 2,
                  mz = (L.nc[2] - pz + 1) / 2;
        const int64_t m = (int64_t)mx * my * mz;
#pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < m; ++t) {
            const int cx = px + 2 * (int)(t % mx);
            const int cy = py + 2 * (int)((t / mx) % my);
            const int cz = pz + 2 * (int)(t / ((int64_t)mx * my));
            const int64_t c = cell_index(&L, cx, cy, cz);
            int64_t g[MAXN * MAXN * MAXN];
            double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
                   G2[MAXN * MAXN * MAXN];
            cell_dofs(&L, cx, cy, cz, g);
            int q = 0;
            for (int q2 = 0; q2 < n1; ++q2)
                for (int q1 = 0; q1 < n1; ++q1)
                    for (int q0 = 0; q0 < n1; ++q0, ++q) {
                        basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                        double ph = 0.0;
                        for (int a = 0; a < nb; ++a) ph += N[a] * phi[g[a]];
                        if (!(fabs(ph) < 1.0)) continue;
                        const double s = gq[c * nb + q] * dc * orc_heaviside_deriv(d, ph);
                        for (int a = 0; a < nb; ++a) gphi[g[a]] += s * N[a];
                    }
        }
    }
}

/* Rows of y = A_D x for selected nodes, each assembled from the (at most 8)
 * cells that contain the node; used to check full-size results one row at a
 * time without assembling the whole matrix. */
void orc_apply_rows(const orc_desc* d, const double* phi, const double* x, const int64_t* rows,
                    int64_t nrows, double* out)
{
    lattice L;
    make_lattice(d, &L);
    const int n1 = L.n1, nb = n1 * n1 * n1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t g = rows[r];
        if (is_dirichlet(d, &L, g)) { out[r] = x[g]; continue; }
        const int64_t i = g % L.N[0], j = (g / L.N[0]) % L.N[1], l = g / (L.N[0] * L.N[1]);
        int64_t lo[3], hi[3];
        const int64_t idx[3] = {i, j, l};
        for (int dd = 0; dd < 3; ++dd) {
            int64_t a, b;
            node_range(idx[dd], L.k, L.nc[dd], &a, &b);
            lo[dd] = a / L.k;           /* first cell */
            hi[dd] = b / L.k - 1;       /* last cell */
        }
        double s = 0.0;
        for (int64_t cz = lo[2]; cz <= hi[2]; ++cz)
            for (int64_t cy = lo[1]; cy <= hi[1]; ++cy)
                for (int64_t cx = lo[0]; cx <= hi[0]; ++cx) {
                    int64_t gg[MAXN * MAXN * MAXN];
                    double N[MAXN * MAXN * MAXN], G0[MAXN * MAXN * MAXN], G1[MAXN * MAXN * MAXN],
                           G2[MAXN * MAXN * MAXN];
                    cell_dofs(&L, (int)cx, (int)cy, (int)cz, gg);
                    int arow = -1;
                    for (int a = 0; a < nb; ++a) if (gg[a] == g) arow = a;
                    int q = 0;
                    for (int q2 = 0; q2 < n1; ++q2)
                        for (int q1 = 0; q1 < n1; ++q1)
                            for (int q0 = 0; q0 < n1; ++q0, ++q) {
                                basis_at_qp(&L, q0, q1, q2, N, G0, G1, G2);
                                double ph = 0.0;
                                for (int a = 0; a < nb; ++a) ph += N[a] * phi[gg[a]];
                                const double W = L.gw[q0] * L.gw[q1] * L.gw[q2] * L.W3;
                                const double cw = orc_coefficient(d, ph) * W;
                                const double mw = d->mass * W;
                                for (int b = 0; b < nb; ++b) {
                                    if (is_dirichlet(d, &L, gg[b])) continue;
                                    s += (cw * (G0[arow] * G0[b] + G1[arow] * G1[b] + G2[arow] * G2[b]) +
                                          mw * N[arow] * N[b]) * x[gg[b]];
                                }
                            }
                }
        out[r] = s;
    }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
