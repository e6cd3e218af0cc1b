/*
 * FP64 CPU oracle for the variable-coefficient pressure-Poisson operator.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library.  It shares no code with
 * the HIP library: its own basis, quadrature, assembly and solver.
 *
 * What it computes (definitions, not an optimised method):
 *   a(p,q) = sum_cells sum_Gauss W_q c(x_q) grad p . grad q     (weak pressure terms, App. F)
 *          + mu sum_cells sum_Gauss W_q p q                      (mass shift; mu = 1 and a
 *            constant c = eta h^2 give the filters of Eqs. normal_vector_regularized and
 *            curvature_regularized in weak form)
 *   c = 1/rho(phi) = H(phi)/rho_l + (1-H(phi))/rho_g            (Eq. rhoEff)
 *   H linear (phi+1)/2, or the sine ramp of Eq. heaviside in d(phi) (Eq. distance)
 *   (k+1)^3 Gauss points per cell (Sec. "Numerical framework")
 *   y = sum_i R_i^T A_i R_i x  realised as an assembled CSR matrix (Sec. "Numerical framework")
 *   Jacobi-preconditioned CG with the stopping rule of Table tab:solver_settings.
 * Every element matrix is built by evaluating the 3D basis gradients at every
 * Gauss point as products of 1D Lagrange polynomials (product formula), with no
 * sum factorisation.
 */
#ifndef VPP_ORACLE_H
#define VPP_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t ncells[3];
    double origin[3];
    double extent[3];
    int32_t degree;      /* 1..4 */
    int32_t bc[6];       /* 0 Dirichlet, 1 Neumann; faces x-,x+,y-,y+,z-,z+ */
    double rho_l, rho_g;
    int32_t heaviside;   /* 0 linear, 1 sine ramp */
    double eps;          /* interface thickness (used by the sine ramp's d(phi)) */
    double mass;         /* mass shift mu: the operator is mu M + K_c (0: pressure operator) */
} orc_desc;

typedef struct orc_csr orc_csr;

/* 1D tables (for the pins). */
void orc_gll_points(int k, double* xi);                       /* k+1 points on [0,1] */
void orc_gauss_rule(int n, double* xi, double* w);             /* n points on [0,1] */
double orc_lagrange(int k, const double* nodes, int a, double x);
double orc_lagrange_deriv(int k, const double* nodes, int a, double x);

/* Coefficient law at one value of the interpolated level set. */
double orc_heaviside(const orc_desc* d, double phi);
double orc_heaviside_deriv(const orc_desc* d, double phi);
double orc_coefficient(const orc_desc* d, double phi);        /* clamps phi to [-1,1] */

int64_t orc_num_dofs(const orc_desc* d);
int64_t orc_num_qpoints(const orc_desc* d);                    /* ncells * (k+1)^3 */

/* c at every Gauss point, cell-major (cell = cx + nx(cy + ny cz)), q0 fastest. */
void orc_coef_qp(const orc_desc* d, const double* phi, double* cq);

/* Assembly.  constrained=1: Dirichlet rows and columns replaced by identity. */
orc_csr* orc_assemble(const orc_desc* d, const double* phi, int constrained);
orc_csr* orc_assemble_cq(const orc_desc* d, const double* cq, int constrained);
void orc_free(orc_csr* A);
int64_t orc_rows(const orc_csr* A);
int64_t orc_nnz(const orc_csr* A);
void orc_export(const orc_csr* A, int64_t* rowptr, int64_t* col, double* val);
void orc_spmv(const orc_csr* A, const double* x, double* y);
void orc_diag(const orc_csr* A, double* dg);

/* Jacobi PCG from x (initial guess in, solution out).  Stops when
 * ||r|| < atol or ||r||/||r0|| < rtol.  Returns 0 converged, 1 max_iter,
 * 2 breakdown (p.Ap <= 0 or non-finite). */
int orc_pcg(const orc_csr* A, const double* b, double* x, double rtol, double atol,
            int max_iter, int* iters, double* relres);

/* Load vectors (all rows, no constraint applied):
 *   rhs_qp:   b_i = sum W_q f_q N_i(x_q)          fq at the (k+1)^3 Gauss points
 *   rhs_flux: b_i = sum W_q F_q . grad N_i(x_q)   F given as 3 arrays of Gauss values */
void orc_rhs_qp(const orc_desc* d, const double* fq, double* b);
void orc_rhs_flux(const orc_desc* d, const double* fx, const double* fy, const double* fz,
                  double* b);

/* Coordinates (3 arrays) and weights of an nq-point Gauss rule in every cell,
 * and the values of the FE function u there. */
void orc_qp_coords(const orc_desc* d, int nq, double* x, double* y, double* z, double* w);
void orc_eval_qp(const orc_desc* d, int nq, const double* u, double* vals);

/* Adjoint pieces.
 * grad_coef: g_q = -W_q grad(lam_h) . grad(p_h) with Dirichlet entries of p, lam
 *            taken as zero (derivative of the constrained operator).
 * grad_phi:  dJ/dphi_j = sum g_q dc/dphi(phi_h(x_q)) [|phi_h(x_q)|<1] N_j(x_q). */
void orc_grad_coef(const orc_desc* d, const double* p, const double* lam, double* gq);
void orc_grad_phi(const orc_desc* d, const double* phi, const double* gq, double* gphi);

/* Selected rows of y = A_D x, each from the cells around its node. */
void orc_apply_rows(const orc_desc* d, const double* phi, const double* x, const int64_t* rows,
                    int64_t nrows, double* out);

int orc_num_threads(void);
void orc_set_num_threads(int n);                               /* n > 0; later calls only */

#ifdef __cplusplus
}
#endif
#endif
