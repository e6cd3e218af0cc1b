/*
 * vpp -- matrix-free variable-coefficient pressure-Poisson operator on MI355X.
 *
 * Problem (App. F, pressure terms of Eq. weakNavierStokes; Sec. "Numerical
 * framework"): find p in Q_k (Dirichlet-constrained) with
 *     a(p,q) = sum_cells sum_{Gauss x_q} W_q c(x_q) grad p . grad q = l(q)
 * on a uniform box of hexahedra, with (k+1)^3 Gauss points per cell and the
 * reciprocal density of Eq. rhoEff as coefficient,
 *     c = 1/rho(phi) = H(phi)/rho_l + (1 - H(phi))/rho_g,
 * where phi is the nodal conservative level set (Eq. initial_phi), interpolated
 * to the Gauss points with the Q_k basis and clamped to [-1,1].  H is either
 * the linear indicator (phi+1)/2 or the sine ramp of Eq. heaviside, which in
 * terms of phi does not depend on eps (via Eq. distance).
 * The operator is applied matrix-free, y = sum_i R_i^T A_i R_i x
 * (Sec. "Numerical framework"), and solved by Jacobi-preconditioned CG with
 * the stopping rule of Table tab:solver_settings.
 *
 * Conventions for every entry point:
 *  - Vectors are device pointers on the problem's device, length N =
 *    prod_d (k n_d + 1), lexicographic node order with x fastest,
 *    g = i + Nx (j + Ny l).  The caller owns them.  Each must be aligned to
 *    its element size (8 bytes for FP64, 4 for FP32 and int32), else
 *    VPP_ERR_INVALID_ARG.
 *  - Dirichlet rows/columns: the operator is A_D = [A_II 0; 0 I] (identity on
 *    nodes of Dirichlet faces; their entries of x never reach free rows).
 *  - `stream` is a hipStream_t passed as void* (NULL = default stream).  Calls
 *    are stream-ordered and asynchronous unless stated otherwise.
 *  - Calls on one problem (or one batch) must not overlap in time: they share
 *    the library's workspace.
 *  - Errors are return codes; argument checks run before any launch.  The
 *    message of the last error on the calling thread is in vpp_last_error().
 */
#ifndef VPP_H
#define VPP_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VPP_ABI_VERSION 1

typedef struct vpp_problem_s* vpp_problem;
typedef struct vpp_batch_s* vpp_batch;

typedef enum {
    VPP_OK = 0,
    VPP_ERR_INVALID_ARG = 1,
    VPP_ERR_UNSUPPORTED = 2,
    VPP_ERR_OUT_OF_MEMORY = 3,
    VPP_ERR_HIP = 4,
    VPP_ERR_NOT_CONVERGED = 5,
    VPP_ERR_BREAKDOWN = 6,
    VPP_ERR_STATE = 7
} vpp_status;

enum { VPP_BC_DIRICHLET = 0, VPP_BC_NEUMANN = 1 };       /* faces x-,x+,y-,y+,z-,z+ */
/* Material law.  VPP_H_LINEAR / VPP_H_PAPER: the reciprocal density of
 * Eq. rhoEff with H = (phi+1)/2 or the sine ramp of Eq. heaviside.
 * VPP_H_LINEAR_ARITH / VPP_H_PAPER_ARITH: the same H with the arithmetic
 * density mean, c = 1/(H rho_l + (1 - H) rho_g), the law App. D contrasts with
 * Eq. rhoEff (its 1D phase-change flow keeps the diffuse pressure jump only
 * with the reciprocal mean).  The arithmetic laws run one kernel configuration
 * per degree (the autotuner has a single candidate), apply / diagonal / CG /
 * vpp_grad_coef; vpp_grad_phi, the mass shift and batches return
 * VPP_ERR_UNSUPPORTED for them. */
enum { VPP_H_LINEAR = 0, VPP_H_PAPER = 1, VPP_H_LINEAR_ARITH = 2, VPP_H_PAPER_ARITH = 3 };
enum { VPP_FP64 = 0, VPP_FP32 = 1, VPP_MIXED = 2 };

/* Mesh, element degree and material law of one problem. */
typedef struct {
    int32_t ncells[3];      /* cells per direction, >= 1 */
    double origin[3];
    double extent[3];       /* box lengths, > 0 */
    int32_t degree;         /* k in {2,3,4} */
    int32_t bc[6];          /* VPP_BC_* per face */
    double rho_l, rho_g;    /* liquid (phi>0) and gas densities, > 0 */
    int32_t heaviside;      /* VPP_H_* (material law) */
    int32_t device;         /* HIP device ordinal */
} vpp_desc;

/* CG controls.  Convergence (Table tab:solver_settings): ||r||_2 < atol or
 * ||r||_2 / ||r0||_2 < rtol, r0 the initial residual.  precision VPP_MIXED runs
 * the PCG recurrences with the FP32 operator and FP32 vectors and keeps the
 * solution, the residual that decides convergence and every CG scalar in FP64:
 * each time the FP32 residual has dropped by inner_rtol (0 = 1e-2) since the
 * last replacement, the FP32 correction is added to the FP64 solution and the
 * FP32 residual is replaced by the FP64 residual b - A x (the search direction
 * is kept).  A breakdown of the FP32 recurrence (p.Ap <= 0 from FP32 rounding,
 * possible when inner_rtol asks for more than the FP32 operator can resolve)
 * restarts it from the FP64 residual; a second one without progress hands the
 * rest of the solve to FP64 PCG.  inner_max_iter (0 = none) caps the FP32
 * iterations between two replacements.  check_every = iterations between host-side checks of the
 * device stop flag (0 = 32).  Scalars of every CG are FP64.
 *
 * deflate (VPP_MIXED only; 0 = off, at most 8): the first FP32 phase is
 * recorded (its FP32 residuals, at most deflate_history of them, 0 = 512, and
 * never more than a quarter of the free device memory, allocated on first use
 * and kept with the problem) and its CG coefficients give the Lanczos matrix
 * of the Jacobi-scaled operator.  Of its `deflate` smallest Ritz values those
 * followed by a gap (the next one at least 10 times larger: isolated near-null
 * modes such as the nearly constant pressure inside a gas bubble) give Ritz
 * vectors W, and every replacement also adds the Galerkin correction
 * x += W (W^T A W)^-1 W^T r.  This keeps the smallest eigenvalues that FP64
 * PCG would have resolved from returning at every replacement; without such a
 * gap nothing is deflated.  A correction that would move the residual by more than a
 * tenth of its norm is skipped (it would no longer fit the kept search
 * direction); if the first one is, the solve continues without deflation. */
typedef struct {
    double rtol, atol;
    int32_t max_iter, precision;
    double inner_rtol;
    int32_t inner_max_iter, check_every;
    int32_t deflate, deflate_history;
} vpp_cg_opts;

typedef struct {
    int32_t iterations;        /* CG iterations (for VPP_MIXED: FP32 plus any FP64 fallback iterations) */
    int32_t outer_iterations;  /* FP64 residual replacements (0 unless VPP_MIXED) */
    int32_t status;            /* vpp_status of the solve */
    double rel_residual;       /* ||r|| / ||r0|| as tracked by the (outer) iteration */
    double true_rel_residual;  /* ||b - A x|| / ||b - A x0|| recomputed in FP64 at the end */
    int32_t deflation_corrections;   /* Galerkin corrections applied (VPP_MIXED with deflate > 0) */
    double deflation_first_change;   /* ||A W c|| / ||r|| of the first correction considered (-1: none) */
} vpp_cg_info;

/* Options of the closest-point projection (vpp_closest_points). */
typedef struct {
    double eps;                /* interface thickness of Eq. distance, > 0 */
    double phi_lim;            /* narrow band |phi| < phi_lim of the node mode, in (0, 1] */
    double tol;                /* stop once |y^(k+1) - y^(k)| < tol, > 0 */
    int32_t max_iter;          /* outer steps, 1..10000 */
    int32_t normal_steps;      /* normal corrections per outer step, 0..100 */
} vpp_cp_opts;

/* Options of the reinitialization step (vpp_reinit_step). */
typedef struct {
    double eps;                /* interface thickness, > 0 */
    double dtau;               /* pseudo-time step, > 0 (the paper takes min(eps, dt)) */
    double rtol, atol;         /* CG stopping rule (Table tab:solver_settings: 1e-12, 1e-20) */
    int32_t max_iter;          /* 0..1e7 */
} vpp_reinit_opts;

/* Kernel configuration: cells of one workgroup tile (tx, ty, tz). */
typedef struct {
    int32_t tile[3];
    int32_t variant;           /* 0 = cell per thread, LDS atomic accumulation (k = 2);
                                  1 = plane per thread (k = 2, 3, 4);
                                  2 = half a cell per thread, z-planes split over a
                                      lane pair (k = 3);
                                  4 = cell per thread, LDS slot exchange (k = 2, 3) */
} vpp_kernel_config;

/* Create a problem on desc->device (host call, allocates device workspace and
 * the per-degree tables).  VPP_ERR_INVALID_ARG for null pointers, degree not in
 * {2,3,4}, ncells < 1, extent <= 0, rho <= 0 or unknown enum values. */
vpp_status vpp_create(const vpp_desc* desc, vpp_problem* out);
vpp_status vpp_destroy(vpp_problem p);

int64_t vpp_num_dofs(vpp_problem p);        /* prod_d (k n_d + 1), -1 on null */
int64_t vpp_num_qpoints(vpp_problem p);     /* prod_d n_d * (k+1)^3, -1 on null */

/* Copy nodal phi (FP64 device pointer, N entries) into the problem and build the
 * Jacobi diagonal for it (Table tab:solver_settings, "diagonal" preconditioner).
 * Must precede apply / solve / gradient calls. */
vpp_status vpp_set_phi(vpp_problem p, const double* phi, void* stream);

/* Mass shift: the operator becomes mu M + K_c (Dirichlet rows stay identity
 * rows), M the Q_k mass matrix with the same (k+1)^3 Gauss rule.  With mu = 1,
 * rho_l = rho_g = 1/(eta h^2) and Neumann faces it is the weak form of the
 * level-set filters n - eta h^2 Lap n = n_bar and kappa - eta h^2 Lap kappa =
 * kappa_bar (Eqs. normal_vector_regularized, curvature_regularized; solved
 * with CG and the diagonal preconditioner, Table tab:solver_settings); the
 * right-hand sides (n_bar, v) are inputs like every b here.  mu >= 0, finite;
 * mu = 0 restores the pressure operator.  With mu != 0 the problem runs the
 * configurations instantiated with the shift (variant 4 for k = 2, 3, variant
 * 1 for k = 4; vpp_set_config rejects others, the current ones are switched
 * if needed).  Rebuilds the diagonal if phi is
 * set; synchronizes `stream` and the problem's stream.  Batches copy their
 * problems' operators when created, so set mu before vpp_batch_create. */
vpp_status vpp_set_mass(vpp_problem p, double mu, void* stream);

/* y = A_D x.  prec VPP_FP64: x, y are double*; VPP_FP32: float* (the
 * coefficient and tables are then FP32 too).  x and y must not alias. */
vpp_status vpp_apply(vpp_problem p, int32_t prec, const void* x, void* y, void* stream);

/* y = A_D x without any allocation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  The problem is described by desc and the nodal phi
 * (FP64 device pointers: phi, x, y, N entries each, y not aliased) instead of
 * a vpp_problem; FP64 only, with a fixed kernel configuration per degree (no
 * autotuning).  The shared-face partials go to a static device array of the
 * library (48 MiB per device, held from the library's load on that device to
 * the end of the process; its address is looked up on the first call on each
 * device): meshes whose partials do not fit (above about 64^3 Q2, 43^3 Q3 or
 * 32^3 Q4 cells) return VPP_ERR_UNSUPPORTED before any launch.  Calls that
 * overlap in time on one device race on that array (serialise them, e.g. on
 * one stream).  Argument checks as vpp_create and vpp_apply; asynchronous on
 * `stream`; no hipMalloc, hipFree or other allocating call. */
vpp_status vpp_apply_noalloc(const vpp_desc* desc, const double* phi, const double* x, double* y, void* stream);

/* diag(A_D) in FP64 (1 on Dirichlet rows). */
vpp_status vpp_diagonal(vpp_problem p, double* diag, void* stream);

/* Jacobi PCG (FP64 or mixed) for A_D x = b.  x holds the initial guess on entry
 * and the last iterate on exit (also when not converged).  Synchronises the
 * stream; returns VPP_ERR_NOT_CONVERGED / VPP_ERR_BREAKDOWN with info filled. */
vpp_status vpp_cg_solve(vpp_problem p, const double* b, double* x, const vpp_cg_opts* opts,
                        vpp_cg_info* info, void* stream);

/* Adjoint pieces for J(p(phi)) with A_D p = b, b independent of phi.
 * grad_coef: g_q = dJ/dc_q = -W_q grad(lam_h) . grad(p_h) at every Gauss point
 *   (Dirichlet entries of p and lam count as zero), where lam solves
 *   A_D lam = dJ/dp.  Output layout: cell-major, cell = cx + nx (cy + ny cz),
 *   Gauss index q0 + (k+1)(q1 + (k+1) q2) within a cell; vpp_num_qpoints entries.
 * grad_phi: dJ/dphi_j = sum_q g_q (1/rho_l - 1/rho_g) H'(phi_h(x_q))
 *   [|phi_h(x_q)| < 1] N_j(x_q)  (chain rule through the clamp, H and Eq. rhoEff). */
vpp_status vpp_grad_coef(vpp_problem p, const double* pv, const double* lam, double* g_q,
                         void* stream);
vpp_status vpp_grad_phi(vpp_problem p, const double* g_q, double* g_phi, void* stream);

/* Closest points on the zero isosurface {phi_h = 0} of the FE level set
 * (appendix "Extension of solution quantities from a level-set isosurface
 * using closest point projection", Eq. cpp), one GPU thread per point.  From
 * y = x each outer step takes opts->normal_steps corrections
 * y <- y - d(y) n(y) (d of Eq. distance from phi_h(y), n = grad phi_h/|grad phi_h|)
 * and one tangential correction y <- y - sum_j ((y - x).t_j) t_j (unit
 * tangents t_0 from v = e_x, or e_y when |n_x| > 0.9, and t_1 = n x t_0), until
 * |y^(k+1) - y^(k)| < tol; y is clipped to the domain box after every
 * correction.  pts: n points, xyz interleaved (device, FP64); or NULL for the
 * narrow band of the mesh's support points: then n is ignored, the outputs
 * have vpp_num_dofs entries and node g is projected iff |phi_g| < phi_lim.
 * y: 3 entries per point (xyz); info: outer steps to convergence, 0 when
 * max_iter steps did not converge (y is the last iterate; the gradient of
 * phi_h jumps across cell faces, so points projecting onto a face can cycle;
 * vpp_closest_points_normal, with a continuous normal, avoids this), -1
 * for a node outside the band (y = x).  Needs vpp_set_phi; VPP_ERR_UNSUPPORTED
 * for more than 2^31 - 2^24 points.  Asynchronous on `stream`. */
vpp_status vpp_closest_points(vpp_problem p, const double* pts, int64_t n, const vpp_cp_opts* opts,
                              double* y, int32_t* info, void* stream);

/* The same projection with the interface normal n_Gamma of Eq. cpp taken as
 * the paper defines it, the filtered normal of Eq. normal_vector_regularized:
 * n(y) = n_h(y)/|n_h(y)| for the nodal field (n0, n1, n2) (N entries each,
 * FP64 device pointers; typically the three solutions of the normal filter
 * system, vpp_set_mass and vpp_normal_rhs).  n_h is continuous across cell
 * faces, so far fewer points cycle than with the gradient of phi_h.  phi_h
 * still gives the distance of Eq. distance.  Errors and outputs as for
 * vpp_closest_points; VPP_ERR_INVALID_ARG if a component is NULL. */
vpp_status vpp_closest_points_normal(vpp_problem p, const double* pts, int64_t n, const double* n0,
                                     const double* n1, const double* n2, const vpp_cp_opts* opts,
                                     double* y, int32_t* info, void* stream);

/* vpp_grad_phi, the filter right-hand sides below and the reinitialization
 * calls form every cell's contributions first and then sum them into the
 * nodes, each node over its cells in a fixed order (no atomics: repeated calls
 * give identical bits).  The contributions go to a scratch buffer of the
 * problem, (k+1)^3 doubles per cell (three times that for vpp_normal_rhs),
 * allocated at the first call that needs it (VPP_ERR_OUT_OF_MEMORY if it
 * cannot be); calls on different streams that use it are ordered by an event.
 *
 * Right-hand sides of the level-set filter systems (vpp_set_mass), assembled
 * on every row of the problem's mesh with its (k+1)^3 Gauss rule, no
 * constraint applied:
 *   vpp_normal_rhs:    b_d = (n_bar_d, v), n_bar = grad phi_h / |grad phi_h|
 *                      (Eq. normal_vector; 0 where the gradient vanishes) for
 *                      the nodal level set phi given here (N entries);
 *   vpp_curvature_rhs: b = (kappa_bar, v), kappa_bar = -div n_h (Eq. curvature)
 *                      for the nodal normal components n0, n1, n2 (N each),
 *                      typically the solutions of the normal filter.
 * FP64 device pointers, outputs not aliased with inputs.  The phi of the
 * problem (vpp_set_phi) is not used.  Asynchronous on `stream`. */
vpp_status vpp_normal_rhs(vpp_problem p, const double* phi, double* b0, double* b1, double* b2, void* stream);
vpp_status vpp_curvature_rhs(vpp_problem p, const double* n0, const double* n1, const double* n2, double* b,
                             void* stream);

/* One step of the level-set reinitialization (Eq. reinitialization): the
 * semi-implicit Euler step in pseudo-time with the compressive flux explicit,
 *   (psi', v)/dtau + eps ((grad psi' . n)(grad v . n))
 *       = (psi, v)/dtau + ((1 - psi^2)/2 n, grad v),
 * solved by Jacobi-preconditioned CG (Table tab:solver_settings) from psi'
 * = psi.  n: the nodal (filtered) normal components n0, n1, n2, interpolated at
 * the Gauss points as they are; the boundary terms of both integrations by
 * parts are dropped (natural conditions on every face, whatever the problem's
 * faces).  The operator, its diagonal and the right-hand side are evaluated
 * per cell by sum factorization into the problem's cell scratch, then summed
 * into the nodes over their cells in a fixed order (no atomics: repeated calls
 * give the same bits).  psi, n0..n2, psi_out: N
 * entries, FP64 device pointers; psi_out may alias psi.  The problem's phi and
 * mass shift are not used.  Synchronizes; info as for vpp_cg_solve. */
vpp_status vpp_reinit_step(vpp_problem p, const double* psi, const double* n0, const double* n1,
                           const double* n2, const vpp_reinit_opts* opts, double* psi_out,
                           vpp_cg_info* info, void* stream);

/* The three pieces of that step on their own, each formed exactly as
 * vpp_reinit_step forms it (same kernels, natural conditions on every face):
 *   vpp_reinit_apply:    y = A x,  A = M/dtau + eps K_n, K_n the matrix of
 *                        ((grad u . n)(grad v . n)) (Eq. reinitialization,
 *                        diffusion implicit);
 *   vpp_reinit_diagonal: diag = diag(A) (the step's Jacobi preconditioner);
 *   vpp_reinit_rhs:      b = (psi, v)/dtau + ((1 - psi_h^2)/2 n, grad v)
 *                        (the explicit compressive flux).
 * Only opts->eps and opts->dtau are read (> 0, finite).  n0..n2, x, psi: N
 * entries; y, diag, b: N entries written (need no initialisation), not
 * aliased with an input.  FP64 device pointers; asynchronous on `stream`. */
vpp_status vpp_reinit_apply(vpp_problem p, const double* n0, const double* n1, const double* n2,
                            const vpp_reinit_opts* opts, const double* x, double* y, void* stream);
vpp_status vpp_reinit_diagonal(vpp_problem p, const double* n0, const double* n1, const double* n2,
                               const vpp_reinit_opts* opts, double* diag, void* stream);
vpp_status vpp_reinit_rhs(vpp_problem p, const double* psi, const double* n0, const double* n1,
                          const double* n2, const vpp_reinit_opts* opts, double* b, void* stream);

/* Extension of a nodal Q_k field f of the mesh from the interface over the
 * narrow band (same appendix: values at the closest points extended to the
 * band): out[g] = f_h(y_g), the FE interpolant at node g's closest point, for
 * every node with info[g] >= 0, and out[g] = f[g] for info[g] = -1.  y, info:
 * the node-mode output of vpp_closest_points (3 N and N entries); f, out: N
 * entries, FP64 device pointers, not aliased.  Asynchronous on `stream`. */
vpp_status vpp_extend(vpp_problem p, const double* y, const int32_t* info, const double* f, double* out,
                      void* stream);

/* Once-refined meshes with hanging nodes (adaptive refinement around the
 * interface, Sec. "Numerical framework", restricted to one level): the box of
 * `coarse` with the coarse cells marked in `refined` (host array, one byte per
 * coarse cell, cx fastest; nonzero = split into 2 x 2 x 2) refined once.
 * Unknowns sit in one vector of vpp_amr_num_dofs entries: the coarse lattice
 * (k n_d + 1 nodes per direction, lexicographic, x fastest) and then the fine
 * lattice over the whole box (2 k n_d + 1 per direction).  Free unknowns are
 * the coarse nodes of unrefined cells and the fine nodes of refined cells that
 * lie on no unrefined cell; a fine node on the closure of an unrefined cell is
 * constrained to that cell's Q_k interpolant (a hanging node, or a copy where
 * it coincides with a coarse node), so the space stays continuous.  The
 * operator is A = C^T A_cells C (C the constraints, A_cells the element
 * matrices of the active cells with the coefficient of Eq. rhoEff from the
 * nodal phi of the cell's own lattice), with identity rows and columns on
 * every entry that is not a free unknown and on free unknowns of Dirichlet
 * faces (as A_D).  The apply and the diagonal run one cell per thread into a
 * cell-major scratch, then sum every entry over the cell results reaching it
 * (lists built on the host, constraint weights included) in a fixed order: no
 * atomics, repeated calls give the same bits; FP64 only.  Calls on one mesh
 * share that scratch and must not overlap.
 *   vpp_amr_create:   host call; VPP_ERR_INVALID_ARG as vpp_create, or for a
 *                     NULL mask, more than 2^27 coarse cells or 2^31 entries.
 *   vpp_amr_set_phi:  nodal phi on both lattices (vpp_amr_num_dofs entries);
 *                     builds the Jacobi diagonal.
 *   vpp_amr_apply:    y = A x (all entries written); x, y not aliased.
 *   vpp_amr_diagonal: diag(A), 1 on identity rows.
 *   vpp_amr_cg_solve: Jacobi PCG as vpp_cg_solve (opts->precision VPP_FP64,
 *                     else VPP_ERR_UNSUPPORTED); synchronizes.
 * vpp_amr_num_free: the number of free unknowns not on Dirichlet faces. */
typedef struct vpp_amr_s* vpp_amr;
vpp_status vpp_amr_create(const vpp_desc* coarse, const uint8_t* refined, vpp_amr* out);
vpp_status vpp_amr_destroy(vpp_amr a);
int64_t vpp_amr_num_dofs(vpp_amr a);
int64_t vpp_amr_num_free(vpp_amr a);
vpp_status vpp_amr_set_phi(vpp_amr a, const double* phi, void* stream);
vpp_status vpp_amr_apply(vpp_amr a, const double* x, double* y, void* stream);
vpp_status vpp_amr_diagonal(vpp_amr a, double* diag, void* stream);
vpp_status vpp_amr_cg_solve(vpp_amr a, const double* b, double* x, const vpp_cg_opts* opts, vpp_cg_info* info,
                            void* stream);

/* Kernel configuration of a problem (what the autotuner chooses), held per
 * precision: the FP64 and the FP32 apply may use different kernels and tiles.
 * Setting an unsupported one returns VPP_ERR_UNSUPPORTED.  vpp_get_config /
 * vpp_set_config read the FP64 choice / set both.  vpp_tune times the
 * candidates of both precisions on this problem (synchronises) and keeps the
 * fastest of each; every timed apply follows a write of a 512 MiB scratch
 * buffer (allocated for the call), so operands come from HBM rather than from
 * the last-level cache.  With a non-NULL cache path the choices are read from /
 * added to that JSON file. */
vpp_status vpp_get_config(vpp_problem p, vpp_kernel_config* cfg);
vpp_status vpp_set_config(vpp_problem p, const vpp_kernel_config* cfg);
/* precision: VPP_FP64 or VPP_FP32 (VPP_ERR_INVALID_ARG otherwise). */
vpp_status vpp_get_config_for(vpp_problem p, int32_t precision, vpp_kernel_config* cfg);
vpp_status vpp_set_config_for(vpp_problem p, int32_t precision, const vpp_kernel_config* cfg);
vpp_status vpp_tune(vpp_problem p, const char* cache_path, void* stream);
/* Candidate list for a degree: writes up to `cap` configs, returns the count. */
int32_t vpp_config_candidates(int32_t degree, vpp_kernel_config* out, int32_t cap);

/* Batch of independent problems (same degree, k = 2 or 3; FP64) with nrhs[i]
 * right-hand sides each, applied by ONE persistent kernel that pulls work
 * items from a device queue, followed by one assembly launch for the
 * shared-face nodes of every (problem, rhs); both launches are recorded in one
 * hipGraph.  k = 2: an item is a (problem, tile), the coefficient of the tile
 * computed once for all right-hand sides of its problem; k = 3: an item is a
 * (problem, tile, rhs), the items of one tile consecutive, the coefficient
 * recomputed per item.  Degree 4 returns VPP_ERR_UNSUPPORTED.
 * tune_cache: JSON cache path for the autotuner, or NULL to tune without a cache.
 * The problems must have phi set and outlive the batch. */
vpp_status vpp_batch_create(const vpp_problem* probs, const int32_t* nrhs, int32_t nprob,
                            const char* tune_cache, vpp_batch* out);
/* x, y: host arrays of sum(nrhs) device pointers, ordered problem-major. */
vpp_status vpp_batch_apply(vpp_batch b, const double* const* x, double* const* y, void* stream);
/* One Jacobi-PCG per (problem, rhs) pair (Sec. "Numerical framework", Krylov
 * solver with the diagonal preconditioner; stopping rule as vpp_cg_solve).
 * rhs, x: host arrays of sum(nrhs) device pointers, ordered problem-major; x
 * holds the initial guesses on entry and the solutions on return.
 * VPP_FP64: the systems of meshes below 2^20 unknowns iterate in lockstep,
 * one iteration being one persistent batched apply and two batched vector
 * launches over every such system that has not stopped (systems that have
 * stopped are skipped), recorded in a hipGraph of check_every iterations; each
 * system's reductions are summed in the order of a single solve on the batch's
 * tiles.  Systems of larger meshes fill the GPU on their own and are solved
 * one after another with vpp_cg_solve (and the problem's tuned kernels), after
 * the lockstep group.  VPP_MIXED: every system is solved with vpp_cg_solve, one
 * after another.  Synchronizes.
 * info: sum(nrhs) entries (may be NULL).  Returns the first non-OK status of
 * the systems (VPP_ERR_NOT_CONVERGED, VPP_ERR_BREAKDOWN) after all of them
 * have been solved; every x then holds its last iterate. */
vpp_status vpp_batch_cg_solve(vpp_batch b, const double* const* rhs, double* const* x,
                              const vpp_cg_opts* opts, vpp_cg_info* info, void* stream);
vpp_status vpp_batch_get_config(vpp_batch b, vpp_kernel_config* cfg);
vpp_status vpp_batch_destroy(vpp_batch b);

const char* vpp_last_error(void);            /* thread-local message, never NULL */
int32_t vpp_abi_version(void);

/* Bounds checks (no passage of the paper: a debugging aid for the index
 * arithmetic of the tile kernels).  The same sources also build
 * libvpp_debug.so with every global and LDS access of the apply tile kernels
 * (all variants, single and batched) and of the shared-node assembly checked
 * against the extent of the buffer it belongs to; an access outside is
 * counted and dropped (a load yields zero), so kernels still complete.
 * Returns the count since the previous call and resets it (synchronizes the
 * current device first); -1 in the release library (no checks compiled in),
 * -2 if the counters could not be read. */
int64_t vpp_debug_bounds_violations(void);

#ifdef __cplusplus
}
#endif
#endif
