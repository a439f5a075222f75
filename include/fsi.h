/*
 * fsi.h -- C ABI of the MI355X generalized-Stokes hot path (libfsi.so).
 *
 * One stage of the semi-implicit ALE fluid-structure scheme (Algorithm 1,
 * Sec. 3.1.1) solves the generalized Stokes system of Sec. 4,
 *
 *     [ A  B^T ] [u]   [g_u]        a(u,v) = (c_m u, v) + (2 eta eps(u), eps(v)),
 *     [ B  0   ] [p] = [g_p],       b(v,q) = (div v, q),
 *
 * (predictor mode: symmetric A; mass coefficient c_m = rho/(gamma*tau) from the
 * BDF stencil of Sec. 3.1, effective viscosity eta from the stress splitting of
 * Sec. 3.1.1), discretised by Taylor-Hood Q2-Q1 elements on the ALE-mapped mesh
 * (Sec. 3.2, Sec. 5: p1 = 2, p2 = 1) and solved by FGMRES preconditioned with
 * the monolithic block V-cycle of Sec. 4 (smoother K_j with A-hat^{-1} =
 * Cheb(A, diag A, k_A) and S-hat^{-1} = ChebMINRES(n_S, k_S)), defaults from
 * Table 4 (predictor column).
 *
 * Conventions
 *  - Meshes are structured boxes of n_fine cells per direction, obtained from
 *    n_coarse by uniform refinement (the level hierarchy of Sec. 4); level 0 is
 *    the coarsest, level L-1 the finest.
 *  - Cells, Q2 velocity nodes ((2n+1)^dim), Q1 pressure nodes ((n+1)^dim) and
 *    quadrature points (3 Gauss points per direction, 3^dim per cell) are
 *    numbered lexicographically with x fastest.
 *  - Velocity vectors are component-major: u[c * n_vel_nodes + node].
 *  - Every vector/array argument is DEVICE memory owned by the caller unless
 *    stated otherwise; the library never frees it.  Calls are asynchronous and
 *    ordered on the context's stream unless stated otherwise.
 *  - Dirichlet (no-slip) faces: bit f of dirichlet_faces marks face f in the
 *    order (x-, x+, y-, y+, z-, z+).  Constrained velocity rows of A act as the
 *    identity (v_c = u_c), constrained columns of A and B are zero, constrained
 *    rows of B^T are zero.
 *  - Not thread safe per context; one context per stream.
 */
#ifndef FSI_H
#define FSI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fsi_ctx fsi_ctx;
typedef int fsi_status;

#define FSI_OK                  0
#define FSI_NOT_CONVERGED       1   /* solve stopped at max_iter; result still written */
#define FSI_ERR_ARG            -1   /* bad pointer, size, level or parameter */
#define FSI_ERR_STATE          -2   /* call needs set_ calls or fsi_setup first */
#define FSI_ERR_HIP            -3   /* a HIP runtime call failed */
#define FSI_ERR_OOM            -4   /* device allocation failed */
#define FSI_ERR_INVERTED_CELL  -5   /* det J <= 0 at some quadrature point */
#define FSI_ERR_BREAKDOWN      -6   /* Krylov breakdown or singular coarse matrix */
#define FSI_ERR_NONFINITE      -7   /* NaN/Inf in an input or a residual */

#define FSI_PREC_FP64   0   /* V-cycle in FP64 */
#define FSI_PREC_MIXED  1   /* V-cycle velocity work in FP32, Schur pressure block FP64 */

typedef struct {
    int dim;                 /* 2 or 3 */
    int n_fine[3];           /* cells per direction on the finest level */
    double extent[3];        /* reference box [0,extent_0] x ... */
    int n_coarse[3];         /* cells per direction on level 0; n_fine/n_coarse = 2^(L-1) in every direction */
    uint32_t dirichlet_faces;
} fsi_mesh_desc;

typedef struct {
    int64_t n_cells, n_vel_nodes, n_vel, n_p, n_qp, n_vert;
    int cells[3], vel_nodes[3], p_nodes[3];
} fsi_sizes;

/* Multigrid parameters (Sec. 4, Table 4).  fsi_default_mg_params fills the
 * predictor column: k_A=4, m=2, n=1, k_S=1, n_S=1.  The Chebyshev interval of
 * D^{-1}A on each level is [cheb_upper*lam/cheb_ratio, cheb_upper*lam] with lam
 * the largest Ritz value of n_eig Lanczos steps on D^{-1/2} A D^{-1/2}.
 * Only k_S = 1 and n_S = 1 are implemented. */
typedef struct {
    int k_A;
    int m;
    int n_cycles;
    int k_S;
    int n_S;
    double cheb_upper;
    double cheb_ratio;
    int n_eig;
    int precision;           /* FSI_PREC_FP64 or FSI_PREC_MIXED (switching needs no new setup) */
    int use_graph;           /* launch the V-cycle as a captured HIP graph (switching needs no new setup) */
    int fused;               /* 1: Chebyshev steps and residuals fused into the cell kernel's
                                last-touch epilogue; 0: separate vector kernels (same results
                                up to rounding; switching needs no new setup) */
    int tuned;               /* 1: autotuned launch variant per level and, with fused = 1, the
                                fused or separate form per level, whichever fsi_autotune
                                measured faster; 0: the default variant, fused everywhere */
    int vertex_geometry;     /* bit 0: FP32 cell kernels, bit 1: FP64 cell kernels on 3D levels
                                form det(J) w J^{-1} = w adj(J) at each quadrature point from the
                                vertex displacements given to fsi_set_displacement (multilinear
                                map, Sec. 3.2) and read only (2 eta, c_m) per point, instead of
                                reading the stored values; 0: stored values (default).  Levels
                                whose geometry came from fsi_set_jacobians always read the
                                stored values.  Switching needs no new setup. */
    int corrector;           /* 1: corrector mode (Sec. 3.1.1, Sec. 4): every level's velocity
                                block is A + N + S with the terms of fsi_set_convection (needed on
                                every level before fsi_setup), the Schur step is one BiCGStab
                                iteration (ChebBiCGStab(1, 1)) instead of MINRES, the fused
                                epilogues are not used; set k_A = 6 for Table 4's corrector
                                column.  0: predictor mode (default).  Changing it needs a new
                                setup. */
    int atomics;             /* 1 (default): with tuned = 1, the operator classes for which
                                fsi_autotune chose the single atomic launch over all processing
                                phases use it (faster on latency-bound levels; the order of the
                                atomic adds varies, so results differ in the last bits from run
                                to run); 0: phased launches only, bitwise reproducible.
                                Switching needs no new setup. */
} fsi_mg_params;

typedef struct {
    double lambda_max;       /* Lanczos estimate of lambda_max(D^{-1}A) */
    double cheb_lo, cheb_hi; /* Chebyshev interval */
    double diagA_norm2;      /* ||diag(A)||_2 (all velocity dofs) */
    double diagS_norm2;      /* ||diag(B diag(A)^{-1} B^T)||_2 */
    int64_t coarse_n;        /* size of the dense coarse system (level 0 only) */
} fsi_level_info;

typedef struct {
    double rtol;             /* relative true residual ||g - M x||_2 / ||g||_2 */
    int max_iter;
    int restart;
    int reorth;              /* Arnoldi by classical Gram-Schmidt: 0 one pass; 1 a second pass
                                when the first cancelled most of the vector (norm drop
                                below 1/sqrt(2), Daniel-Gragg-Kaufman-Stewart); 2 always two */
} fsi_solve_opts;

typedef struct {
    int iters;
    double final_rel_res;    /* true FP64 residual, recomputed at exit */
    double time_ms;          /* wall time of the solve on the stream */
    int n_hist;              /* entries written to res_history */
    double* res_history;     /* HOST buffer of >= max_iter+1 doubles, may be NULL */
} fsi_solve_info;

/* Create a context for the box hierarchy described by *m.  hip_stream is a
 * hipStream_t (NULL: the library creates and owns one).  Allocates the level
 * structure (maps, colours) but no geometry.  Errors: FSI_ERR_ARG for an
 * invalid description (dim, sizes, non power-of-two ratio), FSI_ERR_OOM. */
fsi_status fsi_create(fsi_ctx** out, const fsi_mesh_desc* m, void* hip_stream);
void fsi_destroy(fsi_ctx* ctx);
const char* fsi_last_error(const fsi_ctx* ctx);
void fsi_default_mg_params(fsi_mg_params* p);

fsi_status fsi_get_num_levels(const fsi_ctx* ctx, int* n_levels);
fsi_status fsi_get_sizes(const fsi_ctx* ctx, int level, fsi_sizes* s);

/* Geometry (Sec. 3.2, mapped spaces): J[cell][q][a][b] = d x_a / d xi_b of the
 * ALE map at Gauss point q of the reference cell [0,1]^dim (so an undeformed
 * cell of size h has J = diag(h)).  FP64 device array of n_cells*Q*dim*dim.
 * The library stores det(J) w_q J^{-1} per quadrature point (FP64 and FP32).
 * New geometry invalidates the level's coefficients (set them again).
 * Errors: FSI_ERR_INVERTED_CELL if det J <= 0 anywhere (synchronises). */
fsi_status fsi_set_jacobians(fsi_ctx* ctx, int level, const double* J);

/* Convenience: vertex displacement d[c][vertex] (FP64, dim*n_vert of the finest
 * level) of the multilinear ALE map x = X + d(X); every level receives the
 * values at its own vertices (injection) and its Jacobians are computed on the
 * device.  Same errors as fsi_set_jacobians. */
fsi_status fsi_set_displacement(fsi_ctx* ctx, const double* disp);

/* Coefficients per quadrature point, FP64 [n_cells][Q] each: c_mass is the
 * implicit BDF mass coefficient rho/(gamma*tau) (Sec. 3.1) and eta the
 * effective viscosity of the stress splitting (Sec. 3.1.1); the form is
 * (c_m u, v) + (2 eta eps(u), eps(v)).  Requires the level's geometry.
 * Errors: FSI_ERR_STATE without geometry, FSI_ERR_NONFINITE if an input is not
 * finite (synchronises). */
fsi_status fsi_set_coefficients(fsi_ctx* ctx, int level, const double* c_mass, const double* eta);

/* Changing k_A, m, n_cycles or the Chebyshev/Lanczos settings requires a new
 * fsi_setup; precision, use_graph, fused and tuned may change at any time
 * (fused = tuned = use_graph = 0 with FP64 is the plain per-launch path).  Errors:
 * FSI_ERR_ARG (only k_S = n_S = 1 are implemented). */
fsi_status fsi_set_mg_params(fsi_ctx* ctx, const fsi_mg_params* p);

/* Setup of the preconditioner on every level: diag(A_j), diag(B_j diag(A_j)^{-1}
 * B_j^T) (Sec. 4), Lanczos bounds, Chebyshev coefficients, the dense inverse of
 * the coarsest block matrix M_0, FP32 copies and the V-cycle graphs of both precisions.
 * Synchronises.  Errors: FSI_ERR_STATE if a level lacks geometry or
 * coefficients, FSI_ERR_BREAKDOWN for a singular coarse matrix. */
fsi_status fsi_setup(fsi_ctx* ctx);
fsi_status fsi_get_level_info(const fsi_ctx* ctx, int level, fsi_level_info* info);

/* Matrix-free operators on one level (Sec. 4 block system), FP64:
 *   apply_A:      v = A u
 *   apply_B:      q = B u
 *   apply_BT:     v = B^T p
 *   apply_stokes: v = A u + B^T p, q = B u
 * u, v: [n_vel]; p, q: [n_p]; outputs are overwritten; inputs and outputs must
 * not alias.  Require geometry and coefficients of that level (B and B^T only
 * geometry).  Errors: FSI_ERR_ARG, FSI_ERR_STATE. */
fsi_status fsi_apply_A(fsi_ctx* ctx, int level, const double* u, double* v);
fsi_status fsi_apply_B(fsi_ctx* ctx, int level, const double* u, double* q);
fsi_status fsi_apply_BT(fsi_ctx* ctx, int level, const double* p, double* v);
fsi_status fsi_apply_stokes(fsi_ctx* ctx, int level, const double* u, const double* p,
                            double* v, double* q);
/* FP32 twins of the same operators, with the FP32 copy of geometry and coefficients. */
fsi_status fsi_apply_A_f32(fsi_ctx* ctx, int level, const float* u, float* v);
fsi_status fsi_apply_B_f32(fsi_ctx* ctx, int level, const float* u, float* q);
fsi_status fsi_apply_BT_f32(fsi_ctx* ctx, int level, const float* p, float* v);
fsi_status fsi_apply_stokes_f32(fsi_ctx* ctx, int level, const float* u, const float* p,
                                float* v, float* q);

/* Allocation-free FP32 Stokes apply, for callers that cannot allocate device memory
 * during the call (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same operator, layouts, outputs and errors as
 * fsi_apply_stokes_f32, but the FP64 pressure staging (the copy of p and the sums of
 * q) lives in a file-scope device array of the library instead of the context's work
 * vectors, and the call allocates nothing (fsi_apply_stokes_f32 allocates every
 * level's work vectors at its first use before fsi_setup).  Limit: levels with at most
 * 4194304 (2^22) pressure nodes; larger levels return FSI_ERR_ARG.  The array (64 MiB)
 * is one per device, shared by every context and call on that device and kept until
 * the process ends; calls that overlap on one device (several streams or threads)
 * race on it.  FSI_ERR_HIP if its device address could not be resolved at
 * fsi_create. */
fsi_status fsi_apply_stokes_f32_noalloc(fsi_ctx* ctx, int level, const float* u, const float* p,
                                        float* v, float* q);

/* Corrector-mode terms (2D and 3D): with the semi-implicit advection of the corrector
 * mode (Sec. 3.1.1: the form a_j with v* the unknown and v° known) and the
 * streamline term of Sec. 3.2, the velocity block becomes
 *   a(u, w) + (rho (grad u) v°, w) + sum_K (r (v° . grad u), (v° . grad w))_K.
 * vconv: device [N_c][Q][dim] FP64, v° at the quadrature points (physical
 * components); r: device [N_c][Q] FP64, the streamline parameter (>= 0, e.g. the
 * Peclet law of Sec. 3.2, constant per cell); rho >= 0 the density.  Cells and
 * points as for fsi_set_coefficients.  Needs the level's geometry; a later
 * geometry change clears the terms (set them again).  Copies on the stream and
 * synchronises.  Errors: FSI_ERR_ARG (bad level or rho), FSI_ERR_STATE
 * (no geometry), FSI_ERR_NONFINITE (non-finite input or r < 0). */
fsi_status fsi_set_convection(fsi_ctx* ctx, int level, const double* vconv, const double* r, double rho);
/* Corrector-mode Stokes apply on one level: v = (A + N + S) u + B^T p, q = B u,
 * with N the convection and S the streamline term set by fsi_set_convection
 * (Dirichlet rows act as identity, Dirichlet columns are zero, as for
 * fsi_apply_stokes).  FP64 and FP32 twin; layouts and errors as fsi_apply_stokes,
 * FSI_ERR_STATE without fsi_set_convection.  The V-cycle and the solve use these
 * terms when fsi_mg_params.corrector = 1. */
fsi_status fsi_apply_corrector(fsi_ctx* ctx, int level, const double* u, const double* p,
                               double* v, double* q);
fsi_status fsi_apply_corrector_f32(fsi_ctx* ctx, int level, const float* u, const float* p,
                                   float* v, float* q);

/* One application of the preconditioner: n V-cycles (Sec. 4) on the finest
 * level from a zero initial guess, in the configured precision.  FP64 in and
 * out; casts are internal.  Requires fsi_setup. */
fsi_status fsi_vcycle(fsi_ctx* ctx, const double* r_u, const double* r_p, double* z_u, double* z_p);

/* Solve the finest-level system with right-preconditioned FGMRES (Sec. 5,
 * linear solver settings).  u, p hold the initial guess on entry and the
 * solution on exit.  The stopping test is ||g - M x||_2/||g||_2 <= rtol on the
 * combined (u,p) vector, confirmed on the true FP64 residual.  Synchronises.
 * Returns FSI_NOT_CONVERGED (results still written) if max_iter is reached. */
fsi_status fsi_solve(fsi_ctx* ctx, const double* g_u, const double* g_p, double* u, double* p,
                     const fsi_solve_opts* opts, fsi_solve_info* info);

/* Extension solve: the pseudo-elastic extension Ext of Sec. 2 (its defining
 * boundary-value problem) on the finest level.  Finds u with u = g on the
 * Dirichlet (wall) nodes and a(u, v) = 0 for every v that vanishes there, where
 * a is the context's A form, (c_m u, v) + (2 eta eps(u), eps(v)): set c_m = 0
 * and eta = mu_A / 2 on every level to get (mu_A eps(u), eps(v)).  Solver (Sec. 5,
 * settings of the extension): flexible CG preconditioned by one multigrid V-cycle
 * on A alone (Chebyshev(A, diag A, k_A) pre- and post-smoothing, the nested-space
 * transfers, a direct solve of the free velocity block of A_0), in the configured
 * precision (FSI_PREC_MIXED: FP32 V-cycle, FP64 CG).
 *   g: device [n_vel] (component-major), only the wall entries are read.
 *   u: device [n_vel]; interior entries are the initial guess on entry; on exit
 *      the extension (wall entries = g).
 *   opts: rtol = ||b - A u_I||_2 / ||b||_2 with b = -A_IW g_W (the residual of the
 *      zero interior guess), confirmed on the true FP64 residual; max_iter;
 *      restart and reorth are not used.
 * The first call after fsi_setup builds the velocity-only coarse inverse.
 * Synchronises.  Errors: FSI_ERR_ARG, FSI_ERR_STATE, FSI_ERR_NONFINITE,
 * FSI_ERR_BREAKDOWN; FSI_NOT_CONVERGED (result still written) at max_iter. */
fsi_status fsi_solve_extension(fsi_ctx* ctx, const double* g, double* u, const fsi_solve_opts* opts,
                               fsi_solve_info* info);

/* Interior Dirichlet nodes for the extension Ext of Sec. 2, which is solved on the
 * fluid part only, with the solid's values on the solid: marks every velocity node of
 * the flagged finest-level cells as constrained, exactly like a wall node (identity
 * row, zero column; fsi_solve_extension then keeps u = g there).  Coarser levels
 * constrain the node at the same position (the flagged region should be a union of
 * coarse cells for the best multigrid; otherwise it stays a valid symmetric
 * preconditioner).  fixed: HOST array of n_cells (finest level), nonzero = fixed.
 * Call once, before fsi_setup.  The single atomic launch (variants 16 ..) keeps the fixed
 * nodes as well: in 3D the A apply then reads a per-node wall mask instead of deriving the
 * wall bits from the box faces (the other 3D classes keep the phased launches on such a
 * context), in 2D every class reads the cell's wall bits.  Errors: FSI_ERR_ARG, FSI_ERR_STATE after fsi_setup or a second
 * call. */
fsi_status fsi_set_fixed_cells(fsi_ctx* ctx, const uint8_t* fixed);
/* Boundary data of the extension: g = v on the nodes of the fixed cells, 0 elsewhere
 * (finest level, device [n_vel] both).  Errors: FSI_ERR_ARG, FSI_ERR_STATE without
 * fsi_set_fixed_cells. */
fsi_status fsi_fixed_values(fsi_ctx* ctx, const double* v, double* g);

/* One step of the GCSI_k(M_1, .., M_S) scheme (Algorithm 1, Sec. 3.1.1) is composed by
 * the caller from: fsi_gcsi_displacement (explicit step, new geometry through
 * fsi_set_displacement), fsi_gcsi_set_coefficients, fsi_gcsi_set_convection (corrector
 * stage), fsi_setup, fsi_gcsi_rhs, fsi_solve, then fsi_fixed_values and
 * fsi_solve_extension on a second context (every face fixed, the solid's cells fixed,
 * reference geometry, c_m = 0, eta = mu_A / 2), and fsi_gcsi_displacement once more for
 * the displacement recovery.  Fields are finest-level nodal arrays of the reference
 * mesh (the pull-backs u^{n,i} of Sec. 3.1 have the stored nodal values), device FP64,
 * component-major [dim][n_vel_nodes]; 2D and 3D contexts.
 * Physical data: BDF order k (Sec. 3.1: k = 1 gamma = 1, alpha_1 = -1; k = 2
 * gamma = 2/3, alpha_1 = -4/3, alpha_2 = 1/3), time step tau, densities, fluid
 * viscosity eta_f, solid shear modulus mu_s (solid viscosity gamma tau mu_s, Sec. 3.1.1),
 * volume-correction parameter eta_V (Sec. 3.1.2; <= 0 or infinite: none) and the body
 * acceleration (force density rho * body). */
typedef struct {
    int k;
    double tau;
    double rho_f, rho_s;
    double eta_f, mu_s;
    double eta_V;
    double body[3];
} fsi_gcsi_params;

#define FSI_GCSI_PREDICTOR 0
#define FSI_GCSI_CORRECTOR 1

/* Velocity splitting (Sec. 3.1.1): u_out = gamma tau w - sum_i alpha_i u_i (the
 * explicit displacement u# from w#, and the displacement recovery from w^n), and, if
 * disp_out is not NULL, its vertex values [dim][n_vert] for fsi_set_displacement (the
 * multilinear map through the vertex values of the Q2 field).  u2 is read for k = 2
 * only.  Either output may be NULL.  Errors: FSI_ERR_ARG. */
fsi_status fsi_gcsi_displacement(fsi_ctx* ctx, const fsi_gcsi_params* prm, const double* w, const double* u1,
                                 const double* u2, double* u_out, double* disp_out);
/* Coefficients of the stress splitting on every level, c_m = rho / (gamma tau) and
 * eta = eta_f (fluid) or gamma tau mu_s (solid), then as fsi_set_coefficients.
 * solid_q: HOST array of n_levels DEVICE pointers, each [n_cells][3^dim] uint8 of that
 * level (nonzero: the point lies in the solid).  Call after every geometry change.
 * Errors: as fsi_set_coefficients. */
fsi_status fsi_gcsi_set_coefficients(fsi_ctx* ctx, const fsi_gcsi_params* prm, const uint8_t* const* solid_q);
/* Right-hand side of the M-mode system on the finest level (eq. form_g_j, eq. form_g_p),
 * on the explicit geometry given by its vertex displacement disp ([dim][n_vert]):
 *   g_u(v) = (rho (body - (1/(gamma tau)) sum_i alpha_i v_i), v)
 *            - [predictor] (rho (grad v*) v°, v)        v* = 2 v1 - v2,
 *                                                       v° = 2 (v1 - w1) - (v2 - w2)
 *                                                       (k = 1: v1 and v1 - w1)
 *            + (mu_s [2 eps(sum_i alpha_i u_i) + (grad u#)^T grad u#], eps(v))_solid
 *   g_p(q) = -(1/eta_V) (det(I + grad-hat u#) - 1, q-hat)_{reference solid}
 * (readings: the explicit solid stress as the velocity splitting substituted into the
 * solid stress of Sec. 2.3, sign -2 eps(..) where the paper prints +; v° extrapolates
 * the relative velocity, with w2 in its second term where the paper prints w1; the
 * predictor's convective term explicit as a whole).  solid_q: DEVICE [n_cells][3^dim]
 * uint8 of the finest level; body[2] is not read in 2D.  Dirichlet rows of g_u are zero.  Sums with atomics (the
 * last bits vary from run to run).  u2, v2, w2 are read for k = 2, w1 and w2 in the
 * predictor mode only.  Errors: FSI_ERR_ARG. */
fsi_status fsi_gcsi_rhs(fsi_ctx* ctx, const fsi_gcsi_params* prm, int mode, const uint8_t* solid_q,
                        const double* disp, const double* u_hash, const double* u1, const double* u2,
                        const double* v1, const double* v2, const double* w1, const double* w2, double* g_u,
                        double* g_p);
/* Corrector-mode terms on every level (as fsi_set_convection, rho = rho_f): v° = v# - w#
 * at the Gauss points (the fine fields read at each level's nodes) and the streamline
 * parameter of Sec. 3.2 per cell (p1 = 2, h_K the reference cell diagonal, |v°| the
 * largest point value, eta the cell mean of the last fsi_gcsi_set_coefficients):
 * Pe = |v°| h_K / (2 eta p1), r = h_K / (2 |v°| p1) (coth Pe - 1/Pe) for Pe >= 1, else 0.
 * rho_f suffices: v° vanishes on every node of a solid cell (w# = v# there).  Errors:
 * FSI_ERR_ARG, FSI_ERR_STATE without fsi_gcsi_set_coefficients or geometry. */
fsi_status fsi_gcsi_set_convection(fsi_ctx* ctx, const fsi_gcsi_params* prm, const double* v_hash,
                                   const double* w_hash);

/* Nonzero Dirichlet velocity data (an inflow profile, Sec. 5 test problems) for fsi_solve:
 * with d the data on the Dirichlet nodes of the finest level (other entries are not read),
 * the free rows of g_u lose the constrained columns applied to d, the Dirichlet rows of g_u
 * take d, and g_p loses B's constrained columns applied to d:
 *   g_u <- g_u - (M_u d_W) on free rows, g_u <- d on Dirichlet rows, g_p <- g_p - B d_W,
 * with M_u the velocity block in the configured mode (A, or A + N + S with corrector = 1).
 * Then the solve's Dirichlet rows (identity) take the data and its free rows are the
 * unconstrained equations.  d, g_u: device [n_vel]; g_p: device [n_p]; updated in place.
 * Requires the finest level's geometry and coefficients (and fsi_set_convection in the
 * corrector mode).  Errors: FSI_ERR_ARG, FSI_ERR_STATE, FSI_ERR_NONFINITE (d not finite on
 * the Dirichlet nodes; synchronises). */
fsi_status fsi_lift_dirichlet(fsi_ctx* ctx, const double* d, double* g_u, double* g_p);

/* Autotuner: times the cell-kernel launch variants (wavefronts per workgroup,
 * register cap, cached or streaming geometry loads) for every operator class
 * (A, A with the fused Chebyshev step, Stokes, Stokes with the fused residual,
 * B, B^T), level and precision, and keeps the fastest of each; then, per level,
 * the phased launches of the unfused applies against their single atomic launch
 * (variants 16 .. 22 below on 3D levels, 16 and 17 on 2D levels), on levels where the corrector terms are set
 * (fsi_set_convection) the same choice for the corrector classes (A + N + S alone and in
 * the Stokes apply), and the fused epilogues against the separate vector kernels.  Synchronises; fsi_get_tuning reports the choice for A (16 .. 22 where the
 * atomic launch was chosen) and its measured time per application in best_us. */
fsi_status fsi_autotune(fsi_ctx* ctx);
fsi_status fsi_get_tuning(const fsi_ctx* ctx, int level, int precision, int* variant, double* best_us);
/* Pin the launch variant (0 .. 15) of every operator class on one level and
 * precision, overriding the autotuner (used with tuned = 1).  Variant v < 12: v % 3
 * selects 1, 2 or 4 wavefronts per workgroup sharing a row of cells (3D; 2D: one row
 * per wavefront, at most two); (v / 3) % 2 cached instead of streaming geometry
 * loads; v / 6 a register cap of one more wavefront per SIMD.  v = 12 .. 15: three
 * wavefronts share a row (2D: two rows), (v - 12) % 2 cached loads, (v - 12) / 2 the
 * register cap.  v = 16 .. 22 on 3D levels, 16 and 17 on 2D levels: the unfused applies
 * (A, B, B^T, Stokes, and the corrector classes) run as one launch over all processing
 * phases that adds into zeroed outputs with atomics and writes the wall rows itself.
 * 3D: one (16) or four (17) wavefronts per row, one wavefront over two (18) or four (19)
 * rows along z, four wavefronts over two rows along z (20), where the node plane two rows
 * of a group share is summed in registers and stored once, one wavefront per half (21) or
 * quarter (22) row, where the x-face node two segments share takes atomics from both.  2D: one wavefront per row
 * segment, one (16) or two (17) per workgroup.  Results then vary in the last bits from
 * run to run; the fused epilogues keep variant 0.  fsi_autotune picks this form for a level where it
 * measures it faster.  Errors: FSI_ERR_ARG. */
fsi_status fsi_set_tuning(fsi_ctx* ctx, int level, int precision, int variant);

/* Measurement support: runs `reps` applications of the level operator
 * (mode bits 1 = A, 2 = B^T, 4 = B; 7 = fused Stokes; 9 = A with the fused
 * Chebyshev epilogue, run with zero coefficients; 23 = Stokes with the fused
 * residual epilogue; 33 = A and 39 = Stokes with the corrector terms, after
 * fsi_set_convection) in the given precision on
 * internal work vectors, timing every launch of the cell kernel with HIP events
 * on the context's stream, after three untimed warm-up applications.
 * kernel_us = cell-kernel time of one application (sum over its n_launches
 * launches, one per processing phase; with tuned = 1 on a level where the
 * autotuner chose the single atomic launch, that one launch with the zeroing of
 * its outputs, n_launches = 1), op_us = duration of the whole application
 * (including the wall rows); both are medians over the `reps` timed
 * applications.  Synchronises.  Errors: FSI_ERR_ARG, FSI_ERR_STATE. */
fsi_status fsi_time_operator(fsi_ctx* ctx, int level, int precision, int mode, int reps,
                             double* kernel_us, double* op_us, int* n_launches);

#ifdef __cplusplus
}
#endif
#endif /* FSI_H */
