/*
 * fo_stokes.h -- C ABI of the MI355X (gfx950) first-order Stokes assembly library.
 *
 * The library evaluates, on one GPU, the finite-element residual F(U) and the
 * Newton Jacobian J = dF/dU of the first-order (Blatter-Pattyn) Stokes
 * equations for ice flow (arXiv:2204.04321, Sec. 2, eqs. FOStokes, effvisc,
 * effeps and the bed sliding condition; discrete form eq. residual of Sec. 3.1)
 * on meshes extruded from a 2D triangulation (wedges) or quadrilateral mesh
 * (hexahedra), and solves F(U) = 0 by damped Newton (eq. linearsystem).
 *
 * Conventions (all entry points):
 *   - Ordering.  Base vertex v (a "column") at level k (k = 0 at the bed,
 *     k = L at the surface) is node v*(L+1)+k; dof 2*node+c, c = 0 for u
 *     (x-velocity) and c = 1 for v (y-velocity).  Node elevation
 *     z = (s - H) + sigma_k H.  Units: m, yr, Pa.
 *   - Jacobian storage.  CSR with one row per dof; a row holds every dof that
 *     shares a cell with the row's node (structural zeros included), columns
 *     sorted ascending.  rowptr is int64 [n_dofs + 1], colidx int32 [nnz].
 *   - Memory.  Pointers named *_dev are device pointers owned by the caller
 *     (e.g. PyTorch tensors on the current HIP device).  Host arrays in
 *     fo_mesh_desc are read only during fo_mesh_create.  The opaque fo_mesh
 *     owns its device tables (connectivity, geometry, pattern) until
 *     fo_mesh_destroy.
 *   - Streams.  `stream` is a hipStream_t (NULL = default stream).  Assembly
 *     calls are asynchronous and stream-ordered; fo_mesh_create and
 *     fo_newton_solve synchronise the stream before returning.
 *   - Errors.  Every call returns an fo_status; on failure fo_last_error()
 *     gives a message (thread-local).  Kernel launch failures give FO_EDEVICE.
 */
#ifndef FO_STOKES_H
#define FO_STOKES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FO_OK = 0,
  FO_EINVAL = -1,        /* bad argument: null pointer, size, enum value */
  FO_ENOMEM = -2,        /* device or host allocation failed */
  FO_EDEVICE = -3,       /* HIP runtime or kernel launch error */
  FO_EDEGENERATE = -4,   /* mesh invalid: H <= 0, non-positive cell area, bad sigma */
  FO_ENONFINITE = -5,    /* NaN/Inf met in a residual norm (Newton) */
  FO_ENOTCONV = -6       /* Newton hit its iteration cap or the line search failed */
} fo_status;

/* Base triangles extruded to prisms (FO_WEDGE6) or to three tetrahedra per prism (FO_TET4: the
 * element of the paper's nightly test, Sec. 5.3; the split follows the global order of each
 * triangle's vertices, p0 < p1 < p2: (p0,p1,p2,p0'), (p1,p2,p0',p1'), (p2,p0',p1',p2') with
 * primes one level up, linear basis, exact integrals); base quads extruded to hexahedra
 * (FO_HEX8).  With FO_TET4 the Jacobian keeps the prism's pattern: node pairs of a prism
 * that share no tetrahedron are structural zeros. */
typedef enum { FO_TET4 = 4, FO_WEDGE6 = 6, FO_HEX8 = 8 } fo_elem;
typedef enum { FO_F64 = 0, FO_F32 = 1 } fo_dtype;         /* Jacobian value type */
typedef enum { FO_JAC_NEWTON = 0, FO_JAC_PICARD = 1 } fo_jac_kind;

/* Mesh and physical constants (Sec. 2: A, n, rho, g; beta of the sliding law). */
typedef struct {
  int32_t elem;              /* FO_WEDGE6, FO_TET4 or FO_HEX8 */
  int32_t n_base_verts;      /* V >= 3 */
  int32_t n_base_cells;      /* T >= 1 */
  int32_t n_layers;          /* L >= 1 */
  const double *base_xy;     /* host [V][2], m */
  const int32_t *base_cells; /* host [T][3 or 4 (FO_HEX8)], counter-clockwise, 0 <= id < V */
  const double *surface;     /* host [V], s (m) */
  const double *thickness;   /* host [V], H > 0 (m) */
  const double *beta;        /* host [V], beta >= 0 (Pa yr / m) */
  const double *sigma;       /* host [L+1], 0 = sigma_0 < ... < sigma_L = 1; NULL = uniform */
  double A;                  /* rate factor > 0, Pa^-n yr^-1 */
  double n;                  /* Glen exponent >= 1 */
  double rho;                /* ice density > 0, kg m^-3 */
  double g;                  /* gravity > 0, m s^-2 */
  double eps0;               /* strain-rate regularisation >= 0, yr^-1 */
  /* Ocean fronts (Sec. 2, lateral boundary condition on the marine margin), optional:
   * n_front_edges base-mesh boundary edges (vertex pairs, either order) whose vertical
   * faces take the ocean back-pressure, read as 2 mu eps_i . n - rho g (s - z) n_i =
   * -rho_w g max(-z, 0) n_i with sea level at z = 0 (the printed max(z, 0) and its sign are
   * garbled); the residual gains -int phi p n_i dA, p = rho g (s - z) - rho_w g max(-z, 0),
   * a load that does not depend on U (the Jacobian is unchanged).  All other lateral faces
   * stay natural.  Floating ice is described by beta = 0 where it floats. */
  const int32_t *front_edges;/* host [n_front_edges][2], or NULL */
  int32_t n_front_edges;     /* >= 0; 0 = no fronts */
  double rho_w;              /* sea-water density > 0 (kg m^-3) when n_front_edges > 0 */
} fo_mesh_desc;

typedef struct fo_mesh fo_mesh;

/* Validate the description, build the column-major numbering, the Jacobian
 * pattern and per-column tables once (the paper's memoisation of
 * solution-independent data, Sec. 4.1) and upload them.  FO_EDEGENERATE also
 * if a base vertex lies in no base cell.  On FO_EDEGENERATE nothing is
 * allocated.  FO_EINVAL also if a base vertex lies in more than 64
 * base cells or has more than 90 neighbouring base vertices, itself included (one wave assembles
 * a vertex column's rows in its share of the compute unit's LDS), or if a front edge is
 * not a boundary edge of the base mesh, appears twice, or a vertex lies on more than four
 * front edges.  The front loads are integrated once here (memoised with the rest).
 * Synchronises `stream`. */
fo_status fo_mesh_create(const fo_mesh_desc *desc, void *stream, fo_mesh **out);
void fo_mesh_destroy(fo_mesh *mesh);

/* Sizes: nodes V*(L+1), dofs 2*nodes, cells T*L, Jacobian nonzeros.  Any output may be NULL. */
fo_status fo_mesh_info(const fo_mesh *mesh, int64_t *n_nodes, int64_t *n_dofs,
                       int64_t *n_cells, int64_t *nnz);

/* Copy the Jacobian pattern into caller buffers rowptr_dev [n_dofs+1] (int64)
 * and colidx_dev [nnz] (int32).  Either may be NULL. */
fo_status fo_jacobian_pattern(const fo_mesh *mesh, int64_t *rowptr_dev, int32_t *colidx_dev,
                              void *stream);

/* Residual F(U) of eq. (residual): viscous term with the regularised Glen
 * viscosity 1/2 A^(-1/n) (eps_e^2 + eps0^2)^((1-n)/(2n)) (eqs. effvisc,
 * effeps), gravity rho g grad s, and bed friction beta u.  U_dev, R_dev: FP64
 * [n_dofs]; R is overwritten. */
fo_status fo_assemble_residual(const fo_mesh *mesh, const double *U_dev, double *R_dev,
                               void *stream);

/* Jacobian J = dF/dU (eq. linearsystem) in forward mode over the element dofs (Sec. 3.2):
 * the tangent of each element residual row along every element dof, pushed through strain
 * rate -> eps_e^2 -> mu -> residual by derivative rules written out in the kernel (not an
 * operator-overloading AD type); values written into Jvals_dev [nnz] of type `dtype` (FO_F64: double,
 * FO_F32: float; with FO_F32 the per-cell derivatives are computed in FP32 over
 * an FP64 primal evaluation, summed over cells in FP64 and rounded once).  kind = FO_JAC_PICARD drops the viscosity-derivative
 * term.  If R_dev is not NULL the FP64 residual is written too, from the same
 * pass.  Jvals and R are overwritten.  Any Glen exponent n >= 1, for either element;
 * n = 3 takes a dedicated viscosity evaluation that agrees with the general power
 * law to rounding. */
fo_status fo_assemble_jacobian(const fo_mesh *mesh, const double *U_dev, double *R_dev,
                               void *Jvals_dev, int32_t dtype, int32_t kind, void *stream);

/* Shallow-ice velocity profile (plain Newton initial guess, not part of the
 * paper): U = u_b - 2A/(n+1) (rho g)^n |grad s|^(n-1) grad s [H^(n+1) - (s-z)^(n+1)]
 * with u_b = -rho g H grad s / beta capped at 1e4 m/yr; grad s at a vertex is
 * the area-weighted mean of the adjacent base cells' gradients.  U_dev [n_dofs]. */
fo_status fo_initial_guess_sia(const fo_mesh *mesh, double *U_dev, void *stream);

/* ---- Newton solve (eq. linearsystem: J(U_k) delta = -F(U_k), U_{k+1} = U_k + alpha_k delta) ---- */
typedef enum { FO_INIT_USER = 0, FO_INIT_SIA = 1, FO_INIT_LEARNED = 2 } fo_init;
/* Linear solver of each Newton step.  FO_LIN_GMRES is the method (GMRES, Sec. 3.1).
 * FO_LIN_PCG, an option beyond the paper, runs preconditioned conjugate gradients: the
 * Newton Jacobian is the Hessian of a convex energy and the column block preconditioner is
 * symmetric positive definite in exact arithmetic, so CG applies with a few vectors per
 * iteration instead of the growing Krylov basis.  In floating point the operators are only
 * nearly symmetric: the column factors are stored in FP32 (M^-1 symmetric to about 1e-7
 * relative) and so are the Jacobian values with jac_dtype = FO_F32.  Should a search
 * direction show non-positive curvature, the solve stops with FO_ENOTCONV (GMRES has no such
 * requirement). */
typedef enum { FO_LIN_GMRES = 0, FO_LIN_PCG = 1 } fo_linear_solver;

/* Preconditioner of each Newton step's linear system.  FO_PREC_COLUMN: block LU of each vertical
 * column (block Jacobi over columns).  FO_PREC_MDSC: the two-level column semicoarsening
 * preconditioner of a fo_mdsc object (see fo_mdsc_create), GMRES only. */
typedef enum { FO_PREC_COLUMN = 0, FO_PREC_MDSC = 1 } fo_preconditioner;
typedef struct fo_mdsc fo_mdsc;

typedef struct {
  double tol;              /* stop when ||F(U)||_2 <= tol ||F(0)||_2 (default 1e-8) */
  int32_t max_newton;      /* Newton iteration cap (50) */
  double lin_rtol;         /* GMRES relative residual tolerance (1e-6) */
  int32_t gmres_restart;   /* GMRES restart length, 1..500 (100) */
  int32_t max_lin;         /* GMRES iterations per Newton step (500) */
  int32_t jac_dtype;       /* FO_F64 or FO_F32 Jacobian values for GMRES and preconditioner */
  int32_t max_backtracks;  /* line-search halvings of alpha (10) */
  int32_t init;            /* FO_INIT_USER: U_dev holds the guess; FO_INIT_SIA: shallow-ice guess;
                              FO_INIT_LEARNED: fo_initial_guess_learned with the fields below */
  int32_t linear_solver;   /* fo_linear_solver (FO_LIN_GMRES); lin_rtol and max_lin apply to both */
  const float *mlp_params; /* FO_INIT_LEARNED: device [fo_mlp_param_count()] network parameters */
  const float *mlp_norm;   /* FO_INIT_LEARNED: device [20] feature means then standard deviations */
  int32_t learned_fallback;/* FO_INIT_LEARNED: fallback rule of fo_initial_guess_learned (1) */
  int32_t learned_smooth;  /* FO_INIT_LEARNED: smoothing sweeps of fo_initial_guess_learned (0) */
  int32_t preconditioner;  /* fo_preconditioner (FO_PREC_COLUMN) */
  fo_mdsc *mdsc;           /* FO_PREC_MDSC: a preconditioner object created on this mesh; each Newton
                              step runs fo_mdsc_setup on its Jacobian, so its previous numeric
                              state is overwritten */
} fo_newton_opts;

typedef struct {
  int32_t status;          /* fo_status of the solve */
  int32_t newton_its;
  int64_t lin_its;         /* linear-solver iterations (GMRES or CG) summed over Newton steps */
  int32_t residual_calls;  /* residual-only assemblies (line search, norms) */
  int32_t jacobian_calls;  /* residual + Jacobian assemblies */
  int32_t backtracks;
  double f0_norm;          /* ||F(0)||_2 */
  double final_norm;       /* ||F(U)||_2 at return */
  double final_rel;        /* final_norm / f0_norm */
  double ms_total_fill;    /* timers named as in the paper's Sec. 5 tables */
  double ms_prec_construction;
  double ms_linear_solve;
  double ms_total_solve;
  double res_hist[64];     /* ||F||/||F(0)|| before each Newton step (first 64) */
  int32_t init_used;       /* fo_init whose guess the solve started from (FO_INIT_LEARNED falls
                              back to FO_INIT_SIA when the network's guess is rejected) */
  int32_t learned_fallbacks; /* 1 if FO_INIT_LEARNED was asked for and its guess was rejected */
} fo_newton_report;

void fo_newton_default_opts(fo_newton_opts *opts);

/* Device workspace needed by fo_newton_solve for these options (0 on bad options):
 * Jacobian values, GMRES basis (restart+1 vectors; with FO_INIT_LEARNED at least the
 * learned guess's workspace, which shares that region before the first Krylov step),
 * column factors, vectors. */
size_t fo_newton_workspace_bytes(const fo_mesh *mesh, const fo_newton_opts *opts);

/* Damped Newton with GMRES(restart) right-preconditioned by block LU of each vertical
 * column's 2(L+1) x 2(L+1) block (block-tridiagonal, no pivoting; or, with FO_PREC_MDSC,
 * the two-level preconditioner built on those column factors) and a backtracking
 * line search (alpha = 1, 1/2, ... accepting a decrease by (1 - 1e-4 alpha)).  U_dev
 * [n_dofs] holds the initial guess (unless init = FO_INIT_SIA) and returns the last
 * accepted iterate.  workspace_dev: caller-owned device memory, 256-byte aligned, at
 * least fo_newton_workspace_bytes.  Returns FO_OK on convergence, FO_ENOTCONV (cap or
 * line search), FO_ENONFINITE; the report is filled in every case.  Synchronises. */
fo_status fo_newton_solve(const fo_mesh *mesh, double *U_dev, const fo_newton_opts *opts,
                          fo_newton_report *report, void *workspace_dev, size_t workspace_bytes,
                          void *stream);

/* ---- Two-level column semicoarsening preconditioner (Sec. 3.3, Sec. 4.4) ---------------------
 * The paper preconditions GMRES by multigrid that coarsens the extruded mesh vertically with
 * a matrix-dependent prolongator, built per vertical line from that line's block-tridiagonal
 * system solved by LU without pivoting, down to one layer, and then runs aggregation AMG on
 * the plane with Chebyshev smoothing.  This object implements that design in two levels:
 *   smoother B:   block LU (no pivoting, FP64 recursion, FP32 factors) of every vertex
 *                 column's block-tridiagonal 2(L+1) x 2(L+1) block;
 *   collapse P0:  per column v and component c the weights w = B_v^-1 e_c (e_c: 1 at
 *                 component c of every level), FP64, scaled so the mean of the component-c
 *                 entries is 1 (e_c itself where that mean is not a positive finite number);
 *   plane:        A_0 = P0^T J P0, 2 dofs per base vertex on the base-mesh graph (vertices
 *                 that share a base cell), aggregated level by level until at most 64
 *                 vertices remain (pass 1 in index order: a vertex whose neighbours are all
 *                 unassigned roots an aggregate of itself and its neighbours, isolated
 *                 vertices are grouped 8 at a time; pass 2: every vertex left joins the
 *                 aggregate of its lowest-numbered neighbour assigned in pass 1), unsmoothed
 *                 transfers, Galerkin operators, Chebyshev over [g/30, g] on D^-1 A (D: 2x2
 *                 diagonal blocks, g: the Gershgorin bound max row sum of |D^-1 A|) before
 *                 and after the coarse correction, degree 2 on the first plane level and 1
 *                 below it, the coarsest level solved by its inverse (Gauss-Jordan with
 *                 partial pivoting);
 *   application:  y = V-cycle(P0^T r), z = P0 y + B^-1 (r - J P0 y), with J P0 and the weights
 *                 of P0 and P0^T stored in FP32 (the plane operators are formed from the FP64
 *                 values; any stored precision leaves M a fixed linear operator).
 * All device memory is allocated by fo_mdsc_create and owned by the object; the mesh must
 * outlive it.  Calls on one object must not overlap. */

/* Host-side aggregation of a graph: n vertices, sorted neighbour lists ptr [n+1], idx
 * (each containing the vertex itself), into agg [n] (host) and *n_agg, by the two passes
 * above.  Pure host code, no device needed.  FO_EINVAL on a malformed graph. */
fo_status fo_mdsc_aggregate_graph(int32_t n, const int32_t *ptr, const int32_t *idx, int32_t *agg,
                                  int32_t *n_agg);

/* Build the hierarchy's graphs, aggregates and transfer tables for a mesh (host work plus
 * device allocations: about (L+1)(2 nnz_plane + 15 V) doubles, nnz_plane the number of
 * ordered base-vertex pairs that share a cell, self pairs included).  The mesh's device must
 * be current.  Synchronises `stream`. */
fo_status fo_mdsc_create(const fo_mesh *mesh, void *stream, fo_mdsc **out);
void fo_mdsc_destroy(fo_mdsc *p);

/* Plane levels: *n_levels smoothed levels plus the coarsest; n_verts (may be NULL) receives
 * n_levels + 1 vertex counts, level 0 being the base mesh. */
fo_status fo_mdsc_levels(const fo_mdsc *p, int32_t *n_levels, int32_t *n_verts);

/* Host copies of level `level`'s graph (ptr [n+1], idx [ptr[n]]; either may be NULL) and, for
 * a smoothed level, of its aggregate map agg [n] (may be NULL; FO_EINVAL on the coarsest). */
fo_status fo_mdsc_graph(const fo_mdsc *p, int32_t level, int32_t *ptr, int32_t *idx, int32_t *agg);

/* Numeric setup from a Jacobian J_dev [nnz] of `jac_dtype` (FO_F64 or FO_F32), in the
 * library's Jacobian layout: column factors, weights, J P0, the plane operators, their
 * diagonal inverses and bounds, and the coarsest inverse.  Synchronises `stream` (one
 * status read); FO_ENONFINITE if a diagonal block or the coarsest operator is singular or
 * not finite. */
fo_status fo_mdsc_setup(fo_mdsc *p, const void *J_dev, int32_t jac_dtype, void *stream);

/* z_dev = M^-1 r_dev (FP64 [n_dofs] each, distinct, 16-byte aligned) after fo_mdsc_setup.
 * A fixed linear operator (right preconditioning); asynchronous on `stream`. */
fo_status fo_mdsc_apply(const fo_mdsc *p, const double *r_dev, double *z_dev, void *stream);

/* Copy the numeric setup of the last successful fo_mdsc_setup to the host (FO_EINVAL before
 * one): what = FO_MDSC_WEIGHTS (level ignored): the weights
 * [V][L+1][2 c'][2 c] (count V (L+1) 4); FO_MDSC_PLANE: level `level`'s block values in its
 * graph order, block [2 c + d] (count 4 ptr[n]); FO_MDSC_BOUND: the Gershgorin bound of a
 * smoothed level (count 1).  Synchronises `stream`. */
typedef enum { FO_MDSC_WEIGHTS = 0, FO_MDSC_PLANE = 1, FO_MDSC_BOUND = 2 } fo_mdsc_field;
fo_status fo_mdsc_export(const fo_mdsc *p, int32_t what, int32_t level, double *host, size_t count,
                         void *stream);

/* ---- Batched ensembles (many meshes, one persistent launch) ---------------------------- */
typedef struct fo_ensemble fo_ensemble;

/* Group already-created meshes of one element type (their sizes, beta, A, n may differ).
 * The members must outlive the ensemble; nothing is copied from them but their task tables. */
fo_status fo_ensemble_create(const fo_mesh *const *members, int32_t n_members, void *stream,
                             fo_ensemble **out);
void fo_ensemble_destroy(fo_ensemble *ens);

/* Assemble every member in ONE persistent kernel launch: workgroups take (member, vertex-run)
 * items from a device counter until all are done.  U_dev, R_dev, J_dev are host arrays of
 * n_members device pointers laid out as for fo_assemble_jacobian (R_dev may be NULL, or hold
 * NULL entries, to skip residuals).  J_dev == NULL assembles residuals only (R_dev required).
 * Each member's result equals its own fo_assemble_jacobian / fo_assemble_residual bit
 * for bit when every member has n = 3 or none has; in a mixed ensemble all members take
 * the general power law, which agrees with the n = 3 evaluation to rounding. */
fo_status fo_ensemble_assemble(fo_ensemble *ens, const double *const *U_dev, double *const *R_dev,
                               void *const *J_dev, int32_t dtype, int32_t kind, void *stream);

/* ---- Learned Newton initial guess (not in the paper; feeds eq. linearsystem's first iterate) ----
 * Network 10 -> 128 -> 128 -> 128 -> 22 (tanh hidden layers), parameters as one FP32 vector:
 * for each layer W [out][in] then b [out].  Products use BF16 copies (round to nearest even)
 * of inputs, weights, hidden activations and backpropagated errors on the BF16 matrix cores
 * with FP32 sums.  All buffers are device pointers owned by the caller. */
int32_t fo_mlp_param_count(void);

/* Column features [V][10]: H, ds/dx, ds/dy (area-weighted vertex gradient), log(max(beta,
 * 1e-3)), and H of the 6 nearest base neighbours ordered by angle from -grad s (own H pads).
 * norm: NULL for raw values, else [20] = 10 means then 10 standard deviations. */
fo_status fo_column_features(const fo_mesh *mesh, const float *norm_dev, float *feat_dev, void *stream);

/* Y [B][22] from normalised inputs X [B][10]; acts [3][B][128] receives the FP32 hidden
 * activations that fo_mlp_backward needs. */
fo_status fo_mlp_forward(const float *params_dev, const float *X_dev, int32_t B, float *acts_dev,
                         float *Y_dev, void *stream);

/* Gradients of a loss with dL/dY = dY [B][22] into grads [param_count]; dacts is scratch
 * [2][B][128]. */
fo_status fo_mlp_backward(const float *params_dev, const float *X_dev, int32_t B, const float *acts_dev,
                          const float *dY_dev, float *dacts_dev, float *grads_dev, void *stream);

/* dY = 2 (Y - T) / n (mean squared error over n values); loss_dev (may be NULL) += the loss. */
fo_status fo_mse_grad(const float *Y_dev, const float *T_dev, int64_t n, float *dY_dev, double *loss_dev,
                      void *stream);

/* One Adam step (bias-corrected, step >= 1) on n FP32 parameters with moments m, v. */
fo_status fo_adam_step(float *params_dev, const float *grads_dev, float *m_dev, float *v_dev, int32_t n,
                       float lr, float beta1, float beta2, float eps, int32_t step, void *stream);

/* Training targets T [V][22] (FP32) from a converged solution U_dev and the shallow-ice guess
 * U_sia_dev of the same mesh (both FP64 [n_dofs], L must be 10): the correction of the
 * shallow-ice profile in the network's output scale, T = asinh((U - U_sia) / 10 m/yr), in
 * dof order (a column's 22 dofs are contiguous). */
fo_status fo_learned_targets(const fo_mesh *mesh, const double *U_dev, const double *U_sia_dev, float *T_dev,
                             void *stream);

/* Feature normalisation norm_dev [20] (FP32) from raw features X_dev [n_rows][10]: the 10
 * column means, then the 10 standard deviations (n - 1 in the denominator, n_rows >= 2)
 * plus 1e-6.  Sums in FP64, one pass per moment, deterministic.  If Xn_dev is not NULL it
 * receives the normalised features (X - mean) / std [n_rows][10], as fo_column_features
 * computes them from the same norm. */
fo_status fo_feature_stats(const float *X_dev, int64_t n_rows, float *norm_dev, float *Xn_dev, void *stream);

/* Initial velocity U = U_sia + D, D the network's correction 10 sinh(Y) (Y: its column
 * outputs, L must be 10) after `smooth_sweeps` >= 0 Jacobi sweeps over the base mesh,
 * D_v <- (D_v + mean of D over v's base-mesh neighbours) / 2 (per dof of the column; the
 * network predicts each column alone).  Replaced by the shallow-ice guess U_sia if any
 * value is non-finite, or, with fallback = 1, if ||F(U)|| > ||F(U_sia)|| (fallback = 0:
 * non-finite values only).  *used_network (host) tells which one was kept.  Workspace:
 * fo_learned_workspace_bytes, 256-byte aligned.  Synchronises. */
size_t fo_learned_workspace_bytes(const fo_mesh *mesh);
fo_status fo_initial_guess_learned(const fo_mesh *mesh, const float *params_dev, const float *norm_dev,
                                   double *U_dev, int32_t fallback, int32_t smooth_sweeps, void *workspace_dev,
                                   size_t workspace_bytes, int32_t *used_network, void *stream);

/* fo_initial_guess_learned for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid hipMalloc): the same computation and
 * result, with no workspace argument and no allocation.  Its workspace is a library-owned
 * device array of FO_LEARNED_SCRATCH_BYTES on each GPU it runs on, held until the process
 * ends; a mesh whose fo_learned_workspace_bytes exceeds it (about 14,000 base vertices) is
 * rejected with FO_EINVAL before any device work.  The mesh's device must be current.  All
 * calls on one GPU share that array and every call rewrites what it reads: calls that overlap
 * on one GPU (other streams or threads) race, and the caller must serialise them.
 * Synchronises. */
#define FO_LEARNED_SCRATCH_BYTES ((size_t)32 << 20)
fo_status fo_initial_guess_learned_noalloc(const fo_mesh *mesh, const float *params_dev, const float *norm_dev,
                                           double *U_dev, int32_t fallback, int32_t smooth_sweeps,
                                           int32_t *used_network, void *stream);

/* Measurement support: while enabled, every assembly call records HIP events on
 * its stream around its main assembly kernel (not the zero fills).
 * fo_profile_read synchronises on the last event, returns the summed kernel
 * time in milliseconds and the launch count since the last read, and resets
 * both.  Enabling allocates a few events; disabling releases them. */
fo_status fo_profile_enable(fo_mesh *mesh, int32_t on);
fo_status fo_profile_read(fo_mesh *mesh, double *kernel_ms, int64_t *launches);

const char *fo_status_string(fo_status s);
const char *fo_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FO_STOKES_H */
