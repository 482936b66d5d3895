/*
 * mpm.h -- C ABI of the MI355X (gfx950) implicit-MPM hot path.
 *
 * The library evaluates, for one load step of the implicit material point
 * method of arXiv 2507.09435 ("GeoWarp"):
 *   - the residual r = A_p (f_int,p - f_ext,p)            (Sec. 2.2, the
 *     discrete weak form and the backward-Euler residual equation),
 *   - the Jacobian J = dr/du as a block-sparse matrix built from per-particle
 *     local blocks over the 3^d stencil nodes            (Sec. 3.2, the
 *     localized sparse Jacobian; Table 1: quadratic B-splines, w = 3, so at
 *     most 5^d coupled nodes per node),
 *   - the Newton iteration -J du = r until ||r_k||/||r_0|| <= tol (Sec. 2.2)
 *     with a Krylov solve on the GPU in place of the paper's CPU solvers
 *     (Remark 2),
 *   - one adjoint step: a transposed solve at the converged state and the
 *     particle-wise backpropagation to state and material parameters (the
 *     gradient the paper takes from its tape over the whole run, Sec. 4.5).
 *
 * Conventions shared by every entry point
 *   * All array pointers are DEVICE pointers (memory of the device given to
 *     mpm_create), owned by the caller, unless a comment says "host".  The
 *     library never frees caller memory.
 *   * Calls are asynchronous on the stream given to mpm_create, except where
 *     a result is returned in host memory (then the call synchronises that
 *     stream before returning).
 *   * Grid: a uniform grid of ncell[k] cells of size h per axis starting at
 *     origin[k]; nodes run -1 .. ncell[k]+1 per axis (one ghost node per
 *     side), so (ncell[k]+3) nodes per axis.  The full-grid linear node id is
 *     (i+1) + (nx+3)*((j+1) + (ny+3)*(k+1)) (x fastest).  For a batch, sim s
 *     adds the sum of the full-grid node counts of sims 0..s-1.
 *   * Particles are SoA, component-major: x[k*np + p].  Plane strain (dim 2)
 *     keeps F_zz = 1 and stores b^e as {xx, yy, xy, zz}; dim 3 stores b^e as
 *     {xx, yy, zz, yz, xz, xy}.  F is row-major: F[(i*dim + j)*np + p].
 *   * Unknowns per node: ndof = dim (displacement increment of the step), or
 *     dim + 1 for u-p (the last one is the nodal pore pressure p^{n+1}).
 *   * "Compact" vectors hold the unknowns of the active rows only, node-
 *     interleaved: v[row*ndof + c].  Rows are the active nodes in ascending
 *     full-grid id (sim by sim for a batch); mpm_prepare fixes them.
 *   * Errors: every entry point returns an mpm_status; nothing is thrown
 *     across the ABI.  mpm_last_error(ctx) describes the last failure.
 */
#ifndef MPM_H
#define MPM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  MPM_OK = 0,
  MPM_E_INVALID = -1,        /* bad argument: null pointer, size, dim, mismatch with mpm_prepare */
  MPM_E_NOMEM = -2,          /* device allocation of library scratch failed */
  MPM_E_HIP = -3,            /* a HIP runtime call failed */
  MPM_E_NOT_CONVERGED = -4,  /* Newton did not meet its tolerance in max_iter iterations */
  MPM_E_KRYLOV = -5,         /* Krylov breakdown or iteration limit */
  MPM_E_NONFINITE = -6,      /* a norm or input became NaN / Inf */
  MPM_E_OUT_OF_GRID = -7,    /* a particle's stencil leaves the padded grid */
  MPM_E_RANGE = -8           /* an elastic strain is outside the log evaluator's range (3-D only) */
} mpm_status;

/* One simulation's background grid. */
typedef struct {
  int32_t dim;        /* 2 or 3 */
  int32_t ncell[3];   /* cells per axis (unused axes 0) */
  double h;           /* cell size [m] */
  double origin[3];   /* coordinate of node 0 per axis [m] */
} mpm_grid;

/* Material and time-step data shared by all particles.  E and phi can be
 * overridden per particle (mpm_particles.E / .phi). */
typedef struct {
  int32_t up;         /* 1: u-p poromechanics (Sec. 2.2, Remark 1) */
  int32_t dp;         /* 1: Drucker-Prager return map on top of Hencky elasticity */
  int32_t dp_match;   /* 0: cone through the triaxial-compression meridian of Mohr-Coulomb,
                         1: plane-strain match, 2: triaxial-extension meridian,
                         3: J2 (von Mises, Sec. 4.2): sqrt(2 J2) <= c, phi and psi unused;
                         + 4: associated flow (dilation slope = friction slope, psi unused) */
  int32_t shape;      /* 0: quadratic B-splines; 1: cpGIMP (Sec. 2.2): node weights are the
                         averages of the linear hat functions over the particle domain, a box
                         of half-widths lp0[k] F_kk (convected with the stretch of each axis)
                         that must stay <= h/2; same 3^d stencil and pattern */
  double E, nu;       /* Young's modulus [Pa], Poisson ratio */
  double phi, c, psi; /* friction angle [rad], cohesion [Pa], dilation angle [rad] */
  double rho0;        /* reference density [kg/m^3] */
  double g[3];        /* gravity [m/s^2] */
  double perm, mu_f;  /* intrinsic permeability [m^2], fluid viscosity [Pa s] (u-p) */
  double biot, rho_f; /* Biot coefficient, fluid density [kg/m^3] (u-p) */
  double dt;          /* time step [s] (u-p) */
  double apex_reg;    /* tangent of an apex return = apex_reg x trial elastic tangent (the
                         exact one is zero for c = 0); stresses and residuals are exact */
  double lp0[3];      /* cpGIMP: initial half-width of the particle domain per axis [m] */
  int32_t elastic;    /* elastic law (dp = 0 only): 0 Hencky, tau = lambda tr(eps) 1 + 2 mu eps with
                         eps = 1/2 ln b^e (Sec. 4.2); 1 compressible Neo-Hookean,
                         tau = mu (b - 1) + lambda ln J 1 (Sec. 4.5) */
  int32_t reserved;
} mpm_material;

/* Particle state at the start of the load step (device, SoA). */
typedef struct {
  int64_t np;
  double *x;          /* [dim][np] positions; updated in place on commit */
  const double *vol0; /* [np] reference volume V0 (mass = rho0 * V0) */
  double *F;          /* [dim*dim][np] deformation gradient; updated on commit */
  double *be;         /* [4 | 6][np] elastic left Cauchy-Green tensor; updated on commit */
  const double *fp;   /* [dim][np] applied force per particle (traction x tributary area) or NULL */
  const double *E;    /* [np] per-particle Young's modulus or NULL */
  const double *phi;  /* [np] per-particle friction angle or NULL */
} mpm_particles;

/* A load-step problem: nsim independent simulations sharing one material. */
typedef struct {
  int32_t nsim;               /* >= 1 */
  int32_t reserved;
  const mpm_grid *grids;      /* host [nsim] */
  const int64_t *sim_start;   /* host [nsim+1] particle ranges per sim; NULL when nsim == 1 */
  mpm_material mat;
  mpm_particles P;
  const uint8_t *bc_mask;     /* [total full-grid nodes][ndof] 1 = constrained */
  const double *bc_value;     /* same layout: prescribed value of the unknown */
  const uint8_t *react_mask;  /* same layout or NULL: unknowns whose raw residual (negated)
                                 sums into the per-sim reaction */
} mpm_problem;

typedef struct mpm_ctx mpm_ctx;

/* Create a context bound to a device and a stream (hipStream_t as void*, NULL
 * = the null stream).  *ctx receives the handle.  The first context on a
 * device also looks up that device's address of the fixed scratch array of
 * mpm_residual_noalloc.  Errors: INVALID (device out of range, or at or
 * above MPM_MAX_DEVICES), HIP. */
int mpm_create(mpm_ctx **ctx, int device, void *stream);
/* Release the context and all library scratch.  Accepts NULL. */
int mpm_destroy(mpm_ctx *ctx);
/* Text of the last error on this context (never NULL; "" after success). */
const char *mpm_last_error(const mpm_ctx *ctx);

/* Bin particles by B-spline stencil origin and build the Jacobian pattern
 * for this load step (Sec. 3.2: the block-sparse structure follows from the
 * particle-node locality; a node row couples at most 5^d nodes).
 * Origins: o_k = floor((x_k - origin_k)/h - 1/2); a node is active iff it
 * lies in an occupied stencil; block (i, j) exists iff one occupied stencil
 * holds both nodes.  Outputs (host, may be NULL): n_row, nnzb (blocks), ndof.
 * The particle arrays and grids must stay unchanged until the next call.
 * Zero particles (or a sim without any) is valid: such a sim has no rows.
 * Errors: INVALID, NONFINITE (a coordinate is NaN or infinite), OUT_OF_GRID
 * (an origin outside -1..ncell-1 on some axis), NOMEM, HIP; the context keeps
 * no prepared problem after an error.  Synchronises the stream. */
int mpm_prepare(mpm_ctx *ctx, const mpm_problem *prob, int64_t *n_row, int64_t *nnzb, int32_t *ndof);

/* Residual at compact unknowns du (Sec. 2.2): r = f_int - f_ext with the
 * constrained unknowns (bc_mask, and nodes without material) set to zero.
 * r_raw (may be NULL) receives f_int - f_ext before that.  reaction (host,
 * may be NULL) receives per sim -sum(r_raw over react_mask).  du, r, r_raw
 * are compact [n_row*ndof] (du may be NULL only when n_row is 0).
 * Errors: INVALID (no prepare / different problem), HIP. */
int mpm_residual(mpm_ctx *ctx, const mpm_problem *prob, const double *du, double *r, double *r_raw,
                 double *reaction);

/* mpm_residual without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc.  Same arguments, results and errors as mpm_residual (the
 * same kernels, so the same bits); the context must be prepared
 * (mpm_prepare allocates the pattern and the vectors).  The per-particle
 * force records the plane-strain residual needs (np * 160 bytes) go to a
 * fixed library-owned device array of MPM_NOALLOC_SCRATCH_BYTES per device
 * instead of context memory; a larger problem is rejected with INVALID.  The
 * 3-D residual evaluates its stresses inside its scatter and keeps no
 * records, so it has no such limit.  The array is shared by every call on
 * that device and keeps the last call's contents (nothing in it needs to
 * start at zero): calls that overlap on one device, from any contexts or
 * streams, race and must be serialised by the caller.  reaction (host) makes
 * the call synchronise the stream; without it the call is asynchronous. */
#define MPM_NOALLOC_SCRATCH_BYTES (32u << 20)
#define MPM_MAX_DEVICES 64
int mpm_residual_noalloc(mpm_ctx *ctx, const mpm_problem *prob, const double *du, double *r, double *r_raw,
                         double *reaction);

/* Jacobian J = dr/d(du) at du in BSR form (Sec. 3.2): rowptr [n_row+1],
 * colind [nnzb] (ascending per row), val [nnzb][ndof][ndof] row-major
 * blocks, active_nodes [n_row] full-grid node id of each row.  Each output
 * may be NULL to skip it.  flags & MPM_JAC_RAW: return the raw derivative of
 * f_int; otherwise constrained rows and columns are zeroed with 1 on the
 * diagonal (the matrix Newton solves).  du is needed for val unless n_row
 * is 0.  Errors: INVALID, HIP. */
#define MPM_JAC_RAW 1
int mpm_jacobian_bsr(mpm_ctx *ctx, const mpm_problem *prob, const double *du, int32_t *rowptr,
                     int32_t *colind, double *val, int64_t *active_nodes, int32_t flags);

typedef struct {
  double tol;             /* Newton: stop when ||r_k|| <= tol ||r_0|| (per sim) */
  int32_t max_iter;       /* Newton iteration limit (e.g. 25) */
  int32_t commit;         /* 1: on success write x, F, b^e of the end of the step in place */
  double stall_factor;    /* also stop when ||r_k|| <= stall_factor*tol*||r_0|| and ||r_k|| > ||r_{k-1}||/2 */
  double krylov_rtol;     /* relative residual of each linear solve (0: 1e-12) */
  int32_t krylov_max_iter;
  int32_t line_search;    /* 0: full Newton steps; k > 0: halve the step up to k times until
                             ||r(u + a du)|| < (1 - 1e-4 a) ||r(u)|| */
  int32_t time_spmv;      /* k > 0: time the SpMV launches of every k-th Krylov iteration with
                             HIP events on the context's stream (report fields spmv_*) */
  int32_t krylov_method;  /* 0: block-Jacobi BiCGStab (restarted while it improves) on up to half
                             of krylov_max_iter, then restarted GMRES(100) with the same
                             preconditioner for the sims still above tolerance; 1: GMRES only;
                             2: as 0, with a geometric multigrid V-cycle (coarse levels
                             rediscretized from the particles on grids of 2^l h) preconditioning
                             BiCGStab: plane-strain single-phase levels smoothed by damped
                             block-Jacobi; 3-D and u-p levels (3x3 blocks) smoothed by
                             Chebyshev polynomials, every sim of a batch coarsened to its own
                             depth (its coarsest level as if solved alone) with its own
                             spectral estimate; the V-cycle replayed from a captured HIP graph;
                             3: as 2 with the V-cycle launched kernel by kernel (same
                             arithmetic) */
} mpm_newton_opts;

#define MPM_MAX_REPORT 32
typedef struct {
  int32_t iters;                        /* Newton iterations of the slowest sim */
  int32_t converged;                    /* 1 if every sim converged */
  int64_t krylov_iters;                 /* total Krylov iterations */
  double norms[MPM_MAX_REPORT];         /* ||r_k|| (sim 0 for batches) */
  int32_t krylov[MPM_MAX_REPORT];       /* Krylov iterations per Newton iteration */
  double ms_residual, ms_jacobian, ms_krylov, ms_total;   /* timing of this call */
  double spmv_ms;                       /* summed duration of the timed SpMV launches */
  int64_t spmv_launches;                /* number of timed SpMV launches */
  int32_t *sim_iters;                   /* host [nsim] or NULL */
  int32_t *sim_converged;               /* host [nsim] or NULL */
  double *sim_reaction;                 /* host [nsim] or NULL: reaction at convergence */
  double *sim_rel;                      /* host [nsim] or NULL: ||r_k|| / ||r_0|| at the last iterate
                                           (the stopping tolerance each sim actually reached) */
  int32_t precond_flags;                /* preconditioner faults seen during the step: 8 = a singular
                                           or missing diagonal block was replaced by the identity in
                                           block-Jacobi, 16 = a zero pivot in the coarsest multigrid
                                           solve left a column unreduced (0: none) */
  int32_t reserved;
} mpm_newton_report;

/* One load step of Newton's method (Sec. 2.2).  du: compact unknowns,
 * in = initial guess (constrained entries are overwritten by bc_value),
 * out = converged solution (NULL allowed when n_row is 0).  Requires
 * mpm_prepare for this problem.  With commit = 1 a successful step writes
 * the end-of-step state into the problem's particle arrays, which ends the
 * prepared state: the next residual, Jacobian, Newton or adjoint call needs
 * a new mpm_prepare (else INVALID).
 * Errors: NOT_CONVERGED (du holds the last iterate, nothing committed),
 * KRYLOV (its message names a preconditioner fault when one was seen, see
 * precond_flags), NONFINITE, INVALID, HIP.  Synchronises the stream. */
int mpm_newton_step(mpm_ctx *ctx, const mpm_problem *prob, const mpm_newton_opts *opts, double *du,
                    mpm_newton_report *rep);

/* End-of-step particle update (Sec. 2.2: the last stage of a step, after
 * the grid solve, carries the converged increment back to the particles) at
 * compact du: x += sum w du, F = dF F, b^e = exp(2 eps^e), written to x_out,
 * F_out, be_out (may alias the problem's arrays; when one does, the prepared
 * state ends as after a committed Newton step).  du may be NULL when n_row
 * is 0.  Errors: INVALID, RANGE, HIP. */
int mpm_update(mpm_ctx *ctx, const mpm_problem *prob, const double *du, double *x_out, double *F_out,
               double *be_out);

/* Adjoint of one converged load step (plane strain, single-phase): the
 * gradient the paper obtains by reverse AD through its whole-run tape
 * (Sec. 4.5), here by one transposed solve per step.  prob: the state s_n
 * at the start of the step, prepared with mpm_prepare; du: that step's
 * converged compact increment.  Inputs: react_bar (host [nsim]) = dL/dR_n of
 * the step's reaction (R = -sum of the raw residual over react_mask);
 * sbar_next (device [10][np] in caller order: x (2), F (4), b^e (4)) =
 * dL/ds_{n+1}, or NULL for zero.  Outputs: sbar_n (device [10][np], may be
 * NULL) = dL/ds_n; theta_bar (device [nsim][2]) = this step's contribution
 * to dL/dE and dL/dphi of each sim (E, phi per particle, summed per sim).
 * The transposed system uses the step's Dirichlet-modified Jacobian and is
 * solved by block-Jacobi BiCGStab (GMRES(100) fallback, at most 20000
 * iterations) to a true relative residual of krylov_rtol (0: 1e-12);
 * krylov_iters (host [nsim] or NULL) and krylov_rel (host [nsim] or NULL:
 * the true relative residual each sim reached) describe it.  A solve that
 * stops above 10 x krylov_rtol returns KRYLOV: the gradient would carry its
 * error (pass a looser krylov_rtol to accept that).
 * Errors: INVALID (not prepared, 3-D or u-p), NOMEM, KRYLOV, HIP. */
int mpm_adjoint_step(mpm_ctx *ctx, const mpm_problem *prob, const double *du, const double *react_bar,
                     const double *sbar_next, double *sbar_n, double *theta_bar, double krylov_rtol,
                     int32_t *krylov_iters, double *krylov_rel);

/* y = J x with the BSR values val of this load step's pattern: the
 * matrix-vector product that drives the preconditioned iterative solve of
 * each Newton correction (Remark 2 of Sec. 2.2).  val [nnzb][ndof][ndof]
 * as returned by mpm_jacobian_bsr; x, y compact [n_row*ndof], must not
 * alias.  z (may be NULL): the product also forms the per-row-block partial
 * sums of z.y and y.y that the Krylov iteration fuses into it (kept in
 * library scratch).  Errors: INVALID, HIP. */
int mpm_spmv(mpm_ctx *ctx, const double *val, const double *x, double *y, const double *z);

/* y = J x without forming the matrix: the matrix-free Newton-Krylov variant
 * the paper names for large problems (Sec. 2.2, Remark 2).  Each particle's
 * tangent table V0 dP/dF at du (d^2 x d^2 doubles, the same forward passes as
 * mpm_jacobian_bsr) is stored, and the product is applied on the fly: per
 * particle dF = sum_b x_b (x) grad w_b, dP = T : dF, then the scatter of
 * dP grad w_a like the internal force.  Equal to the BSR product of
 * mpm_jacobian_bsr at the same du up to summation order.  flags &
 * MPM_JAC_RAW: the raw derivative of f_int; otherwise the Dirichlet-modified
 * matrix (constrained columns read as zero, constrained rows return x).
 * flags & MPM_JV_REUSE: reuse the tangent tables of the previous mpm_jv,
 * mpm_jacobian_bsr or Newton assembly of this prepare (du ignored, may be
 * NULL), so a Krylov loop pays one tangent pass per Newton iteration.  x, y
 * compact [n_row*ndof], must not alias.  Single-phase only.
 * Errors: INVALID (u-p, no tables to reuse, aliasing), NOMEM, HIP. */
#define MPM_JV_REUSE 2
int mpm_jv(mpm_ctx *ctx, const mpm_problem *prob, const double *du, const double *x, double *y, int32_t flags);

/* Lanes per BSR row of the SpMV launch shape in use: the pinned one (see
 * mpm_spmv_set_lanes), else the one the autotuner picked for the current
 * pattern (the product is timed on the live matrix with 4, 8 and 16 lanes
 * per row at the first product after mpm_prepare); 0 before that.  No errors. */
int mpm_spmv_lanes(const mpm_ctx *ctx);

/* Pin the SpMV launch shape to lanes = 4, 8 or 16 lanes per BSR row for this
 * context, kept across mpm_prepare calls; lanes = 0 returns to autotuning at
 * the next product.  Every shape sums each row in the same order (block k of
 * a row into partial sum k mod 16, the 16 partial sums in a fixed tree), so
 * products, Krylov iterates and Newton results are bitwise identical for any
 * shape: the pin only fixes the speed, e.g. for timing one shape.
 * Errors: INVALID (another lanes value). */
int mpm_spmv_set_lanes(mpm_ctx *ctx, int32_t lanes);

#ifdef __cplusplus
}
#endif
#endif /* MPM_H */
