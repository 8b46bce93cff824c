/*
 * ofdft.h -- C ABI of the MI355X (gfx950) library for the hot path of periodic
 * real-space orbital-free DFT with higher-order finite differences
 * (Ghosh & Suryanarayana, arXiv:1412.8250).
 *
 * Conventions shared by every call
 * --------------------------------
 * Grid: uniform, periodic, n_x x n_y x n_z points with spacings h_x, h_y, h_z
 *   (Section 4: L_a = n_a h).  Arrays are stored [nz][ny][nx], x fastest,
 *   contiguous.  Complex arrays interleave (re, im); complex128 is two doubles
 *   per point, complex64 two floats.
 * Pointers: every array pointer is a DEVICE pointer owned by the caller; the
 *   library never frees or keeps a caller pointer beyond the call, except where
 *   a create call says so.  Scalars and descriptors live in host memory.
 * Streams: `stream` is a hipStream_t passed as void* (NULL = default stream).
 *   Work is enqueued on it; calls that must read convergence scalars back
 *   synchronise that stream only.
 * Errors: every call returns an int status (OFDFT_OK = 0).  Negative values are
 *   errors, 1 means "finished without meeting the tolerance" (results written).
 *   ofdft_last_error() gives a thread-local message for the last failure.
 *   No C++ exception crosses this boundary.
 * Allocation: device workspaces are allocated by the *_create calls only;
 *   solve/apply/mix/step calls do not allocate.
 */
#ifndef OFDFT_H
#define OFDFT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OFDFT_OK             0
#define OFDFT_NOT_CONVERGED  1
#define OFDFT_INVALID_ARG   (-1)
#define OFDFT_NONFINITE     (-2)
#define OFDFT_BREAKDOWN     (-3)
#define OFDFT_HIP_ERROR     (-4)
#define OFDFT_NO_MEMORY     (-5)

typedef enum { OFDFT_F64 = 0, OFDFT_F32 = 1, OFDFT_C128 = 2, OFDFT_C64 = 3 } ofdft_dtype;

/* Solver forms for the Poisson solve. */
typedef enum {
    OFDFT_PLAIN_F64 = 0,       /* CG in FP64 throughout                                   */
    OFDFT_REFINED_F32 = 1,     /* FP32 stencil + FP32 CG inside FP64 residual refinement  */
    OFDFT_LEARNED = 2,         /* network initial guess + flexible CG with the network as
                                  preconditioner, FP64 vectors; plain CG as fallback      */
    OFDFT_MULTIGRID = 3,       /* CG preconditioned by a geometric multigrid V-cycle of
                                  the second-order operator, FP64 vectors; the cycle's
                                  level arrays in FP32                                    */
    OFDFT_MULTIGRID_F64 = 4,   /* the same with the cycle in FP64 throughout              */
    OFDFT_LEARNED_REFINED = 5, /* the learned form's network correction of the starting
                                  guess, then the refined form (FP32 CG inside FP64
                                  residual refinement) to the tolerance                  */
} ofdft_mode;

typedef struct {
    int nx, ny, nz;            /* points per axis, >= 1                                   */
    double hx, hy, hz;         /* spacings (bohr), > 0                                    */
} ofdft_grid;

typedef struct {
    int iters;                 /* Krylov iterations (inner iterations for refined form)  */
    int outer_iters;           /* refinement steps (refined form), else 0                */
    int nn_applies;            /* network applications (learned form)                    */
    int fell_back;             /* 1 if the learned form fell back to plain CG            */
    int status;                /* OFDFT_* status of this solve                            */
    double rel_res;            /* final true relative residual, recomputed in FP64       */
    double removed_mean;       /* mean removed from the Poisson right-hand side          */
    double seconds;            /* wall time of the call, measured with HIP events        */
} ofdft_solve_stats;

/* Thread-local message of the last failing call; returns its length. */
int ofdft_last_error(char *buf, size_t len);

/* Library version string (static storage). */
const char *ofdft_version(void);

/* ------------------------------------------------------------------------
 * fd_laplacian_apply -- y = alpha * L_h x + beta * y
 *
 * L_h is the order-2N central-difference Laplacian of Section 4 (FD Laplacian
 * equation): sum over p = 0..N of w_p times the six values at offsets +-p along
 * the axes, w_0 = -(1/h^2) sum_{q<=N} 1/q^2 and
 * w_p = 2(-1)^{p+1} (N!)^2 / (h^2 p^2 (N-p)!(N+p)!), per axis with that axis'
 * spacing; indices outside the grid map to their periodic images (applied
 * repeatedly when the grid is shorter than the stencil).
 *   grid    grid descriptor (host)
 *   radius  N in 1..6 (6 = 12th order)
 *   dtype   element type of x and y; alpha/beta are real
 *   x, y    device arrays of nx*ny*nz elements; must not overlap
 *   beta == 0 means y is write-only (its old contents are not read).
 * Errors: INVALID_ARG for bad sizes/radius/dtype or null pointers.
 * ------------------------------------------------------------------------ */
int fd_laplacian_apply(const ofdft_grid *grid, int radius, ofdft_dtype dtype,
                       const void *x, void *y, double alpha, double beta, void *stream);

/* ------------------------------------------------------------------------
 * fd_gradient_apply -- (gx, gy, gz) = grad_h x
 *
 * The order-2N central-difference gradient of Section 4 (FD gradient
 * equation): component a is sum over p = 1..N of w~_p (x(+p) - x(-p)) along
 * axis a, w~_p = (-1)^{p+1} (N!)^2 / (h_a p (N-p)!(N+p)!), periodic images.
 *   grid    grid descriptor (host); radius N in 1..6
 *   x       device FP64 array of nx*ny*nz elements
 *   gx, gy, gz  device FP64 outputs of the same size; x and the outputs must
 *           be four distinct arrays
 * Errors: INVALID_ARG for bad sizes/radius, null or repeated pointers.
 * ------------------------------------------------------------------------ */
int fd_gradient_apply(const ofdft_grid *grid, int radius, const double *x, double *gx, double *gy,
                      double *gz, void *stream);

/* ------------------------------------------------------------------------
 * Periodic Poisson solve (Section 3.3, Poisson equation; Section 4 solver
 * notes): finds phi with -L_h phi = P g and sum(phi) = 0, where
 * P = I - (1/n) 1 1^T removes the mean of the right-hand side.  The paper
 * solves the continuum problem -(1/4 pi) Lap phi = rho + b, so callers pass
 * g = 4 pi (rho + b).  A non-neutral g is not an error: its mean is removed
 * and reported in stats->removed_mean.
 *
 * ofdft_poisson_create allocates the workspace for one grid and one mode.
 *   mode  OFDFT_PLAIN_F64, OFDFT_REFINED_F32, OFDFT_MULTIGRID or
 *         OFDFT_MULTIGRID_F64 (every axis must halve evenly down to at most
 *         16 points; INVALID_ARG otherwise) or
 *         OFDFT_LEARNED or OFDFT_LEARNED_REFINED (need a network, see
 *         ofdft_poisson_set_network).
 *         Multigrid: M = one V(2,2) cycle of the periodic 7-point operator
 *         (damped Jacobi, omega 0.8; full weighting; trilinear
 *         prolongation; exact DFT solve on the coarsest grid), a fixed
 *         symmetric positive definite approximation of the inverse of
 *         -L_h, so the iteration count does not grow with the grid.
 * cg_poisson_solve:
 *   rhs      device FP64 array g (not modified)
 *   x        device FP64 array: initial guess on entry (warm start), solution on
 *            exit, shifted to zero mean
 *   rel_tol  stop when ||P g + L_h x||_2 <= rel_tol ||P g||_2, with the residual
 *            recomputed in FP64 at the end
 *   max_iter maximum Krylov iterations in total
 *   stats    optional (may be NULL)
 * Returns OK, NOT_CONVERGED (x still written), BREAKDOWN (p^T A p <= 0),
 * NONFINITE (NaN/Inf met), INVALID_ARG, HIP_ERROR.
 * ------------------------------------------------------------------------ */
typedef struct ofdft_poisson ofdft_poisson;
int ofdft_poisson_create(const ofdft_grid *grid, int radius, int mode, ofdft_poisson **out);
int ofdft_poisson_destroy(ofdft_poisson *s);
int cg_poisson_solve(ofdft_poisson *s, const double *rhs, double *x, double rel_tol,
                     int max_iter, ofdft_solve_stats *stats, void *stream);
/* ofdft_poisson_rhs: the right-hand side of the solver's grid from a density
 * and the nuclear charge density (Section 3.3, Poisson equation, whose
 * continuum form is -(1/4 pi) Lap phi = rho + b): g = 4 pi (rho + b) with its
 * mean removed (the net-charge projection, FP64 sums).  rho, b, g: device
 * FP64 arrays of the grid (g may alias rho or b).  removed_mean (host,
 * optional) receives the mean removed.  Synchronises the stream. */
int ofdft_poisson_rhs(ofdft_poisson *s, const double *rho, const double *b, double *g, double *removed_mean,
                      void *stream);
/* cg_poisson_solve_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the OFDFT_PLAIN_F64 form of cg_poisson_solve with the same
 * arguments as a solver of that mode (rhs, x, rel_tol, max_iter, stats, stream
 * as above; grid and radius as for ofdft_poisson_create), but no context:
 * its workspace (five FP64 vectors, the device scalars and the reduction
 * partials, about 40.5 MiB) is a static device array of the library that each
 * GPU holds until the process ends.  The call allocates nothing (no device or
 * pinned host memory, events or graphs) and synchronises the stream.
 * Limit: nx*ny*nz <= 2^20 points (96^3 fits); larger grids return
 * INVALID_ARG.  Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams or threads) race and must be serialised
 * by the caller.  Results equal cg_poisson_solve's (same kernels, same order). */
int cg_poisson_solve_noalloc(const ofdft_grid *grid, int radius, const double *rhs, double *x,
                             double rel_tol, int max_iter, ofdft_solve_stats *stats, void *stream);
/* Blocks of 16 CG iterations are captured once as a HIP graph (on a private
 * stream) and replayed; kernels leave early once converged.  enable = 0 turns
 * this off for the solver (results are bitwise identical either way). */
int ofdft_poisson_set_graphs(ofdft_poisson *s, int enable);
/* Refined form: each FP32 inner solve targets 0.3 x (remaining reduction),
 * clamped to [inner_min, inner_max] (defaults 1e-5, 1e-1).  INVALID_ARG unless
 * 0 < inner_min <= inner_max < 1. */
int ofdft_poisson_set_refinement(ofdft_poisson *s, double inner_min, double inner_max);

/* ------------------------------------------------------------------------
 * Batched complex shifted solves (Section 3.1, Helmholtz equations):
 *   (-L_h + kappa_j) u_j = f_j,  j = 0..nsys-1,
 * the paper's  -(2kF)^-2 Lap V + Q V = P f  multiplied by (2kF)^2
 * (kappa = (2kF)^2 Q).  Each system may live on its own grid.  The matrix is
 * complex symmetric; the solver is COCG (conjugate gradients with the
 * unconjugated bilinear form).  Every COCG phase of all systems is one launch
 * (ofdft_batch_set_config below selects the schedule).
 *
 * ofdft_batch_create: nsys systems, grids[j] (host array), one radius, dtype
 *   OFDFT_C128 or OFDFT_C64 (C64 runs COCG in complex64 inside complex128
 *   residual refinement).  Allocates all workspaces.
 * cg_helmholtz_solve_batched:
 *   kappa    host array of 2*nsys doubles (re, im) per system; kappa != 0
 *   rhs      host array of nsys device pointers to complex128 arrays f_j
 *   x        host array of nsys device pointers to complex128 arrays:
 *            initial guess on entry, solution on exit
 *   rel_tol  per-system relative residual target (true residual, complex128)
 *   stats    optional host array of nsys records
 * Returns OK, NOT_CONVERGED if any system missed the tolerance, BREAKDOWN,
 * NONFINITE, INVALID_ARG, HIP_ERROR.
 * ofdft_batch_set_preconditioner: kind OFDFT_PRECOND_NONE (default) or
 *   OFDFT_PRECOND_MULTIGRID: COCG preconditioned by one V(2,2) multigrid cycle
 *   of the second-order operator -Delta_h + kappa_j (damped Jacobi smoothing,
 *   full weighting, trilinear prolongation, exact DFT solve on the coarsest
 *   grid), the real-space preconditioner of Section 5.5 applied to the shifted
 *   systems.  The cycle is complex symmetric, so the preconditioned iteration
 *   keeps the bilinear form r^T z.  Requires dtype C128 and the stepped
 *   schedule (group 0 at solve time, else the solve returns INVALID_ARG);
 *   every axis of every grid must halve evenly down to at most 16 points.
 *   Allocates one complex128 vector per system and multigrid level arrays
 *   per system (about 1.3 fine-grid vectors); consecutive systems on one
 *   grid (up to 64) form a group whose cycles run as one launch per kernel.
 *   INVALID_ARG (nothing changed) or NO_MEMORY.
 * ------------------------------------------------------------------------ */
typedef enum {
    OFDFT_PRECOND_NONE = 0,
    OFDFT_PRECOND_MULTIGRID = 1,      /* cycle with FP32 / complex64 level arrays (reads r and
                                         writes z in FP64 / complex128)                      */
    OFDFT_PRECOND_MULTIGRID_F64 = 2   /* cycle in FP64 / complex128 throughout                */
} ofdft_precond;
typedef struct ofdft_batch ofdft_batch;
int ofdft_batch_create(int nsys, const ofdft_grid *grids, int radius, ofdft_dtype dtype,
                       ofdft_batch **out);
int ofdft_batch_destroy(ofdft_batch *b);
int cg_helmholtz_solve_batched(ofdft_batch *b, const double *kappa, const void *const *rhs,
                               void *const *x, double rel_tol, int max_iter,
                               ofdft_solve_stats *stats, void *stream);
int ofdft_batch_set_preconditioner(ofdft_batch *b, int kind);
/* z = M_j r: one cycle of the preconditioner of system j's grid with shift
 * kappa (host {Re, Im}); r, z device complex128 arrays of that grid, z != r.
 * Synchronises the stream.  INVALID_ARG without a preconditioner set. */
int ofdft_batch_apply_preconditioner(ofdft_batch *b, int j, const double *kappa, const void *r, void *z,
                                     void *stream);

/* ------------------------------------------------------------------------
 * Multi-shift COCG: the shifted systems (-L_h + kappa_r) u_r = f, r = 0 ..
 * nshift-1, of ONE right-hand side (the kernel convolutions of Section 3.1
 * and the order-2 terms of Section 2 apply several shifts to the same f).
 * The Krylov space does not depend on the shift, so one COCG sequence of a
 * seed system serves every shift (shifted COCG: r_k^(r) = r_k / pi_k^(r) with
 * a scalar recurrence for pi), one stencil application per iteration.  All
 * iterates start at zero; a shift is frozen once |r_k| / |pi_k^(r)| <=
 * rel_tol |f|.  No preconditioner (a shift-dependent preconditioner breaks the
 * shared Krylov space: use ofdft_batch_set_preconditioner for that).
 * ofdft_multishift_create: one grid, radius 1..6, up to max_shifts (1..16)
 *   shifts per solve.  Allocates 4 + max(max_shifts - 1, 1) complex128 vectors of
 *   the grid and the solve's device scalars, so a context serves one solve
 *   at a time (solves on one context must not overlap on different streams).
 *   INVALID_ARG or NO_MEMORY.
 * cocg_multishift_solve:
 *   kappa    host array of 2*nshift doubles (re, im); each kappa_r != 0
 *   seed     index of the seed system, or -1: the shift expected to converge
 *            slowest (Re kappa < 0, putting -kappa inside the spectrum of
 *            -L_h, with the smallest |Im kappa|; else the smallest |kappa|)
 *   rhs      device complex128 array f of the grid (not modified)
 *   x        host array of nshift distinct device complex128 arrays of the
 *            grid, none equal to rhs: the solutions on exit (overwritten,
 *            no initial guess)
 *   stats    optional host array of nshift records: iters = steps after
 *            which the shift froze plus the steps of its correction solves,
 *            outer_iters = seed steps taken, rel_res = true relative residual
 *            recomputed in complex128, status, seconds
 *   seed_used optional: the seed index used
 * The recurred residual that freezes a shift and the true residual drift
 * apart in floating point: a frozen shift whose true residual is above
 * rel_tol gets correction solves (d = f - A x, A e = d by a one-shift
 * sequence from zero, x += e; at most 4, within the max_iter budget left).
 * Returns OK (every shift's true residual <= rel_tol), NOT_CONVERGED (a
 * shift missed max_iter or its true residual is still above rel_tol),
 * BREAKDOWN, NONFINITE, INVALID_ARG, HIP_ERROR.  Synchronises the stream.
 * ------------------------------------------------------------------------ */
typedef struct ofdft_multishift ofdft_multishift;
int ofdft_multishift_create(const ofdft_grid *grid, int radius, int max_shifts, ofdft_multishift **out);
int ofdft_multishift_destroy(ofdft_multishift *m);
int cocg_multishift_solve(ofdft_multishift *m, int nshift, const double *kappa, int seed, const void *rhs,
                          void *const *x, double rel_tol, int max_iter, ofdft_solve_stats *stats,
                          int *seed_used, void *stream);

/* ------------------------------------------------------------------------
 * Anderson mixing (Appendix D):
 *   v_{k+1} = v_k + zeta f_k - (S_k + zeta Y_k)(Y_k^T Y_k)^{-1} Y_k^T f_k,
 * S_k, Y_k the last m differences of iterates and of residuals f = vhat - v.
 * The first call (no history) returns v + zeta f.  If Y^T Y is numerically
 * singular (condition estimate >= 1e12) the oldest columns are dropped.
 * ofdft_anderson_create: n grid values per vector, history m in 0..16, zeta.
 *   The context keeps S, Y (m columns each) and the previous v, f in device
 *   memory.
 * anderson_mix: v, f, v_next are device FP64 arrays of n values; v_next may
 *   alias v.
 * ------------------------------------------------------------------------ */
typedef struct ofdft_anderson ofdft_anderson;
int ofdft_anderson_create(int64_t n, int m, double zeta, ofdft_anderson **out);
int ofdft_anderson_destroy(ofdft_anderson *a);
int ofdft_anderson_reset(ofdft_anderson *a);
int anderson_mix(ofdft_anderson *a, const double *v, const double *f, double *v_next,
                 void *stream);

/* ------------------------------------------------------------------------
 * Fixed-point (SCF-type) iteration, Section 3.3 and its flowchart.
 * The mixing variable is v = phi + mu V_LR.  One step:
 *   u      = U(v)  -- minimiser of the local functional
 *            h^3 sum [C_F rho^{5/3} + eps_xc(rho) rho + v rho] - (lambda/2) h^3 sum u L_h u
 *            subject to h^3 sum u^2 = N_e (Appendix C, Algorithm 1: Polak-Ribiere
 *            non-linear CG with restarts, Brent line search, renormalisation)
 *   phi    = Poisson(4 pi (u^2 + b))                               (warm start)
 *   V_LR   = C_F sum_r [alpha rho^{alpha-1} V_{beta,r} + beta rho^{beta-1} V_{alpha,r}]
 *            from the 8 shifted solves of the K_00 term, kappa_r = (2kF)^2 Q_00r,
 *            right-hand sides P_00r (-L_h rho^beta) and P_00r (-L_h rho^alpha)
 *            (Section 3.1 with m = n = 0; Appendix A table)      (mu = 1 only)
 *   vhat   = phi + mu V_LR,  f = vhat - v,  v <- Anderson(v, f)
 * and reports ||f|| / ||v||.
 * fixed_point = 1 takes the paper's own form instead: the mixing variable is
 * the kernel potential V_LR alone and U keeps the electrostatics inside its
 * functional (the map U(V_LR) of Section 3.3), so a step is
 *   u      = U(mu V_LR) -- minimiser of the functional above with
 *            v = mu V_LR + phi[u] and the electrostatic energy
 *            1/2 h^3 sum (rho + b) phi[rho] added, phi re-solved for every u
 *   phi    = Poisson(4 pi (u^2 + b));  Vhat = V_LR[u] (8 shifted solves)
 *   f = Vhat - V_LR,  V_LR <- Anderson(V_LR, f),  reports ||f|| / ||V_LR||
 * (0 for mu = 0, where one step gives the TFW ground state).  U solves two
 * Poisson equations per iteration, for the fields of u d and d^2 (d the
 * search direction); phi along the line u + s d follows from them exactly,
 * and each line-search probe is a pointwise pass.  The potential form mixes
 * the electrostatic response too, which the paper reports (and large cells
 * show) to become unstable as the cell grows.
 * ------------------------------------------------------------------------ */
typedef struct {
    ofdft_grid grid;
    int radius;                /* FD order / 2, 1..6                                     */
    double lambda;             /* von Weizsacker weight (TFW: 0.2)                      */
    int mu;                    /* 0: TFW, 1: add the K_00 linear-response kernel term     */
    double n_electrons;        /* N_e                                                     */
    int history;               /* Anderson history m                                      */
    double zeta;               /* Anderson mixing parameter                               */
    double u_tol;              /* stop U when ||H u - eta u|| / ||u|| <= u_tol            */
    int n_restart;             /* Polak-Ribiere restart period                            */
    int u_max_iter;
    double poisson_tol;        /* relative residual of the Poisson solve                  */
    int poisson_mode;          /* OFDFT_PLAIN_F64, OFDFT_REFINED_F32, OFDFT_MULTIGRID(_F64) */
    double helmholtz_tol;      /* relative residual of each shifted solve                 */
    ofdft_dtype helmholtz_dtype; /* OFDFT_C128 or OFDFT_C64                               */
    int max_iter;              /* Krylov iteration cap per solve                          */
    double line_tol;           /* line search: relative tolerance on the step, 0 = 1e-8  */
    int helmholtz_precond;     /* OFDFT_PRECOND_NONE or OFDFT_PRECOND_MULTIGRID(_F64), C128 */
    int u_precond;             /* density update: OFDFT_PRECOND_NONE (Algorithm 1 as
                                  printed) or OFDFT_PRECOND_MULTIGRID(_F64) (lambda > 0): the
                                  steepest-descent direction r becomes z = M r projected
                                  on <u, z> = 0, M one multigrid cycle of -Delta +
                                  2 sigma / lambda (sigma: u_precond_sigma);
                                  Polak-Ribiere xi = <r - r_prev, z> / <r_prev, z_prev>.
                                  Same minimiser, several times fewer iterations; every
                                  axis must halve evenly down to at most 16 points     */
    int lr_order;              /* kernel terms (mu = 1): 0 = K_00 only (8 shifted systems,
                                  4 solved); 2 = the order-2 expansion of Section 2 with
                                  the K_00, K_10, K_20, K_11 rows of Appendix A (pairs
                                  m + n <= 2): 16 distinct convolutions K_mn rho^a, 64
                                  shifted systems, 32 solved (r = 2, 4 conjugates),
                                  batched 8 at a time                                  */
    double u_precond_sigma;    /* sigma of the density update's preconditioner (hartree);
                                  0 = V_TF(N_e / volume)                               */
    double line_slope_tol;     /* line search: a step is accepted once |dE/ds| is at most
                                  this fraction of its value at s = 0 (or the bracket is
                                  below line_tol); 0 = 1e-6 (an exact line search)      */
    int helmholtz_multishift;  /* 1 = the kernel solves without a warm start (the
                                  context's first kernel potential) by multi-shift COCG
                                  (see cocg_multishift_solve; from zero, complex128): the
                                  systems sharing a right-hand side g (-L_h rho^a for
                                  K_00; rho^a, the same power in several kernels, for the
                                  order-2 terms) in one solve, up to 16 shifts, then
                                  V = c_r U with the system's factor; later kernel
                                  potentials by the batched solver (helmholtz_precond,
                                  helmholtz_dtype) warm-started from the previous
                                  solutions (the multi-shift workspace is freed once
                                  that first potential is formed).  0 = the batched
                                  solver throughout.                                     */
    int autotune;              /* 1 = tune the launch configuration at creation: the
                                  fused stencil passes and the apply on the grid
                                  (ofdft_tune_stencil) and, for mu = 1, the shifted-
                                  system batch on the first batched kernel solve
                                  (ofdft_batch_tune, 8 iterations); 0 = untuned      */
    int fixed_point;           /* 0 = potential mixing (v = phi + mu V_LR, U local);
                                  1 = the kernel-potential fixed point with the
                                  electrostatics inside U (see above); state vector 0
                                  then holds V_LR                                      */
} ofdft_scf_params;

typedef struct ofdft_scf ofdft_scf;
/* b: device FP64 nuclear charge density; u0: device FP64 initial sqrt-density.
 * Both are copied.  Computes v_0 = phi[u0] + mu V_LR[u0] (fixed_point 1:
 * V_LR[u0], and the field of b alone for the electrostatics inside U).
 * Status of create and step: the worst of their parts.  NOT_CONVERGED (the
 * context is still created, the step still taken and *fp_residual written)
 * when U(v) stopped above u_tol (u_max_iter reached, or no descent direction
 * left at FP64 precision) or a Poisson or shifted solve missed its tolerance
 * within max_iter; errors of any part are returned at once (create then
 * frees everything and leaves *out unset). */
int ofdft_scf_create(const ofdft_scf_params *p, const double *b, const double *u0,
                     ofdft_scf **out, void *stream);
int ofdft_scf_destroy(ofdft_scf *s);
int ofdft_scf_step(ofdft_scf *s, double *fp_residual, void *stream);

/* State access for checkpointing and inspection.  which: 0 = v, 1 = u, 2 = phi,
 * 3 = V_LR (device FP64 arrays of nx*ny*nz values); 4.. = the solutions of
 * the shifted systems, kept as their next warm starts (device complex128
 * arrays, 2*nx*ny*nz doubles; mu = 1 only): lr_order 0: 4..11 = system
 * which-4 of the K_00 set (the odd systems are the conjugates of the even
 * ones and are rewritten from them after each step); lr_order 2: 4..35 =
 * solved system which-4, convolution (which-4)/2 with r = 1 (even) or 3 (odd),
 * convolutions ordered by kernel pair (m, n) = (0,0), (0,1), (0,2), (1,0),
 * (1,1), (2,0), then p, q, then the beta-side power before the alpha-side
 * one, each (kernel, power) once.  INVALID_ARG for other values. */
int ofdft_scf_get(ofdft_scf *s, int which, double *dst, void *stream);
int ofdft_scf_set(ofdft_scf *s, int which, const double *src, void *stream);
/* Checkpoint of the whole iteration state to a file and back: every state
 * array of ofdft_scf_get (v, u, phi, V_LR, the shifted systems' warm
 * starts), the Anderson history (S, Y, the previous v and f, ring position)
 * and the line-search step memory, so that a loaded context continues the
 * saved one's trajectory exactly.  load requires a context created with the
 * same grid, spacings, radius, N_e, kernel settings and history length
 * (INVALID_ARG otherwise, or for an unreadable / short file).  Both
 * synchronise the stream; the file holds (4 + warm starts) grid arrays plus
 * 2 m + 2 for Anderson. */
int ofdft_scf_save(ofdft_scf *s, const char *path, void *stream);
int ofdft_scf_load(ofdft_scf *s, const char *path, void *stream);
/* Forget the Anderson history and the line-search step memory, so that the
 * next step behaves like the first step from the current state. */
int ofdft_scf_reset_history(ofdft_scf *s);
/* The four K_00 shifts kappa_r = (2 kF)^2 Q_r (host, 8 doubles re, im) and the
 * factors P_r (8 doubles, may be NULL) of the Appendix A table for the
 * context's cell, kF = (3 pi^2 N_e / |Omega|)^(1/3) (Section 3.1): the
 * shifted systems (-L_h + kappa_r) V_r = P_r (-L_h rho^p) the kernel term
 * solves.  INVALID_ARG for NULL. */
int ofdft_scf_kernel_shifts(ofdft_scf *s, double *kappa8, double *factor8);
/* Statistics of the last step: [0] U iterations, [1] Poisson iterations,
 * [2] total shifted-solve iterations (of the 4 systems solved: r = 1, 3 for
 * both powers; r = 2, 4 are their complex conjugates, Appendix A), [3] U
 * residual, [4] Poisson residual, [5] worst shifted-solve residual, [6] eta. */
int ofdft_scf_stats(ofdft_scf *s, double *out7);

/* Ground-state energy terms and forces on the nuclei (Section 3.3 energy
 * expression and forces; Section 3.2 local electrostatics; Appendix B overlap
 * correction), from the context's current u, phi and kernel solutions (call
 * after ofdft_scf_create or a step).  Pseudocharges are the Gaussians of the
 * stand-in inputs: b_J = charge (2 pi sigma^2)^-3/2 exp(-|x - R_J|^2 / (2
 * sigma^2)) with images, V_J = charge erf(r / (sqrt 2 sigma)) / r; the self
 * term and the forces sum over each atom's grid points within `cutoff`
 * (e.g. 8.5 sigma); the overlap correction is the closed form for Gaussians,
 * E_c = 1/2 sum_{I != J, images} charge^2 erfc(d / (2 sigma)) / d.
 * ofdft_scf_energy: terms (host, 8 doubles, hartree): Thomas-Fermi,
 *   von Weizsacker (-(lambda/2) h^3 <u, L_h u>), exchange-correlation,
 *   electrostatic (1/2 h^3 sum (rho + b) phi), nuclear self energy (-1/2 sum_J
 *   int b_J V_J), overlap correction, kernel energy (mu T_LR of the expansion
 *   in use), total.
 * ofdft_scf_forces: forces (host, 3 doubles per atom, hartree/bohr)
 *   f_J = sum_images h^3 sum grad b_J (phi - V_J) + f^c_J.
 * Both synchronise the stream; INVALID_ARG for a bad context or atoms. */
typedef struct {
    int count;                 /* atoms                                                  */
    const double *pos;         /* host, 3*count (x, y, z) in bohr                        */
    double charge;             /* pseudocharge per atom (-3 for the Al stand-in)         */
    double sigma;              /* Gaussian width (bohr)                                  */
    double cutoff;             /* radius of the per-atom grid sums (bohr)                */
} ofdft_gauss_atoms;
int ofdft_scf_energy(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *terms, void *stream);
int ofdft_scf_forces(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double *forces, void *stream);

/* The same terms and forces in the forms the paper prints:
 *   - von Weizsacker term (lambda/2) h^3 sum |grad_h u|^2 with the FD gradient
 *     of Section 4 (fd_gradient_apply);
 *   - overlap correction by the grid form of Appendix B: reference charges
 *     b~_J = Gaussians of width sigma_ref (same charge), V_c from one Poisson
 *     solve of -L_h V_c = 4 pi (b~ - b) with the context's solver and
 *     poisson_tol, its constant set so that V_c has the mean of
 *     sum_J (V~_J - V_J), i.e. -2 pi charge M (sigma_ref^2 - sigma^2) / |Omega|;
 *       E_c = 1/2 h^3 sum (b~ + b) V_c + 1/2 sum_J h^3 sum b_J V_J
 *             - 1/2 sum_J h^3 sum b~_J V~_J
 *     and the Appendix B force correction f^c_J (per-atom sums).  With
 *     non-overlapping reference charges both tend to the closed forms of
 *     ofdft_scf_energy / ofdft_scf_forces as h -> 0.
 * `cutoff` must cover both Gaussians (e.g. 8.5 max(sigma, sigma_ref)).
 * terms: the 8 doubles of ofdft_scf_energy with [1], [5] and [7] in these
 * forms.  They use the density-update workspace (not during a step).
 * Returns NOT_CONVERGED (results written) if the Poisson solve missed its
 * tolerance; INVALID_ARG for a bad context, atoms or sigma_ref <= 0. */
int ofdft_scf_energy_paper_form(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double sigma_ref,
                                double *terms, void *stream);
int ofdft_scf_forces_paper_form(ofdft_scf *s, const ofdft_gauss_atoms *atoms, double sigma_ref,
                                double *forces, void *stream);

/* The density update U(v) alone (Algorithm 1), using the context's parameters:
 * v, u device FP64; u holds the starting guess on entry and U(v) on exit.
 * iters/residual/eta (host, optional) receive the iteration count, the final
 * ||H u - eta u|| / ||u|| and eta. */
int ofdft_density_update(ofdft_scf *s, const double *v, double *u, int *iters,
                         double *residual, double *eta, void *stream);

/* ------------------------------------------------------------------------
 * Learned solver aid (not in the paper, whose conclusion calls for real-space
 * preconditioners, Section 5.5).  A 4-level periodic 3D convolutional U-Net
 * (channels 16/32/64/64, 3x3x3 periodic convolutions, bias-free, ReLU, 2x
 * average pooling, nearest upsampling, skip concatenation [upsampled, skip])
 * approximating the inverse of -h^2 L_h.  BF16 weights and activations, FP32
 * accumulation on the matrix cores, FP32 master weights and Adam.
 * Grids must be multiples of 8 per axis.
 *
 * ofdft_nn_create: He-normal weights from `seed`.
 * ofdft_nn_param_count: number of FP32 parameters (layer after layer, each
 *   W[t][ci][co] with tap t = (dz+1)*9 + (dy+1)*3 + (dx+1)).
 * ofdft_nn_set_weights / ofdft_nn_get_weights: host FP32 arrays of that size;
 *   get with gradients = 1 returns the last computed weight gradients.
 * ofdft_nn_reserve: allocate the workspace for one grid (done implicitly by
 *   forward/train calls; solves require it beforehand).
 * ofdft_nn_forward: out = scale * rms(in) * N(in / rms(in)) (device FP64).
 * ofdft_nn_gradients / ofdft_nn_train_step: for one pair (device FP64 g,
 *   phi) with t = phi / (h^2 rms g) and e = N(g / rms g) - t, the loss is
 *   kind 0: ||e||^2 / ||t||^2, kind 1 (energy norm): e^T A e / t^T A t,
 *   kind 2 (residual norm): ||A e||^2 / ||A t||^2, with A = -h^2 L_h (12th
 *   order); train_step also applies Adam (beta 0.9/0.999, eps 1e-8) with
 *   learning rate lr.  loss (host) may be NULL.
 * ofdft_nn_set_loss: choose the loss kind (0 default, 1, 2); INVALID_ARG else.
 * ofdft_poisson_set_network: attach a network to an OFDFT_LEARNED or
 *   OFDFT_LEARNED_REFINED solver (the solver keeps the pointer; the network
 *   must outlive its use).
 * ofdft_poisson_set_learned_mode: what the learned form does after the
 *   network's correction of the starting guess (x += a N(r) with the step a
 *   minimising the energy-norm error): precondition 0 (default) = plain FP64
 *   CG to the tolerance; 1 = flexible CG preconditioned by the network,
 *   falling back to plain CG from the best iterate when it stalls (less than
 *   10x residual reduction in 20 iterations) or breaks down.  OFDFT_LEARNED
 *   only (OFDFT_LEARNED_REFINED always continues with the refined form).
 * ------------------------------------------------------------------------ */
typedef struct ofdft_nn ofdft_nn;
int ofdft_nn_create(uint64_t seed, ofdft_nn **out);
int ofdft_nn_destroy(ofdft_nn *net);
size_t ofdft_nn_param_count(void);
int ofdft_nn_set_weights(ofdft_nn *net, const float *w, size_t count);
int ofdft_nn_get_weights(ofdft_nn *net, float *w, size_t count, int gradients);
int ofdft_nn_set_loss(ofdft_nn *net, int kind);
/* ofdft_nn_save / ofdft_nn_load: the network's training state in a file (FP32
 * weights, Adam moments and step count, loss kind, activation storage);
 * load repacks the kernels' weight copies, so training resumes exactly.
 * INVALID_ARG for an unreadable file or one of another network. */
int ofdft_nn_save(ofdft_nn *net, const char *path);
int ofdft_nn_load(ofdft_nn *net, const char *path);
/* ofdft_nn_set_precision: activation storage of the same kernels: 0 = BF16
 *   (default: BF16 activations, gradients and weight copies, FP32
 *   accumulation on v_mfma_f32_16x16x16 bf16), 1 = FP32 (FP32 activations,
 *   gradients and weight copies on v_mfma_f32_16x16x4 f32; for element-wise
 *   checks of the kernels against an FP64 reference).  The workspace is
 *   reallocated on the next forward / gradient call.  INVALID_ARG else. */
int ofdft_nn_set_precision(ofdft_nn *net, int fp32);
int ofdft_nn_reserve(ofdft_nn *net, const ofdft_grid *grid);
int ofdft_nn_forward(ofdft_nn *net, const ofdft_grid *grid, const double *in, double *out,
                     double scale, void *stream);
int ofdft_nn_gradients(ofdft_nn *net, const ofdft_grid *grid, const double *g, const double *phi,
                       double *loss, void *stream);
int ofdft_nn_train_step(ofdft_nn *net, const ofdft_grid *grid, const double *g, const double *phi,
                        double lr, double *loss, void *stream);
/* z = M r with the multigrid preconditioner of an OFDFT_MULTIGRID or
 * OFDFT_MULTIGRID_F64 solver (device FP64 arrays of the solver's grid, z != r);
 * INVALID_ARG for other modes. */
int ofdft_poisson_apply_preconditioner(ofdft_poisson *s, const double *r, double *z, void *stream);
int ofdft_poisson_set_learned_mode(ofdft_poisson *s, int precondition);
int ofdft_poisson_set_network(ofdft_poisson *s, ofdft_nn *net);

/* ------------------------------------------------------------------------
 * Launch configuration and accounting (not part of the method; used by the
 * tuner, the benchmark and the tests).
 *
 * ofdft_stencil_set_config: fix the stencil launch shape for one grid and
 *   element size (elem_bytes 4, 8 or 16), for every kernel family (it
 *   replaces the grid's tuned entries): shape 0 = 64x16 tile of 256 threads
 *   (4 rows per thread), 1 = 64x8 tile of 256, 2 = 32x16 tile of 256, 3 =
 *   64x16 tile of 512, 4 = 64x8 tile of 512, 5 = 64x32 tile of 512 (the plain
 *   FP64 and FP32 applies; 3 elsewhere); zlen = planes per z chunk (0 = automatic).
 *   shape < 0 removes the grid's entries.  INVALID_ARG for unknown shapes.
 * ofdft_batch_set_config: schedule of the shifted-system solver.  group 0
 *   (default) = stepped schedule: one launch per COCG phase over all systems,
 *   replayed from a HIP graph; group P in 1..1024 = persistent schedule, one
 *   cooperative launch in which groups of P workgroups solve whole systems.
 *   shape = stencil tile shape (as for ofdft_stencil_set_config), < 0 =
 *   automatic.
 * ofdft_profile_reset: clear the per-class launch counters; classes whose bit
 *   is set in timed_mask are timed with HIP events on their launch stream.
 *   Classes: 0 apply, 1 CG stencil pass, 2 CG vector update, 3 true-residual
 *   passes, 4 COCG stencil phases (the whole solve when persistent),
 *   5 density-update stencil passes, 6 density-update vector passes,
 *   7 Anderson, 8 other vector passes, 9 network kernels, 10 COCG vector
 *   phase (stepped schedule), 11 multigrid cycles on FP64 vectors (Poisson,
 *   density update), 12 multigrid cycles on complex128 vectors (shifted
 *   systems), 13 multi-shift COCG stencil phase, 14 multi-shift COCG vector
 *   phase.
 * ofdft_profile_read: launches, algorithmic bytes (each operand read once and
 *   each result written once), timed launches and their summed milliseconds
 *   for one class since the last reset (synchronises on pending events).
 * ------------------------------------------------------------------------ */
int ofdft_stencil_set_config(int nx, int ny, int nz, int elem_bytes, int shape, int zlen);

/* ------------------------------------------------------------------------
 * Autotuner of the launch configuration (not part of the method; it decides
 * how the Laplacian of Section 4 is tiled on the chip).  Every candidate
 * computes the same operator; the fused passes' reduction order follows the
 * tiling, so tuned and untuned runs agree to rounding, and runs with one
 * configuration are bitwise repeatable.
 *
 * ofdft_tune_stencil: times each legal (tile shape, z-chunk length) of one
 *   kernel family on `grid` (scratch vectors allocated and freed inside;
 *   `reps` timed launches after one warm-up, HIP events on `stream`) and
 *   records the fastest in the launch table for (grid, element size,
 *   family).  family OFDFT_TUNE_APPLY: fd_laplacian_apply, any dtype;
 *   OFDFT_TUNE_PASS: the fused single-pass stencil kernels (CG, residual and
 *   density-update passes), timed on the CG stencil pass, dtype F64 or F32.
 *   The untuned configuration is a candidate and is kept unless another is
 *   more than 2% faster.  Synchronises the stream.  INVALID_ARG, NO_MEMORY,
 *   HIP_ERROR.
 * ofdft_batch_tune: times `iters` COCG iterations of the batch's systems
 *   (kappa, rhs as for cg_helmholtz_solve_batched; x = starting guesses, read
 *   only: the runs use copies) for each stepped-schedule tile shape and
 *   z-chunk target (40, 80, 160 planes) and, without a preconditioner, the
 *   persistent schedule with 16 and 64 workgroups per group; sets the
 *   fastest as the batch's configuration.
 * out (optional): shape id, zlen (z-chunk length; for a batch the z-chunk
 *   target, planes), group (batch: persistent group size, 0 = stepped),
 *   candidates timed, best_ms and default_ms (per launch; per solve of
 *   `iters` iterations for a batch) of the choice and of the untuned
 *   configuration.
 * ofdft_tune_save / ofdft_tune_load: the launch table as text (one entry per
 *   line: family nx ny nz elem_bytes shape zlen; family -1 = set by hand for
 *   every family); load adds entries (count in *entries, may be NULL).
 * ------------------------------------------------------------------------ */
#define OFDFT_TUNE_APPLY 0
#define OFDFT_TUNE_PASS  1
typedef struct {
    int shape, zlen, group, candidates;
    double best_ms, default_ms;
} ofdft_tune_result;
int ofdft_tune_stencil(const ofdft_grid *grid, int radius, ofdft_dtype dtype, int family, int reps,
                       ofdft_tune_result *out, void *stream);
int ofdft_batch_tune(ofdft_batch *b, const double *kappa, const void *const *rhs, const void *const *x,
                     int iters, ofdft_tune_result *out, void *stream);
int ofdft_tune_save(const char *path);
int ofdft_tune_load(const char *path, int *entries);
int ofdft_batch_set_config(ofdft_batch *b, int shape, int group);
int ofdft_profile_reset(unsigned timed_mask);
int ofdft_profile_read(int cls, int64_t *launches, double *bytes, int64_t *timed, double *ms);

#ifdef __cplusplus
}
#endif
#endif /* OFDFT_H */
