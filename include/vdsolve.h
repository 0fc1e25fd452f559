/*
 * vdsolve -- preconditioned Krylov solves of the variable-density elliptic
 * systems of a semi-implicit pseudo-spectral scheme, on AMD MI355X (gfx950).
 *
 * The operations follow Reynier, Di Pierro, Alizard, Cadiou, Le Penven and
 * Buffat, "A preconditioning for the spectral solution of incompressible
 * variable-density flows":
 *
 *   pressure   L_rho p = div(rho^-1 grad p) = f     (eq. VDINSE.Lrho, and its
 *              time-discrete form eq. VDINSE.Lrho.num), periodic boundaries,
 *              zero-mean gauge (Sec. 4.2);
 *   velocity   rho u - dt_nu Lap u = g               (the implicit viscous
 *              step of eq. VDINSE.num.momentum.proj with the mass-diffusion
 *              terms dropped);
 *   solvers    GMRES(m), conjugate gradient, Richardson minimal residual
 *              (Sec. 3.1), each optionally preconditioned by the exact
 *              inverse of the constant-density operator (Sec. 3
 *              introduction, Sec. 3.2, Sec. 4.2).
 *
 * Conventions (all entry points):
 *   - Grids are Fourier (periodic) on every axis; n[0] = nx is the
 *     contiguous axis.  Physical fields are real FP64 arrays in C order
 *     [nz][ny][nx] (2D: [ny][nx]; 1D: [nx]) with x_j = j L / n.
 *   - Exception: a 2D grid may have basis[1] = VD_CHEB_GL, a wall-normal
 *     axis on the n[1] Chebyshev-Gauss-Lobatto points z_j = cos(pi j /
 *     (n[1]-1)) of [-1, 1] (row 0 is z = +1; length[1] is ignored) with
 *     Neumann walls (Sec. 3, C-F-F decomposition).  Its pressure system is
 *     the Galerkin weak form (Legendre-Gauss-Lobatto quadrature of the
 *     interpolant): A p = b with b = -I^T W I f, A symmetric positive
 *     semi-definite; residuals are measured on that system.  Helmholtz
 *     solves are not available on such grids.
 *   - Every field pointer is DEVICE memory, owned by the caller, valid for
 *     the duration of the call.  The library keeps no pointer to it.
 *   - Work is enqueued on the stream given at grid creation; each call
 *     returns after that work has completed.  A grid handle must not be
 *     used by two threads at once; different handles are independent.
 *   - Status codes: VD_OK = 0; VD_NOT_CONVERGED = 1 is a warning (the best
 *     iterate is written and info is filled); negative codes are errors and
 *     leave outputs unspecified, except that the info of vd_solve_pressure,
 *     vd_solve_helmholtz and vd_solve_pressure_batch, when given, carries
 *     the status (also for arguments rejected before any work).  No C++
 *     exception crosses this interface.
 */
#ifndef VDSOLVE_H
#define VDSOLVE_H

#include <stddef.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VD_OK = 0,
  VD_NOT_CONVERGED = 1,
  VD_EINVAL = -1,     /* bad argument (null pointer, size, option) */
  VD_ENOMEM = -2,     /* device allocation failed */
  VD_EDOMAIN = -3,    /* density not strictly positive and finite */
  VD_EBREAKDOWN = -4, /* non-finite Krylov scalar or residual (also from a non-finite
                         right-hand side or initial iterate) */
  VD_EDEVICE = -5,    /* HIP runtime error */
  VD_ETOOBIG = -6,    /* request larger than a serving budget */
  VD_ENOTSUP = -7     /* valid but not implemented */
} vd_status;

typedef enum { VD_FOURIER = 0, VD_CHEB_GL = 1 } vd_basis;
typedef enum { VD_GMRES = 0, VD_CG = 1, VD_RMR = 2 } vd_solver;
typedef enum { VD_FP64 = 0, VD_FP32_REFINE = 1 } vd_precision;
typedef enum { VD_OP_PRESSURE = 0, VD_OP_HELMHOLTZ = 1, VD_OP_PRESSURE_K = 2 } vd_op_kind;
/* Pressure formulation (Sec. 3.2; the 3D choice of Sec. 4.2): L_rho phi = f directly, or the modified
 * form K_rho Phi = sqrt(rho) f with Phi = phi / sqrt(rho) (eq. VDINSE.Krho). */
typedef enum { VD_FORM_L = 0, VD_FORM_K = 1 } vd_pressure_form;

typedef struct {
  int ndim;         /* 1, 2 or 3 */
  int n[3];         /* points per axis, n[0] = nx (contiguous): powers of two,
                       16 <= n <= 1024 (Fourier); 9..513 (Chebyshev) */
  int basis[3];     /* VD_FOURIER, or VD_CHEB_GL on axis 1 of a 2D grid */
  double length[3]; /* period of each axis (> 0) */
} vd_grid_desc;

typedef struct {
  int solver;        /* vd_solver */
  int restart;       /* GMRES restart length m, 1..32 (default 30) */
  double rtol;       /* stop when ||b - A x||_2 / ||b||_2 <= rtol (default 1e-10) */
  int max_iter;      /* cap on operator applications in the Krylov loop */
  int precond;       /* 1: constant-density inverse as preconditioner; 0: none */
  int precision;     /* vd_precision */
  double inner_rtol; /* FP32_REFINE: relative tolerance of each inner FP32 solve
                        (GMRES inner solves also stop after 3 cycles of `restart`
                        steps; CG and RMR inner solves only at this tolerance or
                        at the remaining max_iter budget) */
  int max_outer;     /* FP32_REFINE: cap on refinement steps */
  double rho0;       /* preconditioner density; NaN = mean of rho */
  int use_x0;        /* 1: the output array holds the initial guess on entry */
  int formulation;   /* pressure solves: vd_pressure_form (default VD_FORM_L) */
  double* history;   /* optional host array for the residual history (default NULL) */
  int history_cap;   /* its length in doubles (default 0: no history) */
} vd_solve_opts;
/* Residual history (the convergence curves of Secs. 3.1, 4.3): entry 0 is
 * ||r_0|| / ||b||, then one entry per Krylov iteration with the method's own
 * residual: GMRES the Givens estimate |g_(j+1)| / ||b|| (restarts add no
 * entry), CG and RMR the recursively updated ||r|| / ||b||.  FP32_REFINE:
 * the FP64 true residual before and after each refinement step.  Several
 * components (vd_solve_helmholtz): component 0.  Batched 1D solves
 * (vd_visc1d_solve): history_cap entries per system, rows one after another.
 * At most history_cap entries are written; info->history_len says how many
 * (for the batched solver: the longest row; row k holds iterations[k] + 1). */

typedef struct {
  int status;            /* same as the return value */
  int iterations;        /* operator applications inside the Krylov loops */
  int refinements;       /* outer FP64 steps (FP32_REFINE), else 0 */
  double rel_residual;   /* true FP64 ||b - A x|| / ||b|| at exit (max over components) */
  double rhs_null_norm;  /* pressure: norm of the removed nullspace part of f */
  double seconds;        /* wall time of the solve on the host clock */
  int gs_second_passes;  /* GMRES: steps whose Gram-Schmidt needed a second pass */
  int history_len;       /* entries written to opts->history */
} vd_solve_info;

typedef struct vd_grid vd_grid;

/* Fill opts with the defaults: GMRES(30), rtol 1e-10, max_iter 2000,
 * precond 1, FP64, inner_rtol 1e-5, max_outer 10, rho0 = NaN, use_x0 0,
 * formulation VD_FORM_L. */
void vd_default_opts(vd_solve_opts* opts);

/* Create a grid and its device resources on `stream` (0 = null stream).
 * Errors: VD_EINVAL (sizes, lengths, basis), VD_ENOMEM, VD_EDEVICE. */
vd_status vd_grid_create(vd_grid** out, const vd_grid_desc* desc, hipStream_t stream);
vd_status vd_grid_destroy(vd_grid* grid);

/* Copy the density rho (device, [nz][ny][nx] FP64) into the grid and derive
 * a = 1/rho (FP64 and FP32 copies) and rho0 = mean(rho).  Every later
 * operator, preconditioner and solve uses it (rho enters L_rho through
 * a = 1/rho, eq. VDINSE.Lrho).  Errors: VD_EDOMAIN if any rho <= 0 or not
 * finite (the grid keeps no density then), VD_EINVAL. */
vd_status vd_set_density(vd_grid* grid, const double* rho);

/* y = A x for the operator `kind` (physical in, physical out, device FP64):
 * VD_OP_PRESSURE: A = -L_rho (symmetric positive semi-definite);
 * VD_OP_HELMHOLTZ: A = rho - dt_nu Lap;
 * VD_OP_PRESSURE_K: A = -K_rho = -Lap - c, c = Lap(rho)/(2 rho)
 *   - 3/4 |grad rho|^2 / rho^2 (eq. VDINSE.Krho), evaluated as
 *   c = -Lap(psi)/psi with psi = rho^-1/2 so that psi is an exact null vector
 *   (Lap spectral, Nyquist kept; dt_nu ignored; Fourier grids only).
 * precision VD_FP32_REFINE evaluates the operator in FP32 (spectral vectors
 * and coefficients rounded to FP32).  Used for per-kernel parity and timing. */
vd_status vd_apply_operator(vd_grid* grid, int kind, int precision, double dt_nu, const double* x, double* y);

/* z = M^-1 r with M the constant-density operator at rho0 (NaN = mean rho):
 * pressure: the pseudo-inverse (zero on the nullspace); Helmholtz: the
 * inverse of rho0 - dt_nu Lap; VD_OP_PRESSURE_K: the pseudo-inverse of -Lap
 * (zero on the constant mode; rho0 and dt_nu ignored). */
vd_status vd_apply_precond(vd_grid* grid, int kind, int precision, double dt_nu, double rho0, const double* r,
                           double* z);

/* Solve L_rho p = f (Sec. 3.2).  f: device FP64 physical values; p:
 * device FP64 output (also the initial guess if opts->use_x0).  f is
 * projected onto the range of the operator (its components on the
 * nullspace -- the modes whose wavenumber along every axis is 0 or n/2 --
 * are removed and their norm reported in info->rhs_null_norm); the
 * solution returned is the one orthogonal to that nullspace (zero mean).
 * The residual is measured in the Euclidean norm of grid values.
 * With opts->formulation = VD_FORM_K (eq. VDINSE.Krho of Sec. 3.2; Fourier
 * grids, as the paper uses it in 3D in Sec. 4.2) the solve
 * runs on Phi = p / sqrt(rho): A = -K_rho, b = -sqrt(rho) f with its
 * component along rho^-1/2 removed (that norm goes to rhs_null_norm), the
 * preconditioner is the pseudo-inverse of -Lap, info->rel_residual is that
 * system's; p = sqrt(rho) Phi is returned with zero mean (removing a
 * constant from p removes a multiple of rho^-1/2, a null vector, from Phi);
 * modulo the checkerboard modes, which L_rho does not see, it agrees with
 * the direct form's solution up to discretisation error.
 * opts == NULL means defaults; info may be NULL.  VD_ENOTSUP: VD_FORM_K on
 * a Chebyshev grid. */
vd_status vd_solve_pressure(vd_grid* grid, const double* f, double* p, const vd_solve_opts* opts,
                            vd_solve_info* info);

/* Solve L_rho p = f on n <= 3 grids of one shape together, each with its own
 * density (Sec. 3.2; grids[k], f[k], p[k] as in vd_solve_pressure; infos:
 * n entries, filled for every grid).  With GMRES on a Fourier grid of two or
 * three dimensions (direct form) the solves share their launches: one per
 * operator pass and per Gram-Schmidt kernel for all of them, each grid
 * keeping its own Krylov state and stopping test; a grid that has converged
 * skips its part of the launches.  Otherwise the grids are solved one after
 * another.  Either way every grid's p and info are bit for bit those of
 * vd_solve_pressure on that grid alone (info.seconds aside: the batch's
 * wall time; the history, if requested, is grid 0's).  The work runs on
 * grids[0]'s stream; the other grids must not be in use by another thread.
 * Returns the worst status (errors before VD_NOT_CONVERGED); infos[k].status
 * is grid k's own.  VD_EINVAL: n outside [1, 3] or infos NULL (nothing
 * written), a NULL pointer, a grid without a density or given twice (every
 * info's status set to it). */
vd_status vd_solve_pressure_batch(vd_grid* const* grids, int n, const double* const* f, double* const* p,
                                  const vd_solve_opts* opts, vd_solve_info* infos);

/* Solve rho u - dt_nu Lap u = g for ncomp independent components stored one
 * after another (g, u: [ncomp][nz][ny][nx]).  Lap keeps the Nyquist modes.
 * dt_nu >= 0.  info->iterations sums the components, rel_residual is the
 * largest component residual. */
vd_status vd_solve_helmholtz(vd_grid* grid, double dt_nu, int ncomp, const double* g, double* u,
                             const vd_solve_opts* opts, vd_solve_info* info);

/* Device bytes the grid plus one solve with these options needs (the
 * serving admission test uses it).  Returns 0 for an invalid descriptor or
 * invalid options; opts == NULL means defaults. */
size_t vd_workspace_bytes(const vd_grid_desc* desc, const vd_solve_opts* opts);

/* The same for vd_solve_helmholtz with ncomp components.  With GMRES on a
 * Fourier grid of two or three dimensions, up to three components are
 * solved together (one launch per operator pass and per Gram-Schmidt kernel
 * for all of them), each with its own Krylov vectors; their results are
 * those of separate solves.  Otherwise equal to vd_workspace_bytes.
 * Returns 0 where vd_workspace_bytes does, or for ncomp < 1. */
size_t vd_workspace_bytes_helmholtz(const vd_grid_desc* desc, const vd_solve_opts* opts, int ncomp);

/* Time spent in each hot kernel since the last read, measured with HIP
 * events on the grid's stream while enabled.  Classes 0..4: the pressure
 * operator's z-first, y-inverse, x, y-forward and z-last passes; 5..9: the
 * same passes of the Helmholtz operator; 10: the GMRES Gram-Schmidt dot
 * pass; 11: the GMRES Gram-Schmidt update pass.  ms[c] = total
 * milliseconds, count[c] = launches, bytes[c] = algorithmic bytes those
 * launches read and wrote (3D grids), for c < nclass (<= 12); any output
 * pointer may be NULL.  Reading resets the totals.  `classes` is a bit mask
 * of the classes to time (bit c = class c; -1 times all, 0 disables); each
 * timed launch adds an event pair on the grid's stream.  A Krylov step that
 * the solver queued past the end of a run does nothing, and its launches are
 * not counted. */
vd_status vd_profile_enable(vd_grid* grid, int classes);
vd_status vd_profile_read(vd_grid* grid, double* ms, long long* count, double* bytes, int nclass);

const char* vd_status_string(vd_status s);

/* C = A B for row-major device matrices A [M][K], B [K][N], C [M][N] in FP64
 * (precision VD_FP64) or FP32 (VD_FP32_REFINE): the MFMA contraction the
 * Chebyshev direction uses (its differentiation, interpolation and
 * eigenbasis products, Sec. 3 C-F-F).  Runs on `stream` and returns after
 * completion. */
vd_status vd_dense_matmul(int precision, const void* A, const void* B, void* C, int M, int N, int K,
                          hipStream_t stream);

/* ------------------------------------------------------------------------
 * One-dimensional implicit viscous systems (Sec. 3.1): batches of
 *     V_rho u = u - (a / rho)(D2 u + rho'' u + rho' D1 u) = b
 * (eq. VDINSE.Vrho, a = dt / (2 Re), Sc = 1), right-preconditioned by the
 * constant-density operator V = I - a D2 (eq. VDINSE.V), with rho' = D1 rho
 * and rho'' = D2 rho.  Basis VD_CHEB_GL: n Chebyshev-Gauss-Lobatto points of
 * [-1, 1] (descending), D1 the collocation matrix, D2 = D1 D1, no-slip walls
 * u(+-1) = 0 (the interior rows are solved; b's wall values are ignored and
 * u's are returned as 0).  Basis VD_FOURIER: n (even) periodic points of
 * [0, length), D1 the spectral derivative with its Nyquist mode zeroed, D2
 * with it kept.  One workgroup solves each group of 16 systems of a batch
 * in lockstep (the shared matrices applied to the group with FP64 MFMA);
 * a system's result does not depend on the rest of the batch.
 * ---------------------------------------------------------------------- */
typedef struct vd_visc1d vd_visc1d;

/* Build the matrices (long double on the host, FP64 on the device) for n
 * points (Chebyshev 9..512; Fourier even, 16..512) and a > 0.  Errors:
 * VD_EINVAL, VD_ENOMEM. */
vd_status vd_visc1d_create(vd_visc1d** out, int basis, int n, double length, double a, hipStream_t stream);

/* The pressure operators of the one-dimensional Chebyshev-collocation study
 * of Sec. 3.2 (Figs. 5-7) on the same batched solver:
 *     form VD_FORM_L:  L_rho u = (1/rho) D2 u - (rho'/rho^2) D1 u
 *                      (eq. VDINSE.Lrho, expanded; rho' = D1 rho),
 *     form VD_FORM_K:  K_rho u = D2 u + c u,  c = -D2 psi / psi with
 *                      psi = rho^-1/2 (eq. VDINSE.Krho; by the chain rule the
 *                      printed c, in a form that makes psi an exact null
 *                      vector),
 * on the n Chebyshev-Gauss-Lobatto points of [-1, 1] (descending) with
 * Neumann walls (Sec. 3.2: d(rho)/dn = d(phi)/dn = 0): the unknowns are the
 * n - 2 interior values, the wall values are those that zero the
 * collocation derivative at both walls (D1 and D2 above include that
 * extension), and the equations are the interior collocation rows.  The
 * preconditioner is the Moore-Penrose pseudo-inverse of the Neumann
 * Laplacian D2 (the inverse of K_rho at constant density; it annihilates
 * the constants).  Both operators are singular (null vectors: constants for
 * L_rho, psi for K_rho), so a right-hand side must lie in the range of the
 * operator, else its component outside the range remains in the residual.
 * The handle is used with vd_visc1d_apply, vd_visc1d_solve,
 * vd_visc1d_solve_noalloc, vd_visc1d_kernel_ms and vd_visc1d_destroy: b's
 * wall values are ignored; solutions and preconditioned vectors carry the
 * wall values of the Neumann extension; operator outputs (equation rows)
 * have zero walls.  n: 9..512.  Errors: VD_EINVAL, VD_ENOMEM, VD_EDEVICE. */
vd_status vd_pres1d_create(vd_visc1d** out, int n, int form, hipStream_t stream);
vd_status vd_visc1d_destroy(vd_visc1d* h);

/* y = A u (precond 0) or y = M^-1 u (precond 1) for `batch` systems, A the
 * handle's operator (V_rho, L_rho or K_rho) and M^-1 its preconditioner;
 * rho, u, y: device FP64 [batch][n].  VD_EDOMAIN if a density is not
 * strictly positive and finite. */
vd_status vd_visc1d_apply(vd_visc1d* h, int batch, const double* rho, const double* u, double* y, int precond);

/* Solve the batch: rho, b: device FP64 [batch][n]; u: device output (initial
 * guess if opts->use_x0).  opts: solver VD_GMRES (restart 1..128), VD_RMR or
 * VD_CG (preconditioned conjugate gradient, run as the paper runs it on
 * these non-symmetric operators; VD_FP32_REFINE gives VD_ENOTSUP), rtol on
 * each system's true relative residual ||b - A u|| / ||b|| over the
 * unknowns, max_iter, precond.  Per-system iterations and relative residuals
 * go to the host arrays when given; info gets the largest of each and the
 * worst status.  The workspace (per group of 16 systems: 16 (5 + restart
 * + 1) rows padded to 64 plus the Hessenberg and rotation arrays, GMRES; 80
 * rows, RMR; 96 rows, CG) is kept by the handle for later calls. */
vd_status vd_visc1d_solve(vd_visc1d* h, int batch, const double* rho, const double* b, double* u,
                          const vd_solve_opts* opts, int* iterations, double* rel_residual, vd_solve_info* info);
/* The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the workspace, per-system outputs and residual histories live in a static
 * device array of VD_NOALLOC_SCRATCH_BYTES that the library holds on every
 * GPU it runs on until the process ends, so the call allocates nothing (the
 * handle, created beforehand, holds the matrices).  It needs
 *   ceil(batch / 16) x per-group workspace (16 (5 + restart + 1) rows padded
 *   to 64 doubles plus the Hessenberg and rotation arrays, GMRES; 80 rows,
 *   RMR; 96 rows, CG) + batch (4 + 8 + 4 + 8 history_cap) bytes, each part rounded up to
 *   256 bytes;
 * e.g. 256 unknowns, GMRES(30): 816 systems; RMR: 6528.  A larger call
 * returns VD_ETOOBIG and does nothing.  Results, iterations and histories are
 * those of vd_visc1d_solve (same kernel).  All calls on one GPU share its
 * array, which keeps the last call's contents: two calls that overlap in time
 * on one GPU (other threads, other streams) race and give undefined results.
 * Histories are cleared with a kernel, not a memset. */
#define VD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
vd_status vd_visc1d_solve_noalloc(vd_visc1d* h, int batch, const double* rho, const double* b, double* u,
                                  const vd_solve_opts* opts, int* iterations, double* rel_residual,
                                  vd_solve_info* info);
/* Duration in ms of the last apply or solve kernel, from HIP events recorded
 * on the handle's stream immediately before and after its launch (0 before
 * any call, -1 if the events could not be read). */
vd_status vd_visc1d_kernel_ms(const vd_visc1d* h, double* ms);

/* ------------------------------------------------------------------------
 * Fractional-step time integration of the variable-density incompressible
 * Navier-Stokes equations (Sec. 2, eq. VDINSE) on the triply periodic box
 * [0, 2 pi)^3 with n^3 points (n a power of two, 16..512).  One step:
 * Adams-Bashforth advection terms (Euler on the first step after a state is
 * set), Crank-Nicolson density (eq. VDINSE.num.mass.proj), rho^(n+1/2) the
 * mean of the two densities, the implicit viscous system
 * u* - dt/2 zeta(rho^(n+1/2), u*) = rhs (eq. VDINSE.num.momentum.proj, zeta
 * of eq. VDINSE.zeta) by GMRES preconditioned with (I - dt/(2 Re) Lap)^-1
 * (eq. VDINSE.V) from u^n, L_rho phi = div(u*) / dt by vd_solve_pressure
 * warm-started from the previous phi (eq. VDINSE.Lrho.num), the projection
 * u^(n+1) = u* - dt grad(phi) / rho^(n+1/2) (eq. VDINSE.num.proj) and the
 * pressure update of eq. VDINSE.num.p.update (its Lap^-1 is the
 * pseudo-inverse of div grad).  Derivatives are spectral (first derivatives
 * with the Nyquist mode zeroed, the Laplacian with it kept).  With s > 0 the
 * body force and mass source that make the Taylor-Green solution of
 * eq. VDINSE.solexact (density ratio s) exact are added at t^(n+1/2).
 * Fields: device FP64, velocity [3][n][n][n] (components along x, y, z),
 * scalars [n][n][n], x contiguous.  All work runs on the handle's stream.
 * ---------------------------------------------------------------------- */
typedef struct vd_ns vd_ns;

typedef struct {
  double re, sc;      /* Reynolds and Schmidt numbers (> 0) */
  double dt;          /* time step (> 0) */
  double s;           /* > 0: manufactured forcing with density ratio s; 0: none */
  double visc_rtol;   /* viscous solve: relative true residual (default 1e-12) */
  double pres_rtol;   /* pressure solve: relative true residual (default 1e-12) */
  int restart;        /* GMRES restart of both solves, 1..30 (default 30) */
  int max_iter;       /* per solve (default 2000) */
  int pres_solver;    /* pressure solve: VD_GMRES (default), VD_CG or VD_RMR */
  int pres_form;      /* pressure solve: VD_FORM_L (default) or VD_FORM_K (eq. VDINSE.Krho) */
} vd_ns_params;

typedef struct {
  double t;                  /* time after the last step */
  int steps;                 /* steps since the state was set */
  int visc_iters, pres_iters;            /* Krylov iterations of the last step */
  int visc_status, pres_status;          /* vd_status of the last step's solves */
  double visc_rel_residual, pres_rel_residual;
  double pres_seconds;       /* host wall time of the last step's pressure solve */
} vd_ns_info;

void vd_ns_default_params(vd_ns_params* p);
/* VD_EINVAL for bad sizes or parameters; VD_ENOMEM.  The handle holds
 * 65 + 3 (restart + 1) fields of n^3 doubles (2.7 GB at 128^3 with
 * restart 30, 21 GB at 256^3) and a pressure grid. */
vd_status vd_ns_create(vd_ns** out, int n, const vd_ns_params* prm, hipStream_t stream);
vd_status vd_ns_destroy(vd_ns* h);
/* Copy u^n, rho^n and p^(n-1/2) (device arrays) in and set the time; the
 * advection history and the pressure warm start are reset. */
vd_status vd_ns_set_state(vd_ns* h, const double* u, const double* rho, const double* p, double t);
/* The state of eq. VDINSE.solexact at t = 0 with p^(-1/2) = p_e(-dt/2)
 * (requires s > 0). */
vd_status vd_ns_init_taylor_green(vd_ns* h);
/* Advance nsteps steps; info (may be NULL) describes the last one.
 * Returns the worse of the last step's solve statuses. */
vd_status vd_ns_step(vd_ns* h, int nsteps, vd_ns_info* info);
/* Copy the state out (device arrays; any may be NULL). */
vd_status vd_ns_get_state(vd_ns* h, double* u, double* rho, double* p, double* t);
/* err[0..3] = RMS over the grid of |u - u_e(t)|, p - p_e(t - dt/2),
 * rho - rho_e(t) (eq. VDINSE.solexact) and div u (requires s > 0). */
vd_status vd_ns_errors(vd_ns* h, double* err);
/* The projection of Sec. 2, P_rho(u) = u - grad(phi) / rho with
 * L_rho phi = div u (eq. VDINSE.Lrho.num without the 1/dt): an exact
 * projection onto the (discretely) divergence-free fields, P_rho(P_rho(u)) =
 * P_rho(u).  rho: device [n^3] (> 0); u, out: device [3][n^3] (out may equal
 * u); the pressure solve uses the handle's pres_rtol, restart and max_iter
 * and reports in info (may be NULL).  Uses the handle's scratch, not its
 * state. */
vd_status vd_ns_project(vd_ns* h, const double* rho, const double* u, double* out, vd_solve_info* info);
/* Optional timing of the handle's work with HIP events on its stream, by
 * class: 0 the FFT transforms (algorithmic bytes 48 n^3 each: three passes
 * reading and writing the field), 1 the pressure solves, 2 the viscous
 * solve's inner products and updates.  Enabling resets the totals; reading
 * returns milliseconds, launch counts and bytes per class. */
vd_status vd_ns_profile_enable(vd_ns* h, int on);
vd_status vd_ns_profile_read(vd_ns* h, double* ms, long long* count, double* bytes, int nclass);

/* ------------------------------------------------------------------------
 * Continuous-batching solve server.  Not in the paper: a serving front end
 * for many independent solves of the kinds above (different grid sizes and
 * densities).  Requests are queued FIFO and admitted as soon as a worker
 * slot is free and their HBM footprint (vd_workspace_bytes) fits the budget
 * next to the grids already held; admitted requests run concurrently, each
 * slot on its own stream, with their Krylov state resident on the device.
 * Pressure requests that can share launches (GMRES, direct form, Fourier
 * grids of two or three dimensions) are batched: when a slot takes such a
 * request while more requests wait than slots are free, up to two later
 * queued requests of the same shape and options (no history) join it if
 * grids for them fit without releasing others, and the slot solves them
 * together (vd_solve_pressure_batch; each still on its own grid, charged as
 * before).  A result does not depend on what else is
 * running or on its batch (fixed launch configurations and reduction
 * orders).
 * ---------------------------------------------------------------------- */
typedef struct vd_server vd_server;

typedef struct {
  vd_grid_desc desc;   /* grid of this request */
  int kind;            /* VD_OP_PRESSURE or VD_OP_HELMHOLTZ */
  double dt_nu;        /* Helmholtz coefficient */
  int ncomp;           /* Helmholtz components (0 or 1 = one) */
  const double* rho;   /* device density, caller-owned until its result is returned */
  const double* f;     /* device right-hand side */
  double* x;           /* device output (initial guess if opts.use_x0); rho, f and x
                          must be ready before submit (the server's streams are not
                          ordered after any of the caller's) and stay allocated until
                          the result is returned */
  vd_solve_opts opts;
  unsigned long long user_tag;
} vd_request;

typedef struct {
  unsigned long long ticket, user_tag;
  int status, iterations, refinements, slot;
  double rel_residual;
  double t_arrive, t_start, t_done; /* seconds since the server was created */
} vd_result;

typedef struct {
  long long queued, in_flight;
  int busy_slots, grids;
  size_t hbm_used, hbm_peak;
  int peak_busy_slots;
} vd_server_stats_t;

/* Start a server with an HBM budget (bytes) and max_slots concurrent solves
 * (1..64).  Errors: VD_EINVAL, VD_ENOMEM. */
vd_status vd_server_create(vd_server** out, size_t hbm_budget, int max_slots);
/* Same scheduler without device work (each request "runs" for the given
 * seconds and returns VD_ENOTSUP): lets the admission policy be tested on a
 * machine without a GPU. */
vd_status vd_server_create_dry(vd_server** out, size_t hbm_budget, int max_slots, double seconds_per_request);
/* Requests per shared batch, 1..3 (default 3; 1 = every request alone in
 * its slot).  Applies to batches formed after the call.  VD_EINVAL outside
 * that range. */
vd_status vd_server_set_batch(vd_server* s, int max_requests);
/* Queue a request; never blocks.  VD_ETOOBIG if its footprint exceeds the
 * whole budget, VD_EINVAL for a bad descriptor/options/pointers. */
vd_status vd_server_submit(vd_server* s, const vd_request* req, unsigned long long* ticket);
/* Move up to cap finished results into out (non-blocking); *n = count. */
vd_status vd_server_poll(vd_server* s, vd_result* out, int cap, int* n);
/* As poll, but first waits up to timeout_s for a result (or until idle). */
vd_status vd_server_wait(vd_server* s, vd_result* out, int cap, int* n, double timeout_s);
vd_status vd_server_stats(vd_server* s, vd_server_stats_t* st);
/* Finish running requests, drop queued ones, release everything. */
vd_status vd_server_destroy(vd_server* s);

#ifdef __cplusplus
}
#endif

#endif /* VDSOLVE_H */
