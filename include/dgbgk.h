/*
 * dgbgk.h -- C ABI of the MI355X (gfx950) nodal discontinuous-Galerkin
 * discrete-Boltzmann BGK solver.
 *
 * Method: Ganeshan & Williams, "A finite element discrete Boltzmann method for
 * high Knudsen number flows" (arXiv:2012.13487).  The library advances the
 * semi-discrete system obtained from the discrete Boltzmann equation with BGK
 * collision (Sec. II.A, eq. (6)) discretised by nodal DG (Sec. II.B, eq. (10))
 * with an upwind numerical flux, Maxwell diffuse-reflection walls (eq. (8),
 * imposed through the exterior state as in Sec. II.B "Implementation of
 * boundary conditions"), and explicit classical RK4 in time (the conclusion,
 * Sec. IV, allows explicit RK of any order).
 *
 * Conventions (all calls):
 *   - uniform Cartesian quadrilaterals, element k = ex + nx*ey, ex in [0,nx),
 *     ey in [0,ny); (p+1)^2 Gauss-Lobatto-Legendre nodes per element, node
 *     n = i + (p+1)*j, i along x, j along y;
 *   - host arrays of the distribution function (set_state, get_state, rhs,
 *     wall_density) are f[q][k][n], velocity-major, FP64; on the device the
 *     library keeps f element-major, f[k][q][n] (the Q velocity rows of an
 *     element, each Np contiguous nodes, are consecutive), so that the tile of
 *     one element streams as a single contiguous block;
 *   - sides / faces: 0 bottom (y = y0), 1 right (x = x0+lx), 2 top
 *     (y = y0+ly), 3 left (x = x0); face nodes ordered by increasing i or j;
 *   - 2-D tensor velocity sets: q = a + m*b with e_q = (x_a, x_b).
 *
 * Errors: every call returns a dgbgk_status (0 = success).  Calls that take a
 * solver record a message readable with dgbgk_last_error(); a NULL solver
 * returns DGBGK_EINVAL.  No exceptions cross the ABI.
 *
 * Ownership: the library copies every input array at the call; output arrays
 * are owned by the caller and must hold the stated number of elements.
 * Device memory is owned by the library unless the caller hands it a region
 * with dgbgk_bind_buffers(), which the caller then keeps alive until
 * dgbgk_destroy().
 *
 * Streams: device work is enqueued on the HIP stream given at create (NULL =
 * the null stream).  dgbgk_step() and dgbgk_residual_async() only enqueue;
 * calls that return host data synchronise the stream.
 *
 * Threads: a solver handle must be used by one host thread at a time.
 */
#ifndef DGBGK_H
#define DGBGK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dgbgk_solver dgbgk_solver;

typedef enum {
  DGBGK_OK = 0,
  DGBGK_EINVAL = -1,     /* invalid argument (message in dgbgk_last_error)   */
  DGBGK_ENOMEM = -2,     /* host or device allocation failed                 */
  DGBGK_EDEVICE = -3,    /* HIP runtime error or no usable gfx950 device     */
  DGBGK_ENONFINITE = -4, /* the state or its right-hand side is not finite   */
  DGBGK_ESTATE = -5,     /* call out of order (e.g. stepping before init)    */
  DGBGK_ENOTSUP = -6     /* valid request the library does not implement     */
} dgbgk_status;

typedef enum { DGBGK_BC_PERIODIC = 0, DGBGK_BC_DIFFUSE_WALL = 1 } dgbgk_bc;

/* Arithmetic of the time step.
 *   DGBGK_FP64: every value FP64.
 *   DGBGK_FP32: the state is stored and streamed in FP32 as the deviation
 *     g = f - w_q rho_ref (rho_ref = 1) from the rest equilibrium; the
 *     volume term, lifted jumps, collision and RK update run in FP32, the node
 *     moments rho, rho u, the diffuse-wall densities of eq. (8) and the wall
 *     exterior states are formed in FP64, and so is the residual.  Host
 *     arrays stay FP64 f (converted on the device).
 *   DGBGK_FP32_BF16MMA: as DGBGK_FP32, with the volume term's contractions
 *     Dr g, Ds g on bf16 matrix cores with FP32 accumulation (DGBGK_ENOTSUP
 *     where the library has no such kernel).
 *   DGBGK_FP32_REF: the reference form.  The state is f = f_r + g with an FP64
 *     reference f_r (not streamed by the stages) and an FP32 correction g in
 *     the RK registers.  The transport part of the right-hand side (volume
 *     term, upwind jumps, and the diffuse-wall exterior state, whose density
 *     of eq. (8) is linear in the outgoing values) is linear, so
 *     L(f_r + g) = L(f_r) + T(g) - g/tau + [f^eq(m_r + m_g) - f^eq(m_r)]/tau
 *     (eq. (5), (6); m = node moments): L(f_r) is evaluated in FP64 when the
 *     reference is set and streamed in FP32, the node moments are reduced in
 *     FP64, and the difference of equilibria is formed from the moment
 *     increments with FP64 node factors.  Every FP32 quantity is then
 *     rounded relative to the correction or to the current rate, which both
 *     vanish at a steady state, so the path reaches the steady-state
 *     residuals FP64 reaches while streaming FP32 (plus L(f_r): 21 bytes per
 *     DOF and stage on average against 32 for FP64).  dgbgk_fold() moves g
 *     into f_r; a caller folds from time to time (e.g. at every residual
 *     check) to keep g small.  p <= 4.
 *   DGBGK_FP32_BF16MMA_REF: the reference form with the bf16 contractions.
 * The FP32 precisions run only the fused form (all velocities of an element
 * in one work-group); create returns DGBGK_ENOTSUP when that does not fit. */
typedef enum {
  DGBGK_FP64 = 0,
  DGBGK_FP32 = 1,
  DGBGK_FP32_BF16MMA = 2,
  DGBGK_FP32_REF = 3,
  DGBGK_FP32_BF16MMA_REF = 4
} dgbgk_precision;

/* Problem statement (Sec. II: mesh and polynomial order, velocity set and
 * weights, relaxation time, wall and lid conditions). */
typedef struct {
  int32_t nx, ny;           /* elements in x and y, >= 1                      */
  double x0, y0, lx, ly;    /* domain [x0, x0+lx] x [y0, y0+ly], lx, ly > 0    */
  int32_t p;                /* polynomial order per direction, 1..8            */
  int32_t q;                /* number of discrete velocities, 1..4096          */
  const double *ex, *ey, *w;/* velocities e_q and weights w_q (length q)      */
  double theta;             /* RT of the second-order equilibrium eq. (5), >0 */
  double tau;               /* BGK relaxation time, > 0; +INF: collisionless  */
  int32_t bc[4];            /* dgbgk_bc per side; periodic sides come in pairs */
  double wall_u[4][2];      /* wall velocity per side; must be tangential     */
} dgbgk_problem;

/* ---- pure host helpers (no device use) -------------------------------- */

/* 2-D tensor Gauss-Hermite set (Sec. II.A, Table I; D2Q16 = n1d 4): nodes of
 * the n1d-point rule for the standard normal weight (RT = 1) and weights
 * summing to one.  Writes n1d*n1d entries to ex, ey, w and theta = 1.
 * n1d in 1..40. */
int dgbgk_velset_gh(int32_t n1d, double *ex, double *ey, double *w, double *theta);

/* 2-D tensor Newton-Cotes set (Sec. III.B): m1d equally spaced nodes on
 * [-vmax, vmax] (units of sqrt(RT)), composite trapezoid coefficients times
 * the Maxwellian at the node, normalised to sum one.  Writes m1d*m1d entries
 * and theta = sum_q w_q e_qx^2 (the discrete RT that keeps eq. (5)
 * conservative).  m1d in 2..64, vmax > 0. */
int dgbgk_velset_nc(int32_t m1d, double vmax, double *ex, double *ey, double *w,
                    double *theta);

/* Relaxation time from the Knudsen number, eq. (7) with c_s = 1:
 * convention 0: tau = Kn L / sqrt(3); convention 1: with Kn scaled by
 * sqrt(pi/6) (the variant named after eq. (7)), tau = Kn L / sqrt(pi/2). */
int dgbgk_tau_from_kn(double kn, double L, int32_t convention, double *tau);

/* Bytes of device memory a solver for this problem needs (state registers,
 * tables and scratch); the size a caller passes to dgbgk_bind_buffers(). */
int dgbgk_required_bytes(const dgbgk_problem *pb, int32_t precision, size_t *bytes);

/* ---- solver lifetime --------------------------------------------------- */

/* Validates and copies the problem, builds the reference element and mesh on
 * the host.  Touches no device: device memory is allocated (or taken from
 * dgbgk_bind_buffers) at the first call that needs it.  hip_stream is a
 * hipStream_t (NULL = null stream).  *out is set to NULL on failure. */
int dgbgk_create(const dgbgk_problem *pb, int32_t precision, void *hip_stream,
                 dgbgk_solver **out);

/* Hand the solver a device region of at least dgbgk_required_bytes() bytes,
 * 256-byte aligned, on the current device (e.g. a torch tensor's storage).
 * Must precede the first device call. */
int dgbgk_bind_buffers(dgbgk_solver *s, void *device_ptr, size_t bytes);

/* Replace the stream used by later calls.  Work the solver enqueues on the new
 * stream is ordered after all work it enqueued before on the old stream (an
 * event recorded on the old stream is waited on by the new one), so a switch
 * right after dgbgk_step() needs no host synchronisation; the call itself does
 * not block the host.  The caller keeps the new stream alive while the solver
 * uses it. */
int dgbgk_set_stream(dgbgk_solver *s, void *hip_stream);

void dgbgk_destroy(dgbgk_solver *s);

/* Message of the last failed call on s (never NULL; "" if none). */
const char *dgbgk_last_error(const dgbgk_solver *s);

/* Version string of the library. */
const char *dgbgk_version(void);

/* ---- queries (host only) ----------------------------------------------- */

/* K = nx*ny elements, Np = (p+1)^2, Nfp = p+1, Q velocities. */
int dgbgk_sizes(const dgbgk_solver *s, int64_t *K, int32_t *Np, int32_t *Nfp, int32_t *Q);

/* Explicit step for a CFL number:
 * dt = cfl * (min(hx,hy)/2) * (smallest GLL spacing on [-1,1]) / max_q(|e_qx|+|e_qy|). */
int dgbgk_stable_dt(const dgbgk_solver *s, double cfl, double *dt);

/* Physical node coordinates, x and y of length K*Np (index k*Np + n). */
int dgbgk_node_coords(const dgbgk_solver *s, double *x, double *y);

/* Host copies of the reference-element tables (debug / tests):
 *  0: Dr (Np x Np, row-major)   1: Ds (Np x Np)   2: M (Np x Np)
 *  3: LIFT (Np x 4Nfp)          4: GLL nodes r (Nfp)   5: M1 (Nfp x Nfp)
 *  6: Fscale per face (4)       7: D1 (Nfp x Nfp). */
int dgbgk_get_operator(const dgbgk_solver *s, int32_t which, double *out);

/* ---- state and marching (device) --------------------------------------- */

/* f_q = f_q^eq(rho0, (ux0, uy0)) at every node (eq. (5)). */
int dgbgk_init_equilibrium(dgbgk_solver *s, double rho0, double ux0, double uy0);

/* State f_q = f^eq_q(rho, u) of eq. (5) with each node's own density and
 * velocity (Sec. II.A): rho, ux, uy are host arrays of K Np doubles in node
 * order k Np + n (element k = ex + nx ey; node n = i + (p+1) j), copied before
 * the call returns.  DGBGK_EINVAL unless count == K Np, every rho > 0 and
 * every value finite.  Resets the step count; synchronises. */
int dgbgk_init_moments(dgbgk_solver *s, const double *rho, const double *ux, const double *uy,
                       size_t count);

/* Copy a full FP64 state f[q][k][n] (count = Q*K*Np doubles) in / out. */
int dgbgk_set_state(dgbgk_solver *s, const double *f, size_t count);
int dgbgk_get_state(dgbgk_solver *s, double *f, size_t count);

/* Device address of the current state, element-major f[k][q][n] (FP64,
 * Q*K*Np doubles; for the FP32 precisions the FP32 deviation g[k][q][n] =
 * f - w_q; for the reference forms the FP32 correction g = f - f_r), valid
 * until the next dgbgk_step(); for zero-copy views. */
int dgbgk_state_device_ptr(dgbgk_solver *s, void **ptr);

/* Advance nsteps classical RK4 steps of size dt (enqueued; returns at once).
 * Each step runs the four stages of the right-hand side
 *   L(f)_q = -e_q . grad f_q  (volume)  + lifted upwind face flux  (surface)
 *            - (f_q - f_q^eq(rho, u)) / tau  (collision)
 * with rho, u and the diffuse-wall densities taken from the stage state. */
int dgbgk_step(dgbgk_solver *s, int64_t nsteps, double dt);

/* Replay RK4 steps from a captured hipGraph: with steps_per_graph = k > 0,
 * dgbgk_step() captures k steps (for the current dt and work decomposition)
 * once, on a capture stream of the library's own, and then enqueues
 * nsteps / k graph launches on the solver's stream plus the remaining steps
 * as ordinary launches; a change of dt or of the work decomposition
 * re-captures (after waiting for replays in flight).  Results are
 * bit-identical to eager steps.  For problems so small that launch overhead,
 * not HBM bandwidth, bounds a stage.  0 (the default) turns replay off.
 * k in 0..1000; DGBGK_EINVAL otherwise. */
int dgbgk_set_graph(dgbgk_solver *s, int32_t steps_per_graph);

/* Evaluate the right-hand side L(f) for a host state f (count = Q*K*Np) into
 * a host array k; the solver's own state is left unchanged.  Synchronises.
 * The reference forms evaluate it as a correction f - f_r to the solver's
 * current reference (DGBGK_ESTATE before init / set_state). */
int dgbgk_rhs(dgbgk_solver *s, const double *f, double *k, size_t count);

/* Diffuse-wall densities (eq. (8)) of a host state f at every face node,
 * out[K][4][Nfp]; entries of non-wall faces are 0.  Synchronises.
 * DGBGK_ENOTSUP for the reference forms. */
int dgbgk_wall_density(dgbgk_solver *s, const double *f, double *out, size_t count);

/* Steady-state residual of the current state:
 *   R = max over nodes of max(|sum_q L_q|, |sum_q e_qx L_q|, |sum_q e_qy L_q|)
 *       * L_ref / (rho_ref U_ref),
 * rho_ref = 1, L_ref = min(lx, ly), U_ref = largest wall speed (1 if none).
 * Synchronises; returns DGBGK_ENONFINITE (and R = NaN) for a non-finite state. */
int dgbgk_residual(dgbgk_solver *s, double *r);

/* Same as dgbgk_residual but enqueued: writes R (one double) to device memory
 * at device_out and returns at once. */
int dgbgk_residual_async(dgbgk_solver *s, double *device_out);

/* Node moments of the current state (Sec. II.A): rho = sum_q f_q,
 * u = sum_q e_q f_q / rho; host arrays of K*Np.  Synchronises; returns
 * DGBGK_ENONFINITE if any value is not finite. */
int dgbgk_moments(dgbgk_solver *s, double *rho, double *ux, double *uy);

/* Reference forms: f_r += g, g = 0, then L(f_r) and the moments of f_r are
 * re-evaluated (FP64).  Enqueued; the state f is unchanged (up to the FP64
 * rounding of the sum).  DGBGK_ENOTSUP for the other precisions. */
int dgbgk_fold(dgbgk_solver *s);

/* Wait for all work enqueued by s. */
int dgbgk_synchronize(dgbgk_solver *s);

/* Work decomposition of the stage kernel.  mode 0: automatic (all
 * velocities of a block of elements per work-group when the tile fits in LDS,
 * else velocity tiles); 1 and 3: force the all-velocity (fused) form with one
 * work-group per element block; 2: force velocity tiles of
 * velocities_per_tile (0 = automatic: the largest of Q, Q/2, Q/4, ... that
 * fits, rounded up to a multiple of 64 where the tile count stays); 4: the
 * fused form run by persistent wave-specialised work-groups that each walk a
 * run of blocks (p <= 3, at most 256 velocity rows per block; DGBGK_EINVAL
 * otherwise).  The tiled form (up to four tiles), and the fused form with one
 * element per work-group at orders 1 and 3 (FP64 and FP32 storage), take the
 * node moments of a stage's input from the update pass of the stage before;
 * a separate pass reduces them once after the state was set (init,
 * set_state, an implicit step, a fold), and in every stage with more than
 * four tiles.  get_tiling reports *fused = 0 (velocity tiles), 1 (fused, one
 * work-group per block) or 2 (fused, persistent), and the LDS bytes per
 * work-group.  The fused forms give bit-identical results, except one
 * element per work-group at orders 1 and 3 (moments handed over: another
 * summation order); the tiled form agrees to rounding.  This exists for
 * testing and tuning. */
int dgbgk_set_tiling(dgbgk_solver *s, int32_t mode, int32_t velocities_per_tile);
int dgbgk_get_tiling(const dgbgk_solver *s, int32_t *fused, int32_t *elems_per_group,
                     int32_t *velocities_per_tile, size_t *lds_bytes);

/* Number of RK4 steps taken since the last init / set_state. */
int dgbgk_steps_taken(const dgbgk_solver *s, int64_t *steps);

/* Elements per work-group of the fused forms (0 = automatic).  The value must
 * divide into a tile that fits in LDS; DGBGK_EINVAL otherwise (the previous
 * choice is kept).  Changing it changes the summation order of the node
 * moments, so results agree with other choices to rounding, not bit for bit. */
int dgbgk_set_block_elements(dgbgk_solver *s, int32_t elems_per_group);

/* Autotuner: times `launches` right-hand-side launches on the current state
 * (the state is not modified) for every admissible number of elements per
 * work-group of the fused form (and, in FP64, velocity tiles of Q, Q/2, ...,
 * unless the caller forced the fused form with dgbgk_set_tiling mode 1 or 3),
 * keeps the fastest and returns its average launch time in microseconds
 * (optional).  Requires a state (DGBGK_ESTATE otherwise); synchronises the
 * solver's stream. */
int dgbgk_autotune(dgbgk_solver *s, int32_t launches, double *best_us);

/* ---- implicit time steps (the paper's time marching) ---------------------
 *
 * One step of a stiffly accurate singly diagonally implicit Runge-Kutta
 * scheme, the family the paper integrates with (Sec. II.B, "Time marching"):
 *   DGBGK_BACKWARD_EULER  1 stage, first order, L-stable;
 *   DGBGK_SDIRK2          Alexander's 2-stage, second order, L-stable
 *                         (gamma = 1 - 1/sqrt(2));
 *   DGBGK_SDIRK4          5-stage, fourth order, L-stable, gamma = 1/4
 *                         (Hairer and Wanner, Solving ODEs II, Sec. IV.6);
 *                         the paper's fourth-order runs name four stages but
 *                         give no coefficients, and no four-stage stiffly
 *                         accurate scheme reaches fourth order.
 * Stage i solves y_i = b_i + dt gamma L(y_i), b_i = f_n + dt sum_{j<i} a_ij L(y_j),
 * by Newton's method with GMRES(m) on (I - dt gamma J) d = -F, the products
 * J v taken matrix-free as (L(y + e v) - L(y)) / e with the same right-hand
 * side kernels as the explicit path; f_{n+1} = y_s.  Vector reductions are
 * deterministic, so a call is bitwise reproducible.  FP64 precision only
 * (DGBGK_ENOTSUP otherwise).  The library allocates a device workspace of
 * (m + stages + 6) state-sized vectors (FP32 basis: stages + 6 plus m + 1
 * vectors of half size) at the first call (kept until destroy,
 * regrown if a later call needs more).  Norms are root-mean-square over all
 * K Np Q values.  A stage's Newton iteration stops when its nonlinear residual
 * |y - b - dt gamma L(y)| falls to newton_rtol times its value at the initial
 * guess y = (previous stage value, f_n for the first stage), or to
 * newton_atol; each GMRES solve stops at krylov_rtol times the Newton
 * residual or a tenth of the Newton target, whichever is larger, after
 * max_krylov iterations, or on breakdown.  The difference step is 1e-6
 * (1 + |y|_2) for a unit vector.  opt may be NULL:
 * max_newton 20, newton_rtol 1e-10, newton_atol 1e-14, restart 30,
 * max_krylov 300, krylov_rtol 1e-6, krylov_fp32 0. */
typedef enum { DGBGK_BACKWARD_EULER = 0, DGBGK_SDIRK2 = 1, DGBGK_SDIRK4 = 2 } dgbgk_implicit_scheme;

typedef struct {
  int32_t max_newton;   /* Newton iterations per stage (1..1000)          */
  double newton_rtol;   /* >= 0                                           */
  double newton_atol;   /* >= 0                                           */
  int32_t restart;      /* longest GMRES cycle m (1..64); cycles start at
                           min(8, m) iterations and double, up to m, after
                           a cycle that reduces the residual by < 10%      */
  int32_t max_krylov;   /* GMRES iterations per Newton step (>= 1)        */
  double krylov_rtol;   /* in (0, 1)                                      */
  int32_t krylov_fp32;  /* 1: the Krylov basis is stored in FP32 (half its
                           traffic; the residual, the Krylov vector being
                           orthogonalised, the projections and the
                           solution stay FP64).  The basis is then
                           orthonormal to about 1e-7, so krylov_rtol must
                           be >= 1e-5.  0: FP64 basis                      */
} dgbgk_implicit_options;

typedef struct {
  int32_t newton_iterations;  /* summed over the stages                    */
  int32_t krylov_iterations;  /* summed over the stages and Newton steps   */
  int32_t rhs_evaluations;
  double max_final_residual;  /* largest final stage residual (RMS)        */
  int32_t converged;          /* every stage met the Newton tolerance      */
} dgbgk_implicit_report;

/* nsteps implicit steps of size dt (synchronises; report may be NULL).
 * Returns DGBGK_ENONFINITE if a residual becomes non-finite; a stage that
 * does not meet its tolerance within max_newton iterations still completes
 * (report->converged = 0). */
int dgbgk_implicit_step(dgbgk_solver *s, int32_t scheme, int64_t nsteps, double dt,
                        const dgbgk_implicit_options *opt, dgbgk_implicit_report *report);

/* For callers that cannot allocate device memory (serving loops and harnesses
 * that forbid hipMalloc): dgbgk_implicit_step with the same arguments, results
 * and errors, except that it allocates nothing.  Its device workspace is a
 * static array of the library, 64 MiB (67108864 bytes) per device, of which
 * a call needs about (restart + stages + 6) x 8 K Np Q bytes (FP32 basis:
 * (restart + 1) x 4 K Np Q of them in FP32); a call that needs more returns
 * DGBGK_EINVAL without touching the state.  The solver must already hold a
 * state (its device memory exists) and its device must be current
 * (DGBGK_ESTATE / DGBGK_EDEVICE otherwise).  Every call on one device
 * shares that device's array and overwrites it: calls that overlap in time on
 * one device (other host threads, other solvers) race and must be
 * serialised by the caller.  Each device the library runs on holds its array
 * until the process ends. */
int dgbgk_implicit_step_noalloc(dgbgk_solver *s, int32_t scheme, int64_t nsteps, double dt,
                                const dgbgk_implicit_options *opt,
                                dgbgk_implicit_report *report);

/* ---- batches: several problems advanced together ------------------------
 *
 * A batch advances n solvers (any mix of meshes, orders, velocity sets, Kn,
 * walls and precisions) in lock step: each RK4 stage is one persistent kernel
 * launch per class of (precision, order p, access width, contraction,
 * reference form, LDS size) that walks a device work list of (problem, element
 * block) items and reads each problem's arguments (state pointers, mesh and
 * velocity tables, tau, walls, and its own dt) from a device descriptor table.
 * Classes (and the large members below) are independent chains of launches:
 * the batch spreads them over up to four streams of its own, forked from and
 * joined to the batch's stream around every call (and inside a captured
 * graph), so that work enqueued later on the batch's stream sees every
 * member's steps complete.  A member of 2^22 DOF
 * (K Np Q) or more fills the GPU by itself and runs its own single-problem
 * stage kernels, in its own decomposition, in the same step instead (with such
 * members a change of dt re-captures the step graph).  The members keep their own
 * device memory and states; while they are in a batch, use the batch to step
 * them.  Each member's result is bit-identical to stepping it alone with the
 * same work decomposition (batch invariance).  Smaller members use the fused form (all
 * velocities of a block of elements per work-group); a smaller member whose
 * fused tile does not fit in LDS is rejected (DGBGK_ENOTSUP).  The members' launch
 * configuration (dgbgk_set_tiling, dgbgk_set_block_elements, dgbgk_autotune)
 * is read when the batch is built and must not change while they are in it
 * (dgbgk_batch_step returns DGBGK_ESTATE).  The solvers must outlive the
 * batch. */
typedef struct dgbgk_batch dgbgk_batch;

/* Builds work lists and descriptor tables on the device (the members' device
 * memory is set up if it is not yet).  hip_stream: stream for all batch work
 * (NULL = null stream). */
int dgbgk_batch_create(dgbgk_solver *const *solvers, int32_t n, void *hip_stream,
                       dgbgk_batch **out);

/* use_graph = k > 0: k RK4 steps of the batch are captured once in a hipGraph
 * and replayed (plus a one-step graph for the remainder of a call;
 * re-captured when the membership changes, not when dt does: the descriptors
 * are device data).  0: ordinary launches.  k in 0..1000. */
int dgbgk_batch_set_graph(dgbgk_batch *b, int32_t use_graph);

/* nsteps RK4 steps of every member; dt[i] is member i's time step (n values,
 * host array).  Enqueues only.  Every member needs a state (DGBGK_ESTATE). */
int dgbgk_batch_step(dgbgk_batch *b, int64_t nsteps, const double *dt);

/* Steady-state residual of every member (as dgbgk_residual, bit for bit) into
 * r[n] (host): one right-hand-side launch per class, one reduction per member,
 * one copy to the host; synchronises.  Non-finite residuals are returned as NaN and the
 * call returns DGBGK_ENONFINITE after filling all entries. */
int dgbgk_batch_residuals(dgbgk_batch *b, double *r);

/* Number of persistent launches per RK4 step (classes x 4 stages). */
int dgbgk_batch_launches_per_step(const dgbgk_batch *b, int32_t *launches);

const char *dgbgk_batch_last_error(const dgbgk_batch *b);
void dgbgk_batch_destroy(dgbgk_batch *b);

/* ---- serving: steady-state solves under continuous batching --------------
 *
 * A server takes requests (a problem and an arrival time on the server's
 * clock, in seconds from the start of dgbgk_server_run) and runs each from
 * rest (f = f^eq(1, 0)) to the steady-state residual target (dgbgk_residual
 * below residual_target), keeping its state on the device the whole time.
 * Arrived requests are admitted first come, first served while the device
 * memory they need (dgbgk_required_bytes) fits in hbm_budget and fewer than
 * max_active are running; admitted problems are advanced together as one
 * batch (dgbgk_batch_*) in chunks of check_every RK4 steps, with the batch
 * rebuilt whenever a request joins or leaves, so requests that arrive while
 * others run share the device with them.  Residuals are checked, and requests
 * join and leave, only at chunk boundaries of each request's own step count,
 * so every result is bit-identical to the same request served alone.  A
 * finished request's node moments are copied to host memory and its device
 * memory is released.  dt = the problem's stable step at cfl.
 *
 * Mixed precision: with precision DGBGK_FP32 (or DGBGK_FP32_BF16MMA) and
 * polish_below > 0, a request runs in that precision until its residual falls
 * below polish_below or stops falling (less than 10% lower than its best over
 * 20 checks), then its state moves to an FP64 solver that finishes the solve
 * (FP32 storage cannot reach residuals much below 1e-5: its rounding floor).
 * The device memory of such a request is reserved at the FP64 size.  With a
 * reference form (DGBGK_FP32_REF, DGBGK_FP32_BF16MMA_REF) a request runs in
 * that precision to the end, its correction folded into the FP64 reference
 * after every residual check (polish_below is ignored). */
typedef struct dgbgk_server dgbgk_server;

typedef struct {
  size_t hbm_budget;        /* bytes of device memory for admitted problems (> 0)   */
  int32_t max_active;       /* problems on the device at once (>= 1)                */
  int32_t precision;        /* dgbgk_precision of every request                     */
  double residual_target;   /* e.g. 1e-6 (> 0)                                      */
  int32_t check_every;      /* RK4 steps between residual checks (>= 1)             */
  int64_t max_steps;        /* per-request cap: stopped unconverged beyond it (>= 1) */
  double cfl;               /* dt = dgbgk_stable_dt(cfl) (> 0)                      */
  int32_t use_graph;        /* replay each batch step from a hipGraph               */
  double polish_below;      /* FP32 precisions: switch to FP64 below this residual  */
} dgbgk_server_options;

typedef enum {
  DGBGK_REQ_WAITING = 0,    /* not yet arrived or not yet admitted      */
  DGBGK_REQ_RUNNING = 1,
  DGBGK_REQ_CONVERGED = 2,  /* residual below the target                */
  DGBGK_REQ_STOPPED = 3,    /* max_steps reached first                  */
  DGBGK_REQ_FAILED = 4      /* non-finite state or an error (see stats) */
} dgbgk_request_status;

typedef struct {
  int32_t status;           /* dgbgk_request_status                     */
  double arrival_s, admit_s, finish_s;  /* server clock, seconds        */
  int64_t steps;            /* RK4 steps taken                          */
  double residual;          /* last residual                            */
  int64_t dof;              /* Q K Np                                   */
  int64_t K, Np;            /* sizes of the moment arrays (K*Np each)   */
  int64_t steps_fp64;       /* of which in FP64 after a precision switch */
} dgbgk_request_result;

typedef struct {
  int64_t submitted, completed;  /* completed = converged + stopped + failed */
  double wall_s;                 /* duration of dgbgk_server_run                */
  double dof_updates;            /* sum over requests of dof x 4 x steps        */
  double latency_p50_s, latency_p99_s;  /* finish - arrival over completed      */
  int64_t batch_rebuilds, chunks;
  int32_t peak_active;
  size_t peak_bytes;
  int64_t precision_switches;    /* requests moved from FP32 to FP64 */
  double dof_updates_all;        /* as dof_updates, with the steps of requests not
                                    completed (running or stopped by a time limit) */
  int64_t admitted;              /* requests admitted so far                     */
} dgbgk_server_stats;

int dgbgk_server_create(const dgbgk_server_options *opt, void *hip_stream, dgbgk_server **out);
/* Copies the problem; *id is its index (0, 1, ...). */
int dgbgk_server_submit(dgbgk_server *sv, const dgbgk_problem *pb, double arrival_s, int64_t *id);
/* Runs until every submitted request has completed, or time_limit_s of wall
 * time have passed (then DGBGK_ESTATE; running requests stay running and a
 * later call resumes, with the clock continuing). */
int dgbgk_server_run(dgbgk_server *sv, double time_limit_s);
int dgbgk_server_result(const dgbgk_server *sv, int64_t id, dgbgk_request_result *out);
/* Node moments of a completed request (host arrays of K*Np). */
int dgbgk_server_moments(const dgbgk_server *sv, int64_t id, double *rho, double *ux, double *uy);
int dgbgk_server_get_stats(const dgbgk_server *sv, dgbgk_server_stats *out);
const char *dgbgk_server_last_error(const dgbgk_server *sv);
void dgbgk_server_destroy(dgbgk_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* DGBGK_H */
