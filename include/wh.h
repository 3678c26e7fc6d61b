/*
 * wh.h -- C ABI of the MI355X WaveHoltz library.
 *
 * WaveHoltz (Appelo, Banks, Henshaw, Schwendeman, "An optimal O(N) Helmholtz
 * solver for complex geometry using WaveHoltz and overset grids") finds the
 * solution u of the discrete Helmholtz problem
 *
 *     c^2(x) Delta_{h,p} u + omega^2 u = f   on the interior nodes,   u = 0 on the walls
 *
 * (Sec. 2.1, eq. HelmholtzBVP with L = c^2 Delta and homogeneous Dirichlet
 * data) by filtering time-periodic solutions of the forced wave equation
 * w_tt = c^2 Delta_h w - f cos(omega t) (Sec. 2.1, eq. waveEquation).
 * This library implements the explicit, single-Cartesian-grid form:
 *   - the explicit leapfrog scheme with the frequency correction of
 *     Appendix A.1 (Sec. 4.2.1, eq. WaveSchemeexplicit),
 *   - the trapezoid time filter with the adjusted parameter alpha_d
 *     (Sec. 4.2.1, eqs. updateDiscreteExplicit and alphad), fused into the
 *     time steps,
 *   - the fixed-point iteration of Alg. 1 and restarted GMRES on the linear
 *     form (I - S_h) v = b of Sec. 5.3.
 *
 * Conventions
 *   Grid      The unit box [0,1]^dim, dim = 2 or 3, with n[m] >= 2 cells per
 *             axis (spacing 1/n[m]).  Order p = 2 (5/7-point) or p = 4
 *             (the b_0 + b_1 expansion of Sec. 6.1, i.e. the 9/13-point star);
 *             for p = 4 ghost values beyond a wall are the odd reflection
 *             u(-j) = -u(j).
 *   Arrays    Every grid function crossing this ABI is a dense array of
 *             (n_z+1)(n_y+1)(n_x+1) (or (n_y+1)(n_x+1)) doubles, x fastest,
 *             holding all nodes including the walls.  Values given on wall
 *             nodes are ignored; outputs hold exactly 0 there.
 *   Memory    Pointers documented as "device" must be device memory of the
 *             context's device (e.g. a torch tensor's data_ptr()).  "host or
 *             device" pointers are told apart by the on_device flag.  The
 *             caller owns every buffer; the library keeps no caller pointer
 *             after a call returns, except the workspace, which the caller
 *             binds once and must keep alive (and unused by anyone else)
 *             until the context is destroyed or rebound.
 *   Streams   All device work is enqueued on the stream given to wh_create
 *             (NULL = the null stream).  Calls returning host scalars
 *             (wh_solve, wh_dot-style diagnostics) synchronise that stream;
 *             wh_apply, wh_apply_A and wh_run_periods do not.
 *   Errors    Every call returns a wh_status; 0 is success.  Arguments are
 *             validated before any device work is enqueued.  wh_last_error
 *             returns a message for the most recent failure on a context.
 *             No C++ exception crosses this boundary.
 *   Threads   A context is not thread safe; distinct contexts are
 *             independent.  Calls that overlap on one context race.
 */
#ifndef WH_H
#define WH_H

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__) || defined(__clang__)
#define WH_API __attribute__((visibility("default")))
#else
#define WH_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wh_ctx wh_ctx;

typedef enum {
  WH_OK = 0,
  WH_EINVAL = -1,     /* bad argument (shape, pointer, range) */
  WH_ENOMEM = -2,     /* workspace missing or too small */
  WH_EDEVICE = -3,    /* a HIP runtime call failed */
  WH_EUNSTABLE = -4,  /* requested time step violates the explicit stability limit */
  WH_ENOTCONV = -5,   /* solver stopped at maxit without reaching rtol */
  WH_ENONFINITE = -6, /* a residual norm became NaN or Inf */
  WH_ESTATE = -7      /* call made before the setters it depends on */
} wh_status;

/* Precision of the wave state and stencil arithmetic.  The filter
 * accumulator, the weights and everything in the outer solvers stay FP64. */
typedef enum { WH_FP64 = 0, WH_FP32_STATE = 1 } wh_precision;

/* Outer solvers of (I - S_h) v = b.  FPI: the fixed-point iteration of Alg. 1.
 * GMRES: restarted GMRES(m) (Sec. 5.3).  CG: conjugate gradients in the inner
 * product <u, v> = sum_i u_i v_i / c^2_i, in which c^2 Delta_h and therefore
 * S_h are self-adjoint; the eigenvalues of A = I - S_h are 1 - beta_d in
 * [0, 3/2] (the discrete filter function lies in [-1/2, 1], Sec. 4.2.1), so A
 * is positive definite away from exact resonance.  CG uses three vectors of
 * the Krylov workspace and needs a workspace sized for restart >= 2. */
typedef enum { WH_SOLVER_FPI = 0, WH_SOLVER_GMRES = 1, WH_SOLVER_CG = 2 } wh_solver;

/* Time parameters of one WaveHoltz application (explicit correction recipe,
 * Appendix A.1; stability limit of Sec. 3.2, eq. dtForCartesian):
 *   nt       time steps per corrected period,
 *   periods  Np, periods per application (filter length Tbar = Np * nt * dt),
 *   dt       (2/omega) sin(pi/nt),
 *   omega    the Helmholtz frequency,
 *   omega_e  corrected forcing frequency 2 pi / (nt dt),
 *   alpha    filter parameter used (alpha_d = tan(pi/nt)/tan(2pi/nt) unless overridden),
 *   cfl      c_max dt sqrt(sum_m n_m^2), the CFL number (stable iff <= C_{2,p},
 *            C_{2,2} = 1, C_{2,4} = sqrt(3)/2),
 *   c2max    maximum of c^2 over interior nodes. */
typedef struct {
  int32_t nt;
  int32_t periods;
  double dt;
  double omega;
  double omega_e;
  double alpha;
  double cfl;
  double c2max;
} wh_time_params;

/* Iteration callback: k = 1-based iteration (applies for FPI, Arnoldi steps
 * for GMRES), rel_res = residual estimate relative to ||b||_2. */
typedef void (*wh_iter_callback)(int32_t k, double rel_res, void *user);

typedef struct {
  int32_t method;   /* wh_solver */
  int32_t restart;  /* GMRES restart length m (1..WH_MAX_RESTART); ignored by FPI */
  int32_t maxit;    /* maximum applies (FPI), Arnoldi steps (GMRES) or iterations (CG) */
  int32_t flags;    /* reserved, must be 0 */
  double rtol;      /* stop when ||b - A v||_2 <= rtol ||b||_2; 0 = run maxit (FPI) */
  wh_iter_callback on_iter; /* nullable */
  void *user;
} wh_solve_opts;

/* Results of wh_solve.  For FPI the residual of iterate k is v^k - v^{k-1}
 * (= b - A v^{k-1}); for GMRES and CG it is the true residual b - A v at exit.
 *   iters       FPI applies, GMRES Arnoldi steps or CG iterations performed
 *   applies     WaveHoltz applications performed (includes b and restarts)
 *   rel_res     ||r||_2 / ||b||_2 at exit
 *   scaled_res  ||r||_2 / sqrt(number of nodes) (the paper's scaled norm, Sec. 7)
 *   cr_last     last residual ratio ||r^k|| / ||r^{k-1}|| (FPI) or the
 *               average per-step reduction (GMRES)
 *   cr_avg      (||r^k|| / ||r^1||)^{1/(k-1)}, average convergence rate
 *   ecr         cr_avg^{1/periods}, the effective rate of Sec. 7
 *   mu_pred     predicted FPI rate max |beta_d(lambda~)| (Theorem 2) for
 *               constant c^2; NaN when c^2 varies
 *   seconds     wall time of the call
 *   bnorm       ||b||_2 with b = W_h(0, f)
 *   point_steps interior-node time steps executed
 *   rel_res_recursive  CG: the residual norm its recursion carried at exit
 *               (/ ||b||), beside the true rel_res recomputed from b - A v
 *               (their gap shows rounding drift); NaN for FPI and GMRES
 *   ritz_min, ritz_max  CG: the extreme eigenvalues of the Lanczos
 *               tridiagonal built from CG's step lengths and residual ratios
 *               over its longest stretch between restarts: estimates of the extreme
 *               eigenvalues of A = I - S_h (1/c^2-weighted inner product);
 *               ritz_max / ritz_min estimates kappa(A).  NaN for FPI/GMRES */
typedef struct {
  int32_t iters;
  int32_t applies;
  double rel_res;
  double scaled_res;
  double cr_last;
  double cr_avg;
  double ecr;
  double mu_pred;
  double seconds;
  double bnorm;
  double point_steps;
  double rel_res_recursive;
  double ritz_min;
  double ritz_max;
} wh_solve_info;

#define WH_MAX_RESTART 4096

/* Version of the ABI (major * 10000 + minor * 100 + patch). */
WH_API int32_t wh_version(void);

/* Human-readable name of a status code (static string). */
WH_API const char *wh_status_string(int32_t status);

/* Pure host computation of the time parameters (no device needed): the
 * explicit correction recipe of Appendix A.1 with the stability limit of
 * Sec. 3.2.  nt_override > 0 fixes nt (rejected with WH_EUNSTABLE if the
 * resulting dt breaks the limit), otherwise nt = max(5, ceil(T / dt_max)),
 * raised until dt meets the limit; alpha < 0 selects alpha_d. */
WH_API wh_status wh_compute_time_params(int32_t dim, const int64_t n[3], int32_t order, double c2max,
                                 double omega, int32_t periods, double cfl_frac,
                                 int32_t nt_override, double alpha, wh_time_params *out);

/* Create a context on HIP device `device`; `stream` is a hipStream_t (NULL
 * for the null stream), e.g. torch.cuda.current_stream().cuda_stream.
 * *out is set on success and must be released with wh_destroy. */
WH_API wh_status wh_create(wh_ctx **out, int32_t device, void *stream);

/* Release a context (NULL is accepted).  Does not free the bound workspace. */
WH_API void wh_destroy(wh_ctx *ctx);

/* Message of the last failure on ctx ("" if none; static text if ctx is NULL). */
WH_API const char *wh_last_error(const wh_ctx *ctx);

/* Define the grid: dim in {2,3}, n[0..dim-1] cells per axis (each >= 2;
 * n[2] ignored for dim = 2), order in {2,4}, precision a wh_precision.
 * Resets c^2, the source, the frequency and the workspace binding. */
WH_API wh_status wh_set_grid(wh_ctx *ctx, int32_t dim, const int64_t n[3], int32_t order, int32_t precision);

/* Bytes of device workspace needed for the current grid when GMRES with
 * restart length gmres_restart will be used (0 = no GMRES: applies and FPI). */
WH_API wh_status wh_workspace_size(const wh_ctx *ctx, int32_t gmres_restart, size_t *bytes);

/* Bind caller-owned device memory (256-byte aligned) as workspace.  The
 * restart length later passed to wh_solve must not exceed the one the size
 * was computed for. */
WH_API wh_status wh_bind_workspace(wh_ctx *ctx, void *device_ptr, size_t bytes, int32_t gmres_restart);

/* Wave speed squared at every node (host or device, flag on_device); must be
 * finite and > 0 on interior nodes.  Copied into the workspace. */
WH_API wh_status wh_set_c2(wh_ctx *ctx, const double *c2, int32_t on_device);

/* Constant wave speed squared c2 > 0 (no per-node array is stored or read). */
WH_API wh_status wh_set_c2_constant(wh_ctx *ctx, double c2);

/* Helmholtz right-hand side f of the problem above (host or device). */
WH_API wh_status wh_set_source(wh_ctx *ctx, const double *f, int32_t on_device);

/* Frequency omega > 0, periods Np >= 1 per application, cfl_frac in (0, 1]
 * of the stability limit, nt_override (0 = automatic), alpha (< 0 = alpha_d).
 * Requires the grid and c^2. */
WH_API wh_status wh_set_frequency(wh_ctx *ctx, double omega, int32_t periods, double cfl_frac,
                           int32_t nt_override, double alpha);

WH_API wh_status wh_get_time_params(const wh_ctx *ctx, wh_time_params *out);

/* One WaveHoltz application (Alg. 1 loop body): W^0 = w0 (device), zero
 * initial velocity, Np * nt leapfrog steps with forcing -s f cos(omega_e t^n)
 * (s = with_forcing != 0), writing the filtered result
 *   filtered = sum_n w_n W^n,  w_n = (2/(Np nt)) sigma_n (cos(omega_e t^n) - alpha/2),
 * and the last state W^{Np nt} into w_final.  Both outputs are device
 * pointers; either may be NULL.  Outputs may not alias w0. */
WH_API wh_status wh_run_periods(wh_ctx *ctx, const double *w0, int32_t with_forcing, double *w_final,
                         double *filtered);

/* out = W_h(v, s f) (device pointers; out may not alias v). */
WH_API wh_status wh_apply(wh_ctx *ctx, const double *v, double *out, int32_t with_forcing);

/* Av = v - W_h(v, 0), the matrix-free operator A = I - S_h of Sec. 5.3
 * (eq. MevalII).  Device pointers; Av may not alias v. */
WH_API wh_status wh_apply_A(wh_ctx *ctx, const double *v, double *Av);

/* Solve (I - S_h) v = b, b = W_h(0, f), by FPI (Alg. 1), restarted GMRES or CG.
 * v (device) holds the initial guess on entry and the iterate on exit.
 * info (nullable) receives the statistics.  Returns WH_ENOTCONV if rtol > 0
 * was not reached within maxit (v still holds the last iterate),
 * WH_ENONFINITE if a residual became NaN/Inf. */
WH_API wh_status wh_solve(wh_ctx *ctx, const wh_solve_opts *opts, double *v, wh_solve_info *info);

/* Solve (I - S_h) v = b for a given right-hand side b (device; b may not
 * alias v) instead of b = W_h(0, f); the source need not be set.  Same
 * methods, options and results as wh_solve (the FPI iterates v <- S_h v + b). */
WH_API wh_status wh_solve_rhs(wh_ctx *ctx, const wh_solve_opts *opts, const double *b, double *v,
                              wh_solve_info *info);

/* Mixed-precision solve by residual correction.  hi: a WH_FP64 context with
 * c^2, source and frequency set and a workspace sized for restart >= 2; lo: a
 * context of the same grid, order and time parameters, normally
 * WH_FP32_STATE.  Each outer iteration forms the FP64 residual
 * r = b - A_hi v (b = W_h(0, f) in FP64), solves A_lo d = r approximately with
 * `inner` on lo (its own workspace), and sets v += d, until ||r|| <= outer->rtol
 * ||b|| or outer->maxit corrections (outer->method is ignored).  info->iters =
 * corrections, info->applies counts both precisions, info->rel_res is the FP64
 * residual.  Returns WH_ENOTCONV if outer->rtol was not reached. */
WH_API wh_status wh_solve_mixed(wh_ctx *hi, wh_ctx *lo, const wh_solve_opts *outer, const wh_solve_opts *inner,
                                double *v, wh_solve_info *info);

/* Diagnostic: res = c^2 Delta_{h,p} u + omega^2 u - f on interior nodes,
 * 0 on the walls (device pointers; res may be NULL), and *rel =
 * ||res||_2 / ||f||_2 (host, nullable).  Synchronises the stream. */
WH_API wh_status wh_helmholtz_residual(wh_ctx *ctx, const double *u, double *res, double *rel);

/* Diagnostic: *out = sum_i x_i y_i over all nodes (device inputs), with the
 * library's deterministic reduction order.  Synchronises the stream. */
WH_API wh_status wh_dot(wh_ctx *ctx, const double *x, const double *y, double *out);

/* Time-stepping kernel families.
 *   WH_KERNEL_AUTO       library choice (2-D: blocked, 6 steps per pass for
 *                        p = 4, 8 for p = 2; 3-D: blocked, 4 steps per pass
 *                        for p = 2 FP32, 3 for p = 2 FP64 and p = 4 FP32, 2
 *                        for p = 4 FP64)
 *   WH_KERNEL_NODE       one node per thread, one step per launch (2-D, 3-D)
 *   WH_KERNEL_BLOCKED_2D kblock leapfrog steps per launch (p = 4: 2..6; p = 2:
 *                        2, 3, 4, 6, 8); tile = rows of the region a
 *                        work-group loads (FP64 p = 4: 40, 80, 100; FP64
 *                        p = 2: 32, 64, 80; FP32: 96, 192; 0 = default),
 *                        halo kblock*p/2 included
 *   WH_KERNEL_ZCOL_3D    one step per launch; tile = consecutive z nodes per
 *                        thread (4, 8, 16), z-neighbours kept in registers
 *   WH_KERNEL_BLOCKED_3D kblock (1..4; FP64 p = 4: 1..2) leapfrog steps per
 *                        launch, pipelined along z over (x, y) tiles of 64
 *                        columns; tile = rows of the tile (16 or 32, more
 *                        than 2*kblock*p/2; 0 = default), halo kblock*p/2
 *                        included
 * Every family evaluates the same expression per node and step; results
 * agree with each other to rounding. */
typedef enum {
  WH_KERNEL_AUTO = 0,
  WH_KERNEL_NODE = 1,
  WH_KERNEL_BLOCKED_2D = 2,
  WH_KERNEL_ZCOL_3D = 3,
  WH_KERNEL_BLOCKED_3D = 4
} wh_kernel;

/* Select the kernel family, steps per launch and tile parameter (see
 * wh_kernel).  WH_EINVAL for combinations the grid, order or precision do
 * not support. */
WH_API wh_status wh_set_tuning(wh_ctx *ctx, int32_t kernel, int32_t kblock, int32_t tile);

/* Autotuner: time `applies` applications (A v on a zero vector) with HIP
 * events for every supported (kernel, kblock, tile) choice of the current
 * grid, precision and order, keep the fastest as the context's tuning, and
 * return it (outputs nullable; ms_per_apply = its mean time).  Requires the
 * grid, workspace, c^2 and frequency; overwrites the workspace's scratch
 * vectors (not c^2, f or the Krylov basis).  Synchronises the stream. */
WH_API wh_status wh_autotune(wh_ctx *ctx, int32_t applies, int32_t *kernel, int32_t *kblock, int32_t *tile,
                             double *ms_per_apply);

/* Current tuning after automatic choices are resolved: kernel family,
 * steps per launch, tile parameter, and the owned tile of one work-group
 * (owned_x, owned_y nodes; nullable outputs). */
WH_API wh_status wh_get_tuning(const wh_ctx *ctx, int32_t *kernel, int32_t *kblock, int32_t *tile,
                               int32_t *owned_x, int32_t *owned_y);

/* Timing of the time-stepping kernels, measured with HIP events recorded on
 * the context's stream around the leapfrog launches of every application
 * (the first-step launch excluded).  Used for roofline reporting.
 *   applies      applications timed
 *   launches     leapfrog kernel launches timed
 *   ms           their total device time in milliseconds
 *   bytes        algorithmic HBM bytes those launches must move: every array
 *                a launch reads or writes counted once per interior node
 *                (state levels, c^2 if it varies, f if forced, the FP64
 *                accumulator; the output and v on the last launch)
 *   point_steps  interior-node time steps those launches performed */
typedef struct {
  int64_t applies;
  int64_t launches;
  double ms;
  double bytes;
  double point_steps;
} wh_profile;

/* enable != 0 resets the counters and starts recording; 0 stops.  Recording
 * adds two event records per application and synchronises the stream every
 * 256 applications. */
WH_API wh_status wh_profile_enable(wh_ctx *ctx, int32_t enable);

/* Synchronise the stream and return the counters accumulated so far. */
WH_API wh_status wh_profile_read(wh_ctx *ctx, wh_profile *out);

/* A v = v - W_h(v, 0), as wh_apply_A, for callers that cannot allocate
 * device memory or use a workspace for it (code under HIP stream capture,
 * tight serving loops, harnesses that forbid allocation): the four state
 * levels and the FP64 filter accumulator of the application are taken from a
 * fixed array of 192 MiB in device memory that the library holds on every GPU
 * it runs on until the process ends (its address is looked up on the first
 * call on each device), instead of the workspace.  c^2 and f are still read
 * from the context's workspace, where wh_set_c2 / wh_set_source put them; v
 * and Av are device arrays owned by the caller as for wh_apply_A.  Nothing is
 * allocated and no event is recorded (profiling counters are not updated).
 * The array is shared by every context on that GPU and keeps the last call's
 * contents (every application overwrites all of it before reading it): calls
 * that overlap on one GPU, from any context or stream, race.  Limit: 4 state
 * levels + the accumulator, each rounded to 256 bytes, must fit in 192 MiB
 * (FP64: about 5.0 million nodes, e.g. 2048^2 or 170^3; FP32 state: about 8.3
 * million); larger grids return WH_EINVAL with the sizes in wh_last_error.
 * Also WH_EINVAL for an implicit-stepping context, NULL or host pointers, or
 * Av == v; WH_ESTATE before grid, workspace, c^2 and frequency are set. */
WH_API wh_status wh_apply_A_noalloc(wh_ctx *ctx, const double *v, double *Av);

/* Diagnostic (host only, no device work): the extreme eigenvalues of
 * A = I - S_h over all sine modes of the unit box (Sec. 5.3: S_h has the
 * eigenvalues beta_d(lambda~) of the discrete filter, Sec. 4.2.1 and App.
 * A.3) for a constant wave speed c2 (> 0) under the context's grid, order
 * and time parameters (wh_set_frequency must have been called; the context's
 * own c^2 is not used, so a variable-c^2 context can be probed with its
 * background value).  *a_min = min (1 - beta_d), *a_max = max (1 - beta_d):
 * a_max / a_min is the condition number of A for that c2; k_min (nullable,
 * 3 int32, 0 for the unused axis) receives the wave numbers of the mode
 * closest to resonance.  Spreads the (n_x-1)(n_y-1)(n_z-1) mode evaluations
 * over the host's hardware threads (up to 2^31 modes).  WH_EINVAL for NULL
 * outputs or a bad c2, WH_EUNSTABLE if c2 puts a mode beyond the stability
 * limit of the context's dt, WH_ESTATE before grid and frequency are set. */
WH_API wh_status wh_filter_spectrum(wh_ctx *ctx, double c2, double *a_min, double *a_max, int32_t *k_min);

/* Streaming-bandwidth reference for reading rooflines (not part of the
 * method): `reps` back-to-back launches of the library's own 16-byte-per-lane
 * grid-stride kernel over `bytes` (a positive multiple of 16, 16-byte-aligned
 * device buffers), after one untimed launch, timed with events on `stream`
 * (a hipStream_t; NULL = null stream), which is synchronised.
 *   kind 0  copy src -> dst (buffers must not overlap; 2 x bytes moved)
 *   kind 1  read src (dst unused, may be NULL; bytes moved)
 *   kind 2  write dst (src unused, may be NULL; bytes moved)
 *   kind 3  the per-node traffic of an FP32-state blocked pass without its
 *           stencil, over nodes = bytes / 36 (bytes a multiple of 144): src
 *           holds three FP32 arrays of `nodes` values (read: W^{n-1}, W^n,
 *           c^2), dst two FP32 arrays (written) followed by one FP64 array
 *           (read and written); src needs bytes / 3 and dst bytes * 4 / 9
 *           bytes, not overlapping (bytes moved)
 * groups = work-groups of 256 lanes (0 = 1024, the fastest copy measured on
 * MI355X).  *ms_per_launch receives the average launch time.  Errors:
 * WH_EINVAL for a bad kind, size, alignment, group count, repetition count
 * (1..10000), overlap or a pointer that is not device memory; WH_EDEVICE if a
 * launch or event call fails. */
WH_API wh_status wh_stream_bandwidth(int32_t kind, const void *src, void *dst, size_t bytes, int32_t groups,
                                     int32_t reps, void *stream, double *ms_per_launch);

/* ------------------------------------------------------------------------
 * Deflation (Alg. 3, Sec. 5.2) with the eigenmodes of the unit box.
 *
 * With constant c^2 the eigenfunctions of L_h are the sine modes
 * phi_k(x) = prod_a sqrt(2/n_a) sin(k_a pi x_a) (k_a = 1..n_a-1, orthonormal in
 * the nodal sum) with the discrete eigenvalues lambda_k^2 of the order-p
 * operator (App. B).  When deflation is set, wh_solve (FPI, GMRES and CG)
 * removes the components along the deflated modes from the right-hand side,
 * the initial guess and every operator output, iterates on the remaining
 * modes (whose rate is max |beta_d| over the modes kept: the theorem on
 * deflated convergence), and finally adds back (f, phi) / (omega^2 -
 * lambda^2) phi for each deflated mode, so that the result is the discrete
 * Helmholtz solution.  info->mu_pred is the deflated rate.  Deflation is
 * cleared by any change of c^2 or the grid; wh_solve_rhs and the solvers
 * built on it reject a context with deflation set.
 * ---------------------------------------------------------------------- */
#define WH_MAX_DEFLATION 1024

/* The `count` modes with the largest |beta_d| (the slowest to converge) for
 * the current grid, c^2 (constant) and frequency: modes (host, count x dim
 * wave numbers k_x, k_y[, k_z]) and, nullable, the predicted rate over the
 * remaining modes.  Grids with more than 2^24 modes are rejected. */
WH_API wh_status wh_select_deflation(wh_ctx *ctx, int32_t count, int32_t *modes, double *mu_after);

/* Bytes of caller-owned device workspace for `count` deflated modes (sine
 * tables, eigenvalues, reduction partials). */
WH_API wh_status wh_deflation_workspace_size(wh_ctx *ctx, int32_t count, size_t *bytes);

/* Deflate the given modes (host array, count x dim; distinct, 1 <= k_a <=
 * n_a - 1) in subsequent wh_solve calls, using `workspace` (256-byte aligned
 * device memory of wh_deflation_workspace_size bytes, owned by the caller,
 * kept until deflation is cleared).  count = 0 clears deflation.  Needs a
 * constant c^2 (WH_EINVAL otherwise). */
WH_API wh_status wh_set_deflation(wh_ctx *ctx, const int32_t *modes, int32_t count, void *workspace, size_t bytes);

/* ------------------------------------------------------------------------
 * Implicit time stepping (Sec. 4.2.2, eq. WaveSchemeImplicit), 2-D grids,
 * FP64-state contexts.
 *
 * Each step solves the trapezoidal-in-time scheme
 *   M W^{n+1} = 2 W^n - M W^{n-1} - dt^2 cos(omega_i t^n) cos(omega_i dt) f,
 *   M = I - (dt^2/2) c^2 Delta_{h,p},
 * and the first step M W^1 = W^0 - (dt^2/2) cos(omega_i dt) f (the zero
 * initial velocity eliminates W^{-1}).  The time step follows the implicit
 * correction recipe (Appendix A.2): N_t = nits >= 5 steps per period,
 * dt = sqrt(2 / cos(2 pi / N_t) - 2) / omega, omega_i = 2 pi / (N_t dt)
 * (returned as omega_e by wh_get_time_params); the filter is the explicit
 * scheme's with omega_i.  The library solves each step in the symmetric form
 * (1/c^2) M X = (1/c^2) R by conjugate gradients preconditioned with one
 * geometric multigrid V-cycle (damped Jacobi, full weighting, bilinear
 * interpolation, 2nd-order coarse operators; levels halve the grid while
 * both axes have an even number of cells), to a relative residual of
 * inner_rtol.  Every solver (FPI, GMRES, CG, deflation) then uses these
 * applications; the batched solve, the adjoint and the autotuner do not.
 * ---------------------------------------------------------------------- */

/* Switch the context to implicit stepping with nits (>= 5) steps per period
 * and inner tolerance inner_rtol (0 < inner_rtol <= 1e-2), or back to
 * explicit stepping with nits = 0.  Clears the frequency and deflation
 * (call wh_set_frequency again).  WH_EINVAL for 3-D grids or FP32 state. */
WH_API wh_status wh_set_implicit(wh_ctx *ctx, int32_t nits, double inner_rtol);

/* Bytes of the caller-owned implicit workspace for the current grid (the
 * multigrid hierarchy and the inner CG vectors: about 7.4 FP64 node arrays). */
WH_API wh_status wh_implicit_workspace_size(const wh_ctx *ctx, size_t *bytes);

/* Bind (or, with NULL, unbind) the implicit workspace (256-byte aligned
 * device memory of at least wh_implicit_workspace_size bytes). */
WH_API wh_status wh_bind_implicit_workspace(wh_ctx *ctx, void *ptr, size_t bytes);

/* Counters of the implicit steps taken since the grid was set: steps, inner
 * CG iterations in total and at most per step, and multigrid levels
 * (nullable outputs). */
WH_API wh_status wh_implicit_stats(const wh_ctx *ctx, int64_t *steps, int64_t *inner_iters, int32_t *max_inner,
                                   int32_t *levels);

/* ------------------------------------------------------------------------
 * Discrete adjoint (FP64-state contexts).
 *
 * One application Y = W_h(v, f) (the explicit scheme of Sec. 4.2.1 and the
 * trapezoid filter) is differentiated exactly, at fixed time parameters
 * (dt, N_t, omega_e, alpha: fix N_t with wh_set_frequency's nt_override when
 * c^2 changes).  With Z^n the adjoint of level W^n, the transpose of the
 * leapfrog runs backwards in time; because Delta_h is symmetric,
 * c^2 Z^n obeys the forward leapfrog recursion forced by w_n c^2 lam.  The
 * forward levels needed on the way back are recomputed from checkpoints
 * taken every s = ceil(sqrt(N)) levels (N = N_t * periods), so memory is
 * O(sqrt(N)) fields and the cost is about two extra forward sweeps.
 *
 * The fixed point of Alg. 1, v* = W_h(v*, f), gives for a misfit J(v*):
 *   (I - S)^T lam = dJ/dv,   dJ/dc^2 = d/dc^2 [lam . W_h(v*, f)],
 *   dJ/df = d/df [lam . W_h(v*, f)].
 * ---------------------------------------------------------------------- */

/* Bytes of device workspace the adjoint needs for the current grid and
 * frequency (checkpoints, recomputed segment, adjoint levels). */
WH_API wh_status wh_adjoint_workspace_size(wh_ctx *ctx, size_t *bytes);

/* Bind (or, with NULL, unbind) the caller-owned adjoint workspace
 * (256-byte aligned device memory of at least wh_adjoint_workspace_size). */
WH_API wh_status wh_bind_adjoint_workspace(wh_ctx *ctx, void *ptr, size_t bytes);

/* Sensitivities of lam . W_h(v, f) (f = the context's source) with respect
 * to c^2 (grad_c2), f (grad_f) and v (grad_v = S^T lam); node arrays on the
 * device, each output nullable, written (not accumulated), 0 on walls;
 * outputs distinct and not aliasing v or lam.  Wall values of v and lam are
 * ignored.  Uses the solver workspace's stepping buffers and the adjoint
 * workspace (WH_ENOMEM if missing or too small).  Enqueued on the stream. */
WH_API wh_status wh_gradient(wh_ctx *ctx, const double *v, const double *lam, double *grad_c2, double *grad_f,
                             double *grad_v);

/* Solve (I - S_h)^T lam = g by the method of opts: (I - S)^T equals
 * C^{-1} (I - S) C with C = diag(c^2), so (I - S) mu = C g is solved with
 * wh_solve_rhs's machinery from the guess C lam and lam = mu / c^2 is
 * returned.  lam (device) holds the guess on entry; info and statuses as for
 * wh_solve (residuals refer to the mu system).  Synchronises. */
WH_API wh_status wh_solve_adjoint(wh_ctx *ctx, const wh_solve_opts *opts, const double *g, double *lam,
                                  wh_solve_info *info);

/* Receiver misfit J = 1/2 sum_r (u[idx_r] - data_r)^2 over nrec receivers
 * (idx: flat node indices, int64, device; data: device) and, if grad is not
 * NULL, grad = dJ/du (device node array, overwritten; repeated indices add
 * up).  WH_EINVAL if any index lies outside the grid.  Synchronises. */
WH_API wh_status wh_receiver_misfit(wh_ctx *ctx, const double *u, const int64_t *idx, const double *data,
                                    int32_t nrec, double *J, double *grad);

/* ------------------------------------------------------------------------
 * Batches: many independent 2-D problems advanced together.  Each problem is
 * a fully configured context (grid, workspace sized for restart >= 2, c^2,
 * source, frequency; same order and precision across the batch; different
 * grid sizes and frequencies allowed).  Every blocked pass of all problems
 * still stepping is one kernel launch, the first steps of all problems are one
 * launch, and the batched CG iteration is captured once in a HIP graph and
 * replayed.  The batch uses the problems' workspaces and its own stream; the
 * contexts must outlive it and must not be used concurrently with it.
 * ---------------------------------------------------------------------- */
typedef struct wh_batch wh_batch;

#define WH_MAX_BATCH 1024

WH_API wh_status wh_batch_create(wh_batch **out, int32_t device, void *stream);
WH_API void wh_batch_destroy(wh_batch *batch);
WH_API const char *wh_batch_last_error(const wh_batch *batch);

/* Append a problem; *index (nullable) receives its position.  Problems with
 * deflation set are rejected (WH_EINVAL): the batched solve does not deflate. */
WH_API wh_status wh_batch_add(wh_batch *batch, wh_ctx *ctx, int32_t *index);

/* Steps per launch and tile rows of the batched blocked kernel (0 = default;
 * same values as WH_KERNEL_BLOCKED_2D up to FP64 80 (p = 4) or 64 (p = 2) and
 * FP32 192 rows).  Before wh_batch_finalize. */
WH_API wh_status wh_batch_set_tuning(wh_batch *batch, int32_t kblock, int32_t tile);

/* Bytes of device workspace for the batch's tables (after adding problems). */
WH_API wh_status wh_batch_workspace_size(wh_batch *batch, size_t *bytes);

/* Bind the table workspace (256-byte aligned, caller-owned) and freeze the
 * batch (no more wh_batch_add). */
WH_API wh_status wh_batch_finalize(wh_batch *batch, void *workspace, size_t bytes);

/* Batch autotuner: time `applies` batched applications (A v, v = 0) for
 * every supported (kblock, tile) choice, keep the fastest and return it
 * (outputs nullable; ms_per_apply = its mean time).  After
 * wh_batch_finalize; overwrites the problems' scratch vectors (not c^2, f or
 * solutions held by the caller).  Synchronises. */
WH_API wh_status wh_batch_autotune(wh_batch *batch, int32_t applies, int32_t *kblock, int32_t *tile,
                                   double *ms_per_apply);

/* Steps per launch and tile rows in use (defaults resolved). */
WH_API wh_status wh_batch_get_tuning(const wh_batch *batch, int32_t *kblock, int32_t *tile);

/* out[i] = W_h(v[i], s f_i) for every problem i (host arrays of device
 * pointers, in wh_batch_add order; out[i] may not alias v[i]).  Enqueued on
 * the batch's stream. */
WH_API wh_status wh_batch_apply(wh_batch *batch, const double *const *v, double *const *out, int32_t with_forcing);

/* Solve every problem's (I - S_h) x_i = b_i, b_i = W_h(0, f_i), by CG in the
 * 1/c^2 inner product (opts->method must be WH_SOLVER_CG; rtol > 0) until
 * each reaches rtol or maxit iterations.  x[i] (device) holds the guess on
 * entry and the iterate on exit; info (nullable) is an array with one entry
 * per problem (rel_res is the true residual at exit).  Synchronises. */
WH_API wh_status wh_batch_solve(wh_batch *batch, const wh_solve_opts *opts, double *const *x, wh_solve_info *info);

/* As wh_batch_solve with given right-hand sides: (I - S_h) x_i = b[i] (device
 * FP64 node arrays, one per problem, not aliasing x[i]; copied at the start).
 * A problem whose b[i] is zero is left as it is (rel_res 0). */
WH_API wh_status wh_batch_solve_rhs(wh_batch *batch, const wh_solve_opts *opts, const double *const *b,
                                   double *const *x, wh_solve_info *info);

/* Residual correction over two finalized batches of the same problems in the
 * same order: `hi` of WH_FP64 contexts, `lo` of WH_FP32_STATE contexts (same
 * grids, orders and time parameters).  Each outer iteration forms every
 * problem's FP64 residual r_i = b_i - A x_i on hi (b_i = W_h(0, f_i) in FP64,
 * once), solves A d_i = r_i approximately by the batched CG on lo (`inner`:
 * CG, its rtol and maxit; problems already at outer->rtol get d_i = 0) and
 * sets x_i += d_i, until every problem has ||r_i|| <= outer->rtol ||b_i|| or
 * outer->maxit corrections were made.  The filter accumulation, the Krylov
 * vectors and the residuals stay FP64; lo's state and stencil are FP32.
 * info[i]: iters = corrections of problem i, applies counts both precisions,
 * rel_res = its FP64 residual.  Returns WH_ENOTCONV if a problem did not
 * reach outer->rtol; WH_EINVAL for mismatched batches or precisions. */
WH_API wh_status wh_batch_solve_mixed(wh_batch *hi, wh_batch *lo, const wh_solve_opts *outer,
                                     const wh_solve_opts *inner, double *const *x, wh_solve_info *info);

#ifdef __cplusplus
}
#endif

#endif /* WH_H */
