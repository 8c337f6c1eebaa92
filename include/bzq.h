/*
 * bzq.h -- the homogeneous Boltzmann collision operator with a non-cutoff
 * angular kernel, evaluated by the fast Fourier spectral method of
 * J. Hu and K. Qi, "A fast Fourier spectral method for the homogeneous
 * Boltzmann equation with non-cutoff collision kernels" (arXiv:2004.11239),
 * on one AMD Instinct MI355X (gfx950).
 *
 * Problem (Section 2, eq. eqnR and the Galerkin system that follows it):
 *   d f_k / dt = Q_k,   k in K_N = {-N/2+1 .. N/2-1}^3,
 *   f_N(v) = sum_k f_k e^{i pi k.v / L} on the periodic box D_L = [-L, L]^3,
 *   Q_k = sum_{l+m=k} G(l,m) f_l f_m                        (eq. sum)
 * with the weight G split into a radial Gauss-Legendre rule on [0, R] and a
 * spherical rule (eq. approxG), which gives the fast form (eq. realQ)
 *   Q_k = sum_{rho,sigma} w_rho w_sigma rho^{2+gamma} F(k, rho, sigma)
 *                         sum_{l+m=k} f_l e^{-i pi rho m.sigma / L} f_m.
 * Collision kernel B = |q|^gamma b(cos th) (eq. Bb) with the angular part
 *   b = c t^{-1-s} (1-t)^{-r},  t = sin^2(th/2),
 * whose singularity at th = 0 is non-integrable for s >= 0 (eq. Bb1 with
 * nu = 2s); F (eq. FF) is the exact angular integral.
 *
 * Data layout of every spectral array exchanged at this boundary:
 *   device pointer to N*N*N complex128 values, interleaved (re, im) doubles,
 *   C order [i1][i2][i3], FFT index order along each axis (index i <-> k = i
 *   for i < N/2, k = i - N otherwise).  Entries with any index equal to N/2
 *   (the Nyquist planes) are not read and are written as 0.
 *   Normalisation: f_k = (2L)^-3 \int_{D_L} f e^{-i pi k.v/L} dv.
 *
 * Ownership and concurrency:
 *   the caller owns f_hat / Q_hat; the plan owns its tables and scratch and is
 *   immutable after creation.  Calls on one plan must not overlap in time:
 *   issue them on one stream (scratch is shared between calls).  All calls
 *   are asynchronous on `stream` (a hipStream_t; NULL = default stream)
 *   unless stated otherwise; errors in argument checking are reported before
 *   anything is enqueued.
 *
 * Errors: functions return bzq_status; no exception crosses this boundary.
 *   bzq_last_error() returns a thread-local description of the last failure.
 */
#ifndef BZQ_H
#define BZQ_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct bzq_plan_s* bzq_plan;
typedef struct bzq_workspace_s* bzq_workspace;
typedef struct bzq_batch_s* bzq_batch;
typedef struct bzq_server_s* bzq_server;
typedef struct bzq_plan2d_s* bzq_plan2d;

typedef enum {
    BZQ_OK = 0,
    BZQ_EINVAL = 1,        /* an argument is out of range                          */
    BZQ_ENOMEM = 2,        /* device memory could not be allocated                 */
    BZQ_EDEVICE = 3,       /* a HIP runtime call failed (details: bzq_last_error)  */
    BZQ_EUNSUPPORTED = 4,  /* valid in principle, but no kernel for this size      */
    BZQ_ENONFINITE = 5,    /* NaN or Inf found in the input                        */
    BZQ_EBUSY = 6          /* the request server's queue is full; nothing queued   */
} bzq_status;

typedef enum {
    BZQ_FP64 = 0,          /* FFTs, products, table and accumulation in FP64           */
    BZQ_FP32_ACC64 = 1     /* FFTs, products and table in FP32; the quadrature
                              accumulation over (rho, sigma), the output and every
                              moment in FP64                                           */
} bzq_precision;

/* Angular kernel of a plan (bzq_plan_create, bzq_plan_create_otf); t = sin^2(th/2):
 *   BZQ_KERNEL_POWER        b = c_s sin^{-(2+2s)}(th/2) = c_s t^{-1-s}, c_s = (1-s)(2-s)/(24 pi),
 *                           0 <= s < 1: the non-cutoff kernel of eq. Bb1 (nu = 2s) with the
 *                           constant that gives the BKW rate lambda = 1/6 of Section 5.1
 *                           (s = 3/4 is the paper's b8 of Section 5.3);
 *   BZQ_KERNEL_CUTOFF_CONST b = 1/(4 pi), the cutoff kernel b5 of Section 5.3 (eq. cutoff3D gives
 *                           its weight in closed form);
 *   BZQ_KERNEL_GENERAL      b = c t^{-1-s} (1-t)^{-r} with (c, s, r) given explicitly
 *                           (bzq_plan_create_otf; bzq_plan_create_general takes them always). */
typedef enum {
    BZQ_KERNEL_POWER = 0,
    BZQ_KERNEL_CUTOFF_CONST = 1,
    BZQ_KERNEL_GENERAL = 2
} bzq_kernel;

/*
 * Create a plan for the operator of eq. realQ (Section 4: the Gauss-Legendre
 * rule in |q| and the sphere rule of eq. approxG, the weight F of eq. FF
 * precomputed as in Section 4.1) with the angular kernel `kernel`
 * (BZQ_KERNEL_POWER or BZQ_KERNEL_CUTOFF_CONST; `s` is ignored for the latter).
 *   N      grid size per axis; one of 8, 16, 24, 32, 48, 64, 128 (EUNSUPPORTED
 *          else; at 128 the plane stage runs in three passes through a row
 *          buffer, since a padded plane of 192^2 values does not fit LDS)
 *   L      half-width of the periodic box D_L (> 0)
 *   R      radius of the ball B_R that truncates |q| (> 0)
 *   gamma  exponent of Phi(|q|) = |q|^gamma, -3 < gamma <= 1 (eq. Bb)
 *   s      order of the angular singularity, 0 <= s < 1 (nu = 2s < 2)
 *   N_rho  number of Gauss-Legendre nodes in |q| on [0, R] (>= 1)
 *   M      size of the Lebedev rule on S^2: 6, 14, 26, 38, 50, 74, 86, 110,
 *          146, 170, 194, 230, 266, 302 or 350
 *   precision  a bzq_precision value
 * Synchronous: builds the weight tables on the device and returns when they
 * are ready.  On failure *out is set to NULL and nothing stays allocated.
 */
bzq_status bzq_plan_create(bzq_plan* out, int N, double L, double R, double gamma, double s,
                           int N_rho, int M, int precision, int kernel, void* stream);

/*
 * Same with a general angular kernel b = c t^{-1-s} (1-t)^{-r}
 * (t = sin^2(th/2)); covers the paper's 3-D kernels of Section 5.3:
 *   b5 (cutoff, 1/(4 pi)): c = 1/(4 pi), s = -1, r = 0
 *   b6: c = 1/(16 pi), s = 0, r = 1/2      b7: c = 1/(12 pi^2), s = 1/2, r = 1/2
 *   b8: c = 5/(384 pi), s = 3/4, r = 0
 * Requires -1 <= s < 1, 0 <= r < 1, c > 0.  n_jacobi (8..256) is the number of
 * Gauss-Jacobi nodes used for the t-integral of F (64 in bzq_plan_create).
 */
bzq_status bzq_plan_create_general(bzq_plan* out, int N, double L, double R, double gamma,
                                   double b_c, double b_s, double b_r, int n_jacobi,
                                   int N_rho, int M, int precision, void* stream);

/* A plan for the Debye-Yukawa kernel of Section 5.6 (eq. ApproximatedDebye),
 *   sin(theta) B(|q|, cos theta) = |q| |log(2 sin(theta/2))| / (2 sin(theta/2)),
 * i.e. Phi = |q| (gamma = 1) and a logarithmic angular singularity, set to
 * zero below theta_cut (eq. ApproximatedDebyecutoff: theta_cut = pi/10; 0 for
 * the non-cutoff kernel; 0 <= theta_cut < pi/3, else BZQ_EINVAL).  The weight
 * F of eq. FF is integrated in t = sin^2(theta/2) with a composite rule for
 * |log(2 sqrt t)| (1-t)^{-1/2} (204 nodes; 120 with the cutoff).  Other
 * arguments and limits as for bzq_plan_create. */
bzq_status bzq_plan_create_debye(bzq_plan* out, int N, double L, double R, double theta_cut, int N_rho, int M,
                                 int precision, void* stream);

/* The operator of eq. realQ (Section 4) with its weights evaluated on the fly
 * (beyond the paper): no table of J N^3 / 2 weights is stored or built.  Before the last stage of
 * each block of pairs (at most 256 MiB of weights, or $BZQ_OTF_MB), a kernel
 * evaluates that block's weights from the Funk-Hecke series of the exact
 * weight of eq. FF,
 *   Re(e^{-ix} F) = sum_{l even} (2l+1) (-1)^{l/2} mu_l j_l(a|k|) P_l(k.sigma/|k|),
 *   mu_l = 2 pi \int b(u) (P_l(u) - 1) du  (finite for every s < 1),
 * truncated at l <= r + 8 r^{1/3} + 12, r = a|k| (below 1e-13 of the sum; at
 * most 80 even terms, r <= ~100).  The plan then holds N_rho x (terms rounded
 * up to 8) x (3 (N/2-1)^2 + 1) coefficients (71 MB at N = 64, N_rho = 64)
 * instead of the weight table (4.8 GB FP32, 9.7 GB FP64 at N = 64, M = 302),
 * and its workspace one block of weights.  `kernel` selects the angular kernel
 * (bzq_kernel): BZQ_KERNEL_POWER takes s = b_s (b_c, b_r ignored),
 * BZQ_KERNEL_CUTOFF_CONST ignores all three, BZQ_KERNEL_GENERAL takes
 * b = b_c t^{-1-b_s} (1-t)^{-b_r} with the limits of bzq_plan_create_general
 * (there is no n_jacobi: the series moments use their own exact Gauss-Jacobi
 * rule).  Every other call accepts the plan unchanged.
 * BZQ_EUNSUPPORTED, before any device work, if the series would need more
 * than 80 terms. */
bzq_status bzq_plan_create_otf(bzq_plan* out, int N, double L, double R, double gamma, int kernel,
                               double b_c, double b_s, double b_r, int N_rho, int M, int precision,
                               void* stream);

/* A plan for another gamma that shares the tables of `base` (weights,
 * phases, twiddles: they do not depend on gamma, which enters eq. realQ only
 * through c_p = w_rho rho^{2+gamma} with Phi = |q|^gamma).  The new plan holds
 * its own c_p table, workspace and scratch; the shared tables stay allocated
 * until every plan holding them is destroyed, so `base` may be destroyed
 * first.  Results equal, bitwise, those of a plan created from scratch with
 * the same arguments and gamma.  Synchronous; BZQ_EINVAL for a NULL base or
 * gamma outside (-3, 1]. */
bzq_status bzq_plan_derive_gamma(bzq_plan* out, bzq_plan base, double gamma, void* stream);

/* Device bytes of the tables a plan shares with the plans derived from it
 * (bzq_plan_device_bytes counts them too). */
size_t bzq_plan_shared_bytes(bzq_plan p);

/* Q_hat = Q(f_hat, f_hat): the truncated weighted convolution of eq. sum with
 * G replaced by its quadrature eq. approxG, evaluated in the fast form of
 * eq. realQ (Section 4).  f_hat and Q_hat: device, complex128 N^3 (layout
 * above); the two byte ranges must not overlap (BZQ_EINVAL).  Q_hat[0] is
 * exactly 0 (the remark after eq. realQ: F(0, rho, sigma) = 0).
 * Non-finite input: the first stage of the evaluation (the copy of f_hat into
 * the padded spectrum) also reduces a NaN/Inf flag over every entry it reads
 * (all but the Nyquist planes); the call waits for that flag (a stream
 * synchronisation up to this stage) and returns BZQ_ENONFINITE before any
 * launch that writes Q_hat, which is then left untouched.  Otherwise the rest
 * of the evaluation is enqueued asynchronously. */
bzq_status bzq_collision(bzq_plan p, const double* f_hat, double* Q_hat, void* stream);

/* bzq_collision for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same operator and arguments; it calls no allocating routine of any kind.
 * Its pipeline scratch (compact spectrum, f on the padded grid, the two
 * intermediates of a chunk of pairs and the partial sums) is a static device
 * array of 128 MiB that each GPU running the library holds until the process
 * ends; the chunk of pairs is shrunk to fit it (results then differ from
 * bzq_collision in summation order only).  Plans whose scratch cannot fit even
 * with one pair-two per chunk give BZQ_EUNSUPPORTED; every plan of the sizes
 * above fits.  All calls on one GPU share that array: calls that overlap in
 * time on one GPU (other streams, other threads) race and must not be issued.
 * No NaN/Inf check (nothing synchronises): a non-finite f_hat gives a
 * non-finite Q_hat.  Asynchronous on `stream`. */
bzq_status bzq_collision_noalloc(bzq_plan p, const double* f_hat, double* Q_hat, void* stream);

/* Advance the Galerkin system d f_k/dt = Q_k (Section 2, the ODE system that
 * follows eq. weak) by n_steps steps of Heun's method (explicit trapezoid:
 * f* = f + dt Q(f), f <- f + dt/2 (Q(f) + Q(f*))), in place on the device
 * array f_hat.  dt finite, n_steps >= 0, else BZQ_EINVAL.  The input state is
 * checked as in bzq_collision: BZQ_ENONFINITE, with f_hat untouched, if it
 * holds NaN/Inf (the states inside the n_steps are the library's own). */
bzq_status bzq_step(bzq_plan p, double* f_hat, double dt, int n_steps, void* stream);

/* The same with the classical fourth-order Runge-Kutta method, the time
 * integrator of the paper's experiments (Section 5): four evaluations per step,
 *   k1 = Q(f), k2 = Q(f + dt/2 k1), k3 = Q(f + dt/2 k2), k4 = Q(f + dt k3),
 *   f <- f + dt/6 (k1 + 2 k2 + 2 k3 + k4),
 * in place on the device array f_hat (FP64 state and stage sums).  Arguments,
 * errors and the check of the input state as for bzq_step. */
bzq_status bzq_step_rk4(bzq_plan p, double* f_hat, double dt, int n_steps, void* stream);

/*
 * FP64 diagnostics of f on the N^3 grid v_j = -L + j 2L/N (Section 1):
 *   out[0] mass (2L)^3 Re f_0 (Remark 4.1)
 *   out[1..3] momentum \int f v, out[4] energy \int f |v|^2 (trapezoid rule)
 *   out[5] entropy dissipation \int Q ln f over points with f > 1e-14 max f
 *          (H-theorem: <= 0); Q is Q_hat if given, else Q(f_hat) is evaluated.
 * `out` is host memory (6 doubles).  Synchronous on `stream`.
 */
bzq_status bzq_moments(bzq_plan p, const double* f_hat, const double* Q_hat, double* out,
                       void* stream);

/* Synchronous check of f_hat for NaN/Inf: BZQ_OK or BZQ_ENONFINITE. */
bzq_status bzq_check_finite(bzq_plan p, const double* f_hat, void* stream);

/*
 * Extra scratch for concurrent use of one plan: a plan's tables are
 * read-only, so evaluations on different streams may share it as long as each
 * stream uses its own workspace (the plan's built-in workspace serves
 * bzq_collision / bzq_step).  Results are bitwise identical to the built-in
 * path.  bzq_workspace_destroy synchronises the device.
 */
bzq_status bzq_workspace_create(bzq_workspace* out, bzq_plan p);
/* bzq_collision / bzq_step (eq. realQ; Heun's method) with scratch from w, with
 * the same argument checks and the same BZQ_ENONFINITE behaviour. */
bzq_status bzq_collision_ws(bzq_plan p, bzq_workspace w, const double* f_hat, double* Q_hat,
                            void* stream);
bzq_status bzq_step_ws(bzq_plan p, bzq_workspace w, double* f_hat, double dt, int n_steps,
                       void* stream);
size_t bzq_workspace_bytes(bzq_workspace w);
bzq_status bzq_workspace_destroy(bzq_workspace w);

/*
 * Independent cells, simple form: Q_hats[i] = Q(f_hats[i]) of eq. realQ under
 * plans[i] (each cell is its own spatially homogeneous problem, Section 2),
 * enqueued cell after cell on `stream` with each plan's built-in workspace.
 * Each result is bitwise identical to bzq_collision.  Arrays are host arrays
 * of `count` device pointers; BZQ_EINVAL for NULL entries, count < 1 or an
 * f/Q pair that overlaps.  No input check for NaN/Inf (asynchronous).
 */
bzq_status bzq_collision_batch(const bzq_plan* plans, const double* const* f_hats,
                               double* const* Q_hats, int count, void* stream);

/*
 * Independent cells, fused form (eq. realQ and Heun's method per cell, the
 * cells being independent homogeneous problems, Section 2).  A batch binds `count` cells (state arrays
 * f_hats[i], device, complex128 N_i^3, owned by the caller and kept alive as
 * long as the batch) to plans (which may repeat and may differ in N, gamma,
 * kernel and precision).  Cells sharing a plan run in the same launches, up
 * to 64 cells per launch; cells_per_launch = 0 lets an autotuner choose per
 * plan, timing the
 * candidates 1, 2, 4 ... 64 on these cells once (best of three evaluations
 * of at least 64 cells each; a larger count is kept only when it is at
 * least 1 % faster), with the choice cached in the file $BZQ_TUNE_CACHE or ~/.cache/bzq_autotune.txt;
 * workspaces are capped by $BZQ_BATCH_WS_MB, default 8192.  Creation is
 * synchronous and allocates the workspaces.
 *   bzq_batch_collision: Q_hats[i] = Q(f_hats[i]).
 *   bzq_batch_step: n_steps Heun steps of every cell in place; use_graph != 0
 *     captures one step of the whole batch into a HIP graph on first use (and
 *     again when dt changes) and replays it.
 * Every cell's result is bitwise identical to bzq_collision / bzq_step with
 * its plan.  bzq_batch_group_info: out[4] = {N, cells, cells per launch,
 * 1 if chosen by timing}.
 */
bzq_status bzq_batch_create(bzq_batch* out, const bzq_plan* plans, double* const* f_hats, int count,
                            int cells_per_launch, void* stream);
/* Mixed sizes in one launch (cells of N = 16, 24, 32 in one launch per
 * pipeline stage over a device table of (cell, workgroup) work items) is
 * switched off: its first run on the device ended in a memory fault whose
 * cause is not known.  cells_per_launch = -1, which demands it, returns
 * BZQ_EUNSUPPORTED; 0 and > 0 keep one group of launches per plan.
 * bzq_batch_rounds: the rounds of the mixed launches (always 0 while they are
 * switched off). */
int bzq_batch_rounds(bzq_batch b);
bzq_status bzq_batch_collision(bzq_batch b, double* const* Q_hats, void* stream);
bzq_status bzq_batch_step(bzq_batch b, double dt, int n_steps, int use_graph, void* stream);
int bzq_batch_groups(bzq_batch b);
bzq_status bzq_batch_group_info(bzq_batch b, int group, int* out);
size_t bzq_batch_device_bytes(bzq_batch b);
bzq_status bzq_batch_destroy(bzq_batch b);

/*
 * Request server with continuous batching.  A request is one cell of the
 * power-law operator (BZQ_KERNEL_POWER) with its own parameters and asks for
 * either Q_hat = Q(f_hat) (kind BZQ_REQ_COLLISION, eq. realQ) or n_steps Heun
 * steps of the Galerkin system of Section 2 (kind BZQ_REQ_STEP).
 *   bzq_server_create: budget_bytes of device memory (>= 64 MiB) for cached
 *     plans, workspaces and request state; `slots` (1..16) requests run
 *     concurrently, each on its own stream; at most max_queued requests wait
 *     (0 = no limit); flags: BZQ_SERVER_TUNE times the kernel schedule of
 *     every new plan on its first request's input (bzq_plan_autotune, with
 *     the tuning cache) before that request runs.  A worker thread owns all
 *     device work.
 *   bzq_server_submit: copies f_host (host, complex128 N^3) and queues the
 *     request; returns its id at once.  N is any size bzq_plan_create takes
 *     (BZQ_EINVAL for odd N or N < 8, BZQ_EUNSUPPORTED for a size without an
 *     FFT schedule); requests use table plans.  BZQ_EBUSY (nothing queued,
 *     counted as rejected) when max_queued requests already wait.
 *     Thread-safe.
 *   bzq_server_poll: 1 = done (result, the new state or Q_hat, copied to f_out
 *     if not NULL, request released), 0 = not yet, -1 = unknown id, -2 =
 *     failed (bzq_last_error tells why; released).  times (optional, host
 *     double[3]) = arrival, start and completion on the server's monotonic
 *     clock, seconds.
 *   bzq_server_wait: blocks until request id is done or failed, or timeout.
 *   bzq_server_stats: out[9] = submitted, completed, failed, queued, running,
 *     device bytes in use, peak device bytes, plans evicted, rejected.
 * Requests are admitted in arrival order when their plan (if not cached), a
 * workspace and their state fit the budget; idle plans are evicted least
 * recently used first.  A request that cannot fit while nothing else runs
 * fails with ENOMEM (it never waits for memory that no completion can free).
 * Each result is bitwise identical to bzq_step / bzq_collision run alone on a
 * plan of the same parameters and schedule.
 */
typedef enum { BZQ_REQ_STEP = 0, BZQ_REQ_COLLISION = 1 } bzq_request_kind;
typedef enum { BZQ_SERVER_TUNE = 1 } bzq_server_flags;

typedef struct {
    int N;
    double L, R, gamma, s;
    int N_rho, M, precision;
    double dt;        /* BZQ_REQ_STEP only */
    int n_steps;      /* BZQ_REQ_STEP only */
    int kind;         /* a bzq_request_kind */
} bzq_request;

bzq_status bzq_server_create(bzq_server* out, size_t budget_bytes, int slots, int max_queued, int flags);
bzq_status bzq_server_submit(bzq_server s, const bzq_request* req, const double* f_host,
                             unsigned long long* id);
int bzq_server_poll(bzq_server s, unsigned long long id, double* f_out, double* times);
bzq_status bzq_server_wait(bzq_server s, unsigned long long id, double timeout_s);
bzq_status bzq_server_stats(bzq_server s, double* out);
bzq_status bzq_server_destroy(bzq_server s);

/*
 * The two-dimensional operator (d = 2, the setting of the paper's Section 5.2
 * and Table 1): K_N = {-N/2+1 .. N/2-1}^2, f_k = (2L)^{-2} \int f e^{-i pi k.v/L},
 * weight T = w_rho w_sigma rho^{1+gamma} F(k, rho, sigma) with F the angular
 * integral of eq. FF2D1 for b = c t^{-1-s} (1-t)^{-r} (t = sin^2(th/2);
 * -1 <= s < 1/2, -1 < r < 1/2, covering b1-b4 of Section 5.2), a Gauss-Legendre
 * rule of N_rho nodes on [0, R] and the midpoint rule of N_sigma (even) points
 * on the circle.  f_hat, Q_hat: device complex128 N^2, C order [i1][i2], FFT
 * index order, Nyquist rows/columns not read and written 0.  N in {8, 16, 24,
 * 32, 48, 64}; precision as for 3-D plans.  Creation is synchronous; the plan
 * owns its scratch, so calls on one plan must not overlap in time.
 */
bzq_status bzq_plan2d_create(bzq_plan2d* out, int N, double L, double R, double gamma, double b_c,
                             double b_s, double b_r, int n_jacobi, int N_rho, int N_sigma, int precision,
                             void* stream);
bzq_status bzq_collision2d(bzq_plan2d p, const double* f_hat, double* Q_hat, void* stream);

/* Time integrators of the 2-D Galerkin system, as for 3-D plans. */
typedef enum { BZQ_HEUN = 0, BZQ_RK4 = 1 } bzq_method;

/* Advance d f/dt = Q(f, f) by n_steps steps of Heun's method (BZQ_HEUN) or of
 * the classical fourth-order Runge-Kutta method (BZQ_RK4, the integrator of the
 * paper's 2-D experiments, Section 5.2), in place on the device array f_hat
 * (N^2 complex128, FP64 state and stage sums).  Stage buffers belong to the
 * plan.  dt > 0, n_steps >= 0, otherwise BZQ_EINVAL before any device work. */
bzq_status bzq_step2d(bzq_plan2d p, double* f_hat, double dt, int n_steps, int method, void* stream);
bzq_status bzq_plan2d_destroy(bzq_plan2d p);

/* Device bytes held by the plan (tables + scratch), for admission control. */
size_t bzq_plan_device_bytes(bzq_plan p);

/* The same figure computed before creating a plan of this geometry. */
size_t bzq_plan_bytes_estimate(int N, int N_rho, int M, int precision);

/* Device bytes one more concurrently served cell of size N needs besides its
 * plan's tables: its state f_hat and Q_hat (complex128 N^3 each) plus the
 * scratch of one workspace (bzq_workspace_create) of any plan of this N and
 * precision (an upper bound over N_rho and M: the pipeline's chunk of pairs
 * is capped).  0 for an invalid N or precision. */
size_t bzq_request_device_bytes(int N, int precision);

/*
 * Introspection for tests:
 *   bzq_plan_info: host out[8] = {N, P (padded FFT size), number of antipodal
 *     quadrature pairs (rho_p, sigma_q+), pairs per chunk, K3 splits,
 *     precision, n_jacobi, table bytes}.
 *   bzq_plan_pairs: host out[npairs*6] = {rho_p, sigma_x, sigma_y, sigma_z,
 *     w_sigma, w_rho rho^{2+gamma}} per pair, sigma taken from the half of the
 *     sphere rule whose first non-zero coordinate is positive.
 *   bzq_plan_weights: the stored real weight of pair j at every half-spectrum
 *     mode, as FP64 into host memory out[((N-1)^2+1)/2 * (N-1)]; entry
 *     [c][i3] is mode k = (i1 - N/2 + 1, i2 - N/2 + 1, i3 - N/2 + 1) with
 *     c = i2 (N-1) + i1 (c <= ((N-1)^2-1)/2).  The value is
 *     2 w_sigma Re(e^{-ix} F(k, rho, sigma)) / P^3, x = pi rho k.sigma / (2L).
 *     Synchronous.
 */
bzq_status bzq_plan_info(bzq_plan p, double* out);
bzq_status bzq_plan_pairs(bzq_plan p, double* out);
bzq_status bzq_plan_weights(bzq_plan p, int pair, double* out);

/*
 * Schedule of a plan: the kernel variant of each pipeline stage {0 modulation
 * and FFT along axis 3, 1 plane transforms and product, 2 FFT along axis 3,
 * weighting and accumulation}: 1 = one whole pencil per lane, 2 = two waves
 * per pencil (stages 0, 1: N = 32, 48, 64) or the pipelined producer/consumer
 * kernel (stage 2: N = 16, 24, 32, 48, 64); 3 (stage 1, FP64 at N = 64 only) = the plane
 * taken by column parity in half the LDS; 0 = the default variant.  s_target is the
 * number of workgroups the last stage aims at (512, 1024 or 2048).  Every
 * schedule evaluates eq. realQ; schedules differ in rounding order only
 * (results agree within the precision's tolerance) and one schedule always
 * gives bitwise identical results.
 *   bzq_plan_set_schedule: host sched[4] = {v0, v1, v2, s_target}; EINVAL for a
 *     variant this plan does not have.  No work may be pending on the plan.
 *   bzq_plan_schedule: host out[5] = {v0, v1, v2 as used, s_target, splits}.
 *   bzq_plan_autotune: times evaluations of f_hat (device, as bzq_collision)
 *     under the variants of one stage at a time (and the three s_target values
 *     for the last stage), keeps the fastest and records it in the tuning cache
 *     ($BZQ_TUNE_CACHE or ~/.cache/bzq_autotune.txt; key: N, P, precision,
 *     pairs, chunk).  With use_cache != 0 a recorded schedule is applied without
 *     timing.  Synchronous; uses the plan's own workspace.
 */
bzq_status bzq_plan_set_schedule(bzq_plan p, const int* sched);
bzq_status bzq_plan_schedule(bzq_plan p, int* out);
bzq_status bzq_plan_autotune(bzq_plan p, const double* f_hat, int use_cache, void* stream);

/*
 * Kernel timing for measurement: the launches of the stages selected by
 * `enable` are each bracketed by HIP events on the caller's stream (enable:
 * 0 = off, 1 = every stage, otherwise a mask with bit s set for stage s, e.g.
 * 4 = the plane stage only, which keeps the events off the other launches;
 * the prep stage cannot be selected alone).
 * bzq_plan_stage_times (synchronous) returns into host out[10] the summed
 * milliseconds of the timed launches of each stage {0 prep (ingest, f on the
 * padded grid, accumulator clear), 1 modulate + inverse FFT along axis 3,
 * 2 plane transforms and product, 3 forward FFT along axis 3 + weighting and
 * accumulation, 4 finalisation} followed by the launch count of each stage,
 * and clears the record.  Setting the mask clears it too.
 */
bzq_status bzq_plan_set_timing(bzq_plan p, int enable);
bzq_status bzq_plan_stage_times(bzq_plan p, double* out);

bzq_status bzq_plan_destroy(bzq_plan p);
const char* bzq_status_string(bzq_status s);
const char* bzq_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BZQ_H */
