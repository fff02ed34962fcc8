/*
 * bl_lddmm.h -- C interface of the MI355X (gfx950) library for band-limited PDE-constrained
 * LDDMM on the state equation, optimised by Gauss-Newton-Krylov.
 *
 * Paper: M. Hernandez, "Newton-Krylov optimization in PDE-constrained diffeomorphic
 * registration parameterized in the space of band-limited vector fields" (arXiv:1807.05117).
 *
 * Problem statement (Section 3.2, equation BLEnergy and the constraints after it): given a
 * source image I0 and a target image I1 on a periodic grid, find band-limited velocity
 * coefficients v~ minimising
 *     E(v~) = 1/2 <L~ v~, v~>_l2 + sigma^-2 || m(1) - I1 ||^2,
 *     d_t m + grad m . iota(v~) = 0,  m(0) = I0,
 * with L = (Id - alpha Lap)^s (Section 2.1) applied diagonally in Fourier.
 *
 * Conventions shared by every call
 * --------------------------------
 *  Grid      n[0] x n[1] (x n[2]) voxels, x fastest: voxel (x, y, z) is element
 *            x + n[0] * (y + n[1] * z).  Isotropic voxels of size 1/N_ref with
 *            N_ref = max_j n[j]; the domain is periodic.  For dim == 2, n[2] and k[2] are
 *            ignored (treated as 1).
 *  Images    float32, one value per voxel, prod(n) values.
 *  Band      float32 complex interleaved (re, im), layout [c][kz][ky][kx], c = 0..dim-1 the
 *            velocity component along x, y (, z); index j on an axis of size K stands for
 *            the integer frequency j - K/2, so a band vector holds dim * prod(k) complex
 *            values (2 * dim * prod(k) floats).  The function it represents is
 *                v_c(x_i) = Re sum_k v~_c(k) exp(2 pi i sum_j k_j i_j / n_j).
 *            Inputs are projected onto the admissible set before use: Hermitian
 *            symmetrisation (v~(k) + conj v~(-k)) / 2 and zero on the unpaired planes
 *            k_j = -K_j/2.  Outputs are always admissible.
 *  Inner     <a, b>_l2 = Re sum conj(a) b over the full band; image norms use the unit
 *  products  volume average (1/prod(n)) sum_i.
 *  Time      nt uniform semi-Lagrangian steps of length 1/nt; stationary v~.
 *  Pointers  by default host memory: calls copy inputs to the GPU, compute, copy results
 *            back and return when done.  With BL_DEVICE_PTRS in problem->flags every image
 *            and band pointer is device memory of the current HIP device, and work is
 *            ordered on problem->stream (a hipStream_t, NULL = the null stream).  Scalar
 *            outputs (energy, stats) are always host memory; calls that produce them wait
 *            for the stream.  The library keeps no caller pointer after a call returns.
 *  Errors    every call returns BL_OK (0) or a negative code; bl_lddmm_last_error() gives a
 *            message for the calling thread.  Arguments are validated on the host before
 *            any device work.  No C++ exception crosses this interface.
 *  Results   are deterministic: identical inputs give bitwise identical outputs (fixed
 *            reduction orders, no atomics in value paths).
 */
#ifndef BL_LDDMM_H
#define BL_LDDMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define BL_OK             0
#define BL_E_INVALID     -1   /* bad dim, n, k, nt, alpha, s, sigma, opts or NULL pointer     */
#define BL_E_UNSUPPORTED -2   /* unknown precision, a flag combination or model the call does
                                 not serve (see the flags and the individual calls)             */
#define BL_E_NOMEM       -3   /* the working set does not fit in free device memory         */
#define BL_E_DEVICE      -4   /* a HIP runtime error                                          */
#define BL_E_NONFINITE   -5   /* NaN/Inf in an input, in E, in the gradient or in H v         */
/* -6 (BL_E_CANCELLED) and 1 (BL_PENDING) belong to the serving calls below                   */

/* precision forms */
#define BL_FP32   0   /* FP32 transforms and transports, FP64 reductions                     */
#define BL_MIXED  1   /* band<->grid contractions on BF16 MFMA with split hi/lo operands and
                         FP32 accumulation; FP32 transports; FP64 reductions                  */

/* flags */
#define BL_DEVICE_PTRS 1
/* Hessian products (bl_lddmm_hessvec, contexts, the solver of bl_lddmm_register) are the full
 * Newton ones of the second-order system of Section 2.2 / the Hessian of Section 3.2 equation
 * BLHessianStateEquation: the incremental adjoint keeps its source div(lambda dv) and the
 * product keeps pi(lambda grad dm); without the flag they are Gauss-Newton (Section 3.4). The
 * Newton product may be indefinite away from a minimum; PCG then stops at the first direction
 * of non-positive curvature (the preconditioned gradient if it is the first). Needs 2 Nt + 4
 * more grid planes of device memory (bl_lddmm_footprint includes them). */
#define BL_NEWTON      2
/* Non-stationary velocity: one band field per time node t_n = n / nt, n = 0..nt, so every
 * band velocity argument (v_hat, dv_hat, g_hat, hv_hat, the serving v_hat) holds nt + 1
 * consecutive fields, node-major [n][c][kz][ky][kx].  The regulariser is integrated by the
 * trapezoid rule in time; each semi-Lagrangian step uses the velocity at both of its ends;
 * gradients and products are given per node (the pointwise-in-time expressions of Section 2.2,
 * i.e. representers in the trapezoid-weighted inner product, which the solver uses for its
 * dot products and norms).  Not combined with BL_NEWTON (BL_E_UNSUPPORTED).  Needs 7 (nt - 1)
 * more grid planes of offsets (bl_lddmm_footprint includes them). */
#define BL_NONSTATIONARY 4
/* Deformation state equation (Section 3.3, with the continuous system of Section 2.3): the
 * state is the band displacement u~ = phi~ - id of the inverse map phi, stepped in the band by
 * the classical fourth-order Runge-Kutta method (nt steps) of d_t u~ = -v~ - D~u~ * v~ with
 * truncated convolutions *; the warped source is m(1) = I0 o phi(1) (d-linear interpolation at
 * i + N_ref iota(u~(1))).  The gradient L~ v~ + int (I + D~u~)^T * rho~ dt uses the band adjoint
 * -d_t rho~ - div~(rho~ * v~) = 0 with rho~(1) = pi(lambda(1) (grad I0) o phi(1)), taken as the
 * exact transpose of the Runge-Kutta step; products are Gauss-Newton (the terms that Section
 * 3.4 removes for this method are dropped).  Truncated convolutions are formed on a product
 * grid of 3 K_j / 2 points per axis (rounded up to even).  Stationary velocity; not combined
 * with BL_NEWTON or BL_NONSTATIONARY (BL_E_UNSUPPORTED).  BL_MIXED applies to the image-grid
 * transforms only.  bl_lddmm_ctx_get_field gives BL_FIELD_STATE index 0 (I0) and nt (m(1))
 * only. */
#define BL_DEFORMATION 8

/* registration status */
#define BL_CONVERGED 0
#define BL_MAXITER   1
#define BL_STALLED   2

typedef struct {
  int32_t dim;        /* 2 or 3                                                            */
  int32_t n[3];       /* grid size per axis (x, y, z), 4 <= n[j] <= 2048, prod < 2^30        */
  int32_t k[3];       /* band size per axis, even, 2 <= k[j] <= n[j], k[2] <= 128             */
  int32_t nt;         /* time steps, 1 <= nt <= 256                                         */
  double  alpha;      /* L = (Id - alpha Lap)^s: alpha >= 0                                 */
  int32_t s;          /*                          0 <= s <= 8                               */
  double  sigma;      /* data weight 1/sigma^2, sigma > 0                                   */
  int32_t gamma;      /* incompressibility switch of Section 2.2 (0 or 1; else INVALID):
                         1 restricts v~ to divergence-free band vectors; inputs are projected
                         and gradients and products are their divergence-free parts (the
                         multiplier term gamma grad~ p~ of Section 3.2), per band index
                         v~ - q (q . v~) / |q|^2 with q_j = 2 pi k_j / l_j                    */
  int32_t precision;  /* BL_FP32 or BL_MIXED                                                */
  int32_t flags;      /* BL_DEVICE_PTRS | BL_NEWTON | BL_NONSTATIONARY | BL_DEFORMATION, or 0 */
  void*   stream;     /* hipStream_t used with BL_DEVICE_PTRS (NULL: null stream)           */
} bl_problem;

typedef struct {
  int32_t max_gn;       /* Gauss-Newton iterations, 0 <= max_gn <= BL_MAX_GN (default 10)  */
  int32_t max_pcg;      /* PCG steps per iteration, >= 1 (default 10)                       */
  double  gtol;         /* stop when |g|_inf / |g_0|_inf < gtol (default 1e-3)              */
  double  c1;           /* Armijo constant (default 1e-4)                                   */
  int32_t max_halvings; /* step halvings in the line search, >= 0 (default 10)              */
} bl_solver_opts;

#define BL_MAX_GN 64

typedef struct {
  int32_t status;        /* BL_CONVERGED, BL_MAXITER or BL_STALLED                          */
  int32_t gn_iters;      /* accepted Gauss-Newton iterations                                */
  int32_t hessvecs;      /* Hessian-vector products evaluated                               */
  int32_t gradients;     /* gradients evaluated                                             */
  int32_t evaluations;   /* energy evaluations (initial + line-search trials)               */
  int32_t pcg_total;     /* PCG steps over all iterations                                   */
  double  E[BL_MAX_GN + 1];         /* energy after each accepted iteration (E[0]: start)   */
  double  mse_rel[BL_MAX_GN + 1];   /* 100 |m(1) - I1|^2 / |I0 - I1|^2 (percent)            */
  double  ginf_rel[BL_MAX_GN + 1];  /* |g|_inf / |g_0|_inf                                  */
  int32_t pcg_iters[BL_MAX_GN];     /* PCG steps of each iteration                          */
  int32_t ls_trials[BL_MAX_GN];     /* line-search trials of each iteration                 */
  double  eps[BL_MAX_GN];           /* accepted step length (0 when stalled)                */
  double  seconds;                  /* wall time of the call                                */
} bl_stats;

typedef struct bl_ctx bl_ctx;

/* Default solver options (10 GN iterations, 10 PCG steps, gtol 1e-3, c1 1e-4, 10 halvings). */
void bl_lddmm_default_opts(bl_solver_opts* opts);

/*
 * Gradient of E at v~ (Section 3.2, gradient of the band-limited state-equation method):
 *     g~ = L^ (.) v~ + pi( int_0^1 lambda grad m dt ),
 * with lambda the adjoint of Section 2.2 (equation FirstOrder2, final condition
 * lambda(1) = -(2/sigma^2)(m(1) - I1)), transported backward by semi-Lagrangian steps.
 *   I0, I1   images (prod(n) floats)          v_hat  band vector (input)
 *   g_hat    band vector (output)             energy E(v~) (host, may be NULL)
 */
int bl_lddmm_gradient(const bl_problem* prob, const float* I0, const float* I1,
                      const float* v_hat, float* g_hat, double* energy);

/*
 * Gauss-Newton Hessian-vector product at v~ applied to dv~ (Section 3.2 equation
 * BLHessianStateEquation with the Gauss-Newton rule of Section 3.4): the incremental state
 * is transported forward from dm(0) = 0, the incremental adjoint backward from
 * dlambda(1) = -(2/sigma^2) dm(1), and
 *     H dv~ = L^ (.) dv~ + pi( int_0^1 dlambda grad m dt ).
 * The operator is symmetric positive definite up to discretisation error.
 *   v_hat    point of linearisation        dv_hat  direction        hv_hat  result
 */
int bl_lddmm_hessvec(const bl_problem* prob, const float* I0, const float* I1,
                     const float* v_hat, const float* dv_hat, float* hv_hat);

/*
 * bl_lddmm_hessvec for callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): the same product, arguments,
 * layouts and results, computed in a fixed device scratch array that the library holds on
 * each GPU it runs on until the process ends (bl_lddmm_noalloc_limit() bytes, 512 MiB:
 * enough for 128^3 with Nt = 10).  The call allocates no device, pinned-host or runtime
 * memory and creates no stream or event; with BL_DEVICE_PTRS it runs on problem->stream,
 * else on the null stream, and returns when the result is in hv_hat.  Launch shapes are the
 * ones tuned earlier in the process for the grid (else the defaults); they never change
 * results.  Calls on one GPU share the scratch array and must not overlap: a call while
 * another runs on the same GPU races.  Errors as bl_lddmm_hessvec, plus BL_E_NOMEM (checked
 * on the host before any device work) when the problem's working set exceeds the limit and
 * BL_E_UNSUPPORTED for BL_NONSTATIONARY or BL_DEFORMATION.
 */
int bl_lddmm_hessvec_noalloc(const bl_problem* prob, const float* I0, const float* I1,
                             const float* v_hat, const float* dv_hat, float* hv_hat);
uint64_t bl_lddmm_noalloc_limit(void);

/*
 * Registration by reduced-space Gauss-Newton-Krylov in the band (Section 3.4, equations
 * BLNewton and BLKKT): PCG on H dv~ = -g~ preconditioned by K~ = L~^-1, then
 * v~ <- v~ + eps dv~ with Armijo backtracking (eps = 1, 1/2, ...).
 *   opts     solver options (NULL: defaults)
 *   v_hat    in: initial guess (may be zero); out: result
 *   warped   out: m(1) = I0 transported by the result (prod(n) floats, may be NULL)
 *   stats    out: per-iteration statistics (host, may be NULL)
 */
int bl_lddmm_register(const bl_problem* prob, const bl_solver_opts* opts, const float* I0,
                      const float* I1, float* v_hat, float* warped, bl_stats* stats);

/*
 * Forward state only: warped = m(1), the source transported by the stationary velocity
 * iota(v~) (Section 2.2 equation StateEquation).  I1 is not needed.
 */
int bl_lddmm_warp(const bl_problem* prob, const float* I0, const float* v_hat, float* warped);

/*
 * Band -> grid (Section 3.1, the inclusion iota) of `ncomp` band components (each prod(k)
 * complex, projected first) into `ncomp` grid fields (each prod(n) floats).
 */
int bl_band_to_grid(const bl_problem* prob, int32_t ncomp, const float* band, float* grid);

/*
 * Grid -> band (Section 3.1, the projection pi): band = (1/M) sum_i f_i exp(-2 pi i k.i/n),
 * zero on the unpaired planes, for `ncomp` fields.
 */
int bl_grid_to_band(const bl_problem* prob, int32_t ncomp, const float* grid, float* band);

/*
 * Contexts keep the images and the state of one velocity resident on the device, so that
 * many Hessian-vector products (as inside PCG) reuse the transported state.
 *   ctx_create       copies I0, I1 (host or device per prob->flags); owns device memory
 *                    until ctx_destroy.  *ctx is NULL on error.
 *   ctx_set_velocity setup + forward state + energy at v~ (energy may be NULL); if g_hat is
 *                    not NULL also the gradient.
 *   ctx_hessvec      H dv~ at the velocity last set.  With BL_DEVICE_PTRS it is only
 *                    enqueued on the stream (no wait).
 *   ctx_get_field    copy an internal grid field into out (host or device per flags):
 *                    which = BL_FIELD_* below, index = component or time step.
 * A context is not thread safe; distinct contexts may be used from distinct threads.
 */
int bl_lddmm_ctx_create(const bl_problem* prob, const float* I0, const float* I1, bl_ctx** ctx);
int bl_lddmm_ctx_set_velocity(bl_ctx* ctx, const float* v_hat, double* energy, float* g_hat);
int bl_lddmm_ctx_hessvec(bl_ctx* ctx, const float* dv_hat, float* hv_hat);
int bl_lddmm_ctx_get_field(bl_ctx* ctx, int32_t which, int32_t index, float* out);
void bl_lddmm_ctx_destroy(bl_ctx* ctx);

#define BL_FIELD_VELOCITY 0   /* iota(v~)_c, index = component                               */
#define BL_FIELD_DIV      1   /* iota(div~ v~)                                               */
#define BL_FIELD_X        2   /* forward departure offset (voxels), index = component        */
#define BL_FIELD_Y        3   /* backward departure offset (voxels), index = component       */
#define BL_FIELD_A        4   /* adjoint reaction factor                                     */
#define BL_FIELD_STATE    5   /* m^n, index = time step n in 0..nt                           */

/* Bytes of device memory a context for this problem needs (0 if prob is invalid). */
uint64_t bl_lddmm_footprint(const bl_problem* prob);

/*
 * The one-shot calls (bl_lddmm_register, _gradient, _hessvec, _warp) keep the device context
 * of a successful call (its footprint) and reuse it for the next call on the same problem
 * (same grid, band, nt, alpha, s, sigma, precision, flags, device), so repeated calls
 * allocate no device memory and rebuild no tables.  At most 8 idle contexts and 32 GiB are
 * kept; a call that finds too little free memory frees them first.  Concurrent calls never
 * share a context.  This call frees every idle cached context (it waits for nothing: cached
 * contexts have no work in flight).
 */
void bl_lddmm_release_cached(void);

/* Message of the last error on the calling thread ("" if none). */
const char* bl_lddmm_last_error(void);

/* 1 if a HIP device is visible, else 0 (never fails). */
int bl_lddmm_device_count(void);

/*
 * Per-kernel timing with HIP events, for benchmarks: while enabled, each launch of a timed
 * kernel records an event pair at its own dispatch's start and end (kernel time alone, no gap
 * to its neighbours; up to 4096 launches between reads, later ones are not timed).
 * bl_kernel_timing_read returns the number of timed launches and their summed milliseconds
 * per class and resets: 0 = forward state step, 1 = incremental forward step, 2 = adjoint step,
 * 3 = z stage of iota of the direction in a Gauss-Newton product, 4 = z stage of pi of the
 * product's body force, 5 = body-force pass, 6 = departure-point setup.
 * Classes 3-5 are timed in Gauss-Newton products and gradients of the stationary state
 * equation only.  Errors: BL_E_INVALID for a NULL argument or a class outside [0, 6].
 */
int bl_kernel_timing_enable(bl_ctx* ctx, int32_t on);
int bl_kernel_timing_read(bl_ctx* ctx, int32_t kclass, int64_t* launches, double* ms);

/*
 * Launch shapes of the transport kernels.  A 3D transport launch runs tiles of 64 x 4 x zv
 * voxels (zv voxels per thread along z, zv in {1, 2, 4, 8}) per kernel class: zv_out[0] forward
 * state step, [1] incremental state, [2] adjoint steps, [3] body force.  Every shape computes
 * bitwise the same values.  The library times the candidates on the context's own fields at
 * the first velocity set on a grid shape and keeps the fastest per shape for the process; the
 * environment variable BL_TRANSPORT_ZV = 1, 2, 4 or 8 forces one shape for all classes, and 0
 * keeps the built-in defaults without timing.  Reads the shapes in use (all 1 in 2D, and the
 * defaults before the first velocity).  Errors: BL_E_INVALID for NULL arguments.
 */
int bl_lddmm_ctx_launch_shapes(bl_ctx* ctx, int32_t zv_out[4]);

/*
 * The autotuner: besides the transports' zv, it chooses the setup kernel's voxels per thread
 * and the z-chunking of the FP32 iota z stage, all bitwise-invariant, by timing at the first
 * velocity of each (GPU architecture, grid, band, precision): every candidate is launched
 * once, then all are timed in turn three times over and each keeps its fastest round; another
 * shape must beat the default by 5%.  BL_TUNE_LOG=1 prints the times and choices to stderr.
 * Choices are kept for the process and appended to a cache file read by later processes:
 * BL_TUNE_CACHE (a path, or "off"), else $XDG_CACHE_HOME/bl_lddmm/launch_shapes_v2.txt or
 * ~/.cache/bl_lddmm/launch_shapes_v2.txt (lines with a value a class does not accept are
 * skipped).  BL_LAUNCH_SHAPES="s0,...,s6" fixes all classes
 * (state, incremental, adjoint, body force, setup, iota z, iota x/y); only through it can the
 * iota x/y stages run as one fused kernel with 32 or 16 rows per block (s6 = 32 or 16; 0 = the
 * two separate stages, the default), which times faster alone but runs slower in products.
 * bl_lddmm_tune_reload forgets the choices of this process and reads the cache file again.
 */
void bl_lddmm_tune_reload(void);

/*
 * Serving: a request loop for many registrations on one GPU (continuous batching).
 *
 * Requests (bl_lddmm_register problems, host pointers, any mix of grid sizes, band sizes,
 * time steps and precisions) enter a FIFO queue.  The head of the queue is admitted as soon
 * as a slot is free and its device footprint (bl_lddmm_footprint) fits in the remaining
 * budget; each slot registers its pair on its own HIP stream in a device arena it reuses, so
 * the work of all resident pairs overlaps on the device and a slot takes the next request
 * the moment its pair finishes.  Every result is identical to bl_lddmm_register's on the same
 * inputs (same kernels, same launch shapes, fixed-order reductions).
 *   server_create   budget_bytes: device memory the resident pairs may use (0: 80% of free);
 *                   max_slots: pairs resident at once (1..64); the slots' streams share
 *                   the process's hardware queues (GPU_MAX_HW_QUEUES, 4 unless set), and
 *                   more slots than queues contend: on MI355X four slots served the most
 *                   pairs per second
 *   server_submit   validates, copies I0, I1 (and v_hat if not NULL: initial guess; zero
 *                   otherwise) and returns a ticket; opts may be NULL (defaults); flags must
 *                   not contain BL_DEVICE_PTRS.  BL_E_NOMEM if the footprint exceeds the budget.
 *   server_wait     waits up to timeout_s (< 0: forever) for the request; on completion copies
 *                   v_hat, warped (each may be NULL), stats and times (may be NULL), releases
 *                   the ticket and returns the registration's return code; BL_PENDING if it
 *                   is still queued or running when the timeout expires.
 *   server_cancel   removes a queued request (its wait returns BL_E_CANCELLED); a running one
 *                   completes.
 *   server_destroy  lets running requests finish, drops queued ones, frees everything.
 * Times are seconds since server_create (steady clock).
 */
#define BL_PENDING        1
#define BL_E_CANCELLED   -6

typedef struct bl_server bl_server;

typedef struct {
  double submitted;   /* bl_server_submit returned                                         */
  double admitted;    /* taken by a slot (budget and slot available)                        */
  double finished;    /* result ready                                                       */
  int32_t slot;       /* slot that ran it                                                   */
} bl_request_times;

typedef struct {
  uint64_t budget_bytes;     /* admission budget                                             */
  uint64_t peak_bytes;       /* largest sum of footprints resident at once                  */
  int32_t  max_slots;
  int32_t  peak_resident;    /* most pairs resident at once                                  */
  int64_t  submitted, completed, failed, cancelled;
} bl_server_info;

int bl_server_create(uint64_t budget_bytes, int32_t max_slots, bl_server** server);
/*
 * Cohort server: the same queue, budget, submit / wait / cancel / info / destroy calls, a
 * different engine.  At most max_pairs (1..64) pairs are resident at once.  Requests of equal
 * problems (grid, band, Nt, alpha, s, sigma, gamma, precision) share a cohort of resident
 * pairs, as many as fit the last-level cache with their time-step working sets; every kernel of the
 * Gauss-Newton-Krylov path is one launch for all pairs of a cohort (each pair's buffers at a
 * fixed stride of one arena, a per-pair gate in device memory), and each Newton step -- up to
 * 10 PCG iterations with their stopping tests evaluated on the device, the line-search slope,
 * one Armijo trial, and the gradient at an accepted trial -- is one replay of a HIP graph
 * captured when the cohort is created.  The host reads one control block per pair after a
 * step, records the statistics, retires finished pairs and fills free slots with queued
 * requests of the same problem.  The budget is charged with each cohort's whole arena while
 * the cohort exists (capacity = min(max_pairs, cache-sized count, free budget / footprint)); an empty cohort is
 * freed when a request of another problem needs the memory.  The queue is strictly FIFO.
 * Every result is bitwise the one bl_lddmm_register gives alone (same per-element arithmetic,
 * same reduction order, the same FP64 decisions).  Only the stationary Gauss-Newton
 * state-equation model is served (gamma 0 or 1, BL_FP32 or BL_MIXED): a request with
 * BL_NEWTON, BL_NONSTATIONARY or BL_DEFORMATION completes at once with BL_E_UNSUPPORTED.
 * bl_request_times.slot is the pair's slot within its cohort.
 */
int bl_server_create_batched(uint64_t budget_bytes, int32_t max_pairs, bl_server** server);
int bl_server_submit(bl_server* server, const bl_problem* prob, const bl_solver_opts* opts,
                     const float* I0, const float* I1, const float* v_hat, uint64_t* ticket);
int bl_server_wait(bl_server* server, uint64_t ticket, double timeout_s, float* v_hat,
                   float* warped, bl_stats* stats, bl_request_times* times);
int bl_server_cancel(bl_server* server, uint64_t ticket);
int bl_server_info_get(bl_server* server, bl_server_info* info);
void bl_server_destroy(bl_server* server);

#ifdef __cplusplus
}
#endif
#endif /* BL_LDDMM_H */
