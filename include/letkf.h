/*
 * letkf.h -- C ABI of the MI355X (gfx950) local ETKF library.
 *
 * The library keeps an m-member ensemble of the adaptive-optics state
 * resident in device memory and advances it one frame at a time:
 *
 *   letkf_analyse   per-domain local ETKF update from one slope frame
 *                   (paper Sec. 2.2-2.3: every estimation domain is updated
 *                   from its own observation region, independently).
 *   letkf_forecast  AR(1)/AR(2) prediction of every member (Sec. 2.1).
 *   letkf_submit_frame  the same two steps driven by a serving loop that
 *                   batches the frames of several resident instances into
 *                   shared kernel launches.
 *
 * State (Sec. 2.1): x_k = [phi_k ; phi_{k-1}] on the n_act valid actuators,
 * n = 2 n_act.  Observations (Sec. 2.1, Sec. 3): x then y slope of each
 * of the n_sub valid subapertures, p = 2 n_sub, through the WFS matrix D
 * (p x n_act, CSR), observing the current instant, H = [D 0], or the
 * previous one, H = [0 D] (letkf_model.obs_instant).
 *
 * Analysis of domain l (actuators E_l, subapertures O_l; ensemble-space ETKF
 * of the paper's refs [8]-[10], localized per ref [14]):
 *   X' = X - xbar 1^T,  Y' = H X' = D X'_obs,  d = y - D xbar_obs  (obs: the
 *   observed instant's rows),
 *   r = taper * R^-1 on O_l,   C = Y'_O^T diag(r) Y'_O,   b = Y'_O^T diag(r) d_O,
 *   A = (m-1)/rho I + C = U Lambda U^T,  wbar = A^-1 b,
 *   W = U ((m-1) Lambda^-1)^(1/2) U^T  (symmetric root, ref [9]),
 *   Z_l = xbar_E 1^T + X'_E (W + wbar 1^T);
 * rows covered by several domains are merged with the map's weights
 * (whole-pupil reconstruction, Sec. 3.2).
 *
 * Forecast: phi_{k+1} = a1 .* phi_k + a2 .* phi_{k-1} + sigma_v z, with z
 * standard normal from Philox4x32-10 (Salmon et al., SC'11):
 *   counter = (member, actuator, frame mod 2^32, frame div 2^32),
 *   key = (seed mod 2^32, seed div 2^32);  outputs (x0..x3) give
 *   u1 = ((x0 2^21 + x1 div 2^11) + 1/2) 2^-53, u2 likewise from (x2, x3),
 *   z = sqrt(-2 ln u1) cos(2 pi u2).  frame = number of forecasts done
 *   since create (or the value given to letkf_set_state).
 *
 * Conventions for every call
 *   - Every function returns an int status: LETKF_OK (0) or a negative code.
 *     No C++ exception crosses this interface.  letkf_last_error() returns a
 *     thread-local message for the last failure of the calling thread.
 *   - "host" pointers are ordinary CPU memory, "device" pointers are HIP
 *     device memory of the handle's GPU.  All host input arrays are read
 *     (and copied where needed) before the call returns; the caller keeps
 *     ownership of every pointer it passes.
 *   - Matrices are row-major.  Ensemble matrices are n x m: row = state
 *     variable (rows 0..n_act-1 = phi_k, n_act..n-1 = phi_{k-1}), column =
 *     member.
 *   - stream: a hipStream_t passed as void* (NULL = the default stream).
 *   - Limits: 2 <= m <= 256 (above 128: LETKF_FP64 only, no
 *     LETKF_FLAG_PISTONS, plain path only; the analysis is then a sequence of
 *     launches over per-domain scratch, the global ETKF of Sec. 3.1);
 *     n_act, n_sub >= 1; every domain has >= 1 actuator.  Violations return
 *     LETKF_EINVAL before any device work.
 *   - A handle is used by one thread at a time.
 */
#ifndef LETKF_H
#define LETKF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define LETKF_OK        0
#define LETKF_EINVAL   (-1)  /* invalid argument, map or dimension */
#define LETKF_ENOMEM   (-2)  /* workspace / arena too small, HBM budget exceeded */
#define LETKF_EAGAIN   (-3)  /* no free frame slot; try again */
#define LETKF_EDEVICE  (-4)  /* a HIP runtime call failed */
#define LETKF_ENUMERIC (-5)  /* non-finite input, or the eigensolver did not converge */
#define LETKF_ESTATE   (-6)  /* call not valid in the handle's state (e.g. no debug buffers) */

/* ---- precision paths --------------------------------------------------
 * The eigensolve (Cholesky, one-sided Jacobi rotations), wbar and W are FP64
 * on every path (the rotations unless LETKF_FLAG_FP32_ROTATIONS is given);
 * the paths differ in the storage of the ensemble and slopes
 * and in the two dense contractions, C = Y'^T diag(r) Y' and X' T.
 * LETKF_FP64: ensemble, slopes and both contractions in FP64 (C on FP64
 *             MFMA for m <= 64, FP64 FMA above); Jacobi tolerance 32 M eps.
 * LETKF_FP32: FP32 ensemble and slopes; C on FP32 MFMA (v_mfma_f32_16x16x4f32),
 *             each 4-observation k-step's FP32 product added into an FP64
 *             accumulator; X' T on FP32 MFMA with FP32 accumulation; Jacobi
 *             tolerance 1e-6 and two refinement steps of wbar.
 * LETKF_BF16: FP32 ensemble and slopes; C on BF16 MFMA from split operands
 *             (sqrt(r) Y' = hi + lo, both BF16; hi hi^T + hi lo^T + lo hi^T)
 *             with FP32 accumulation; X' T on BF16 MFMA with BF16 X' and a
 *             hi + lo split of T, FP32 accumulation; Jacobi tolerance 1e-4 and
 *             three refinement steps of wbar; m <= 128.
 * b = Y'^T diag(r) d is accumulated in FP64 on every path.                 */
#define LETKF_FP64 0
#define LETKF_FP32 1
#define LETKF_BF16 2

/* ---- create flags ----------------------------------------------------- */
#define LETKF_FLAG_DEBUG 0x1u  /* keep per-domain C, lambda, T for letkf_debug_domain */
/* Remove the differential pistons between domain estimates before the merge
 * (Sec. 3.2 names the step, not its method).  Each domain's analysed rows of
 * each instant and member are shifted by one constant, chosen by least
 * squares so that domains agree on the actuators they share (minimum-norm
 * solution of the overlap-graph normal equations, then the constant that
 * keeps each member's merged phase sum).  The create call forms the
 * n_dom x n_dom operator on the host (O(n_dom^3) once) and keeps it in the
 * workspace (8 n_dom^2 bytes). */
#define LETKF_FLAG_PISTONS 0x2u
/* letkf_step replays a hipGraph of the frame's launch sequence (slopes,
 * analysis, pistons, merge + forecast, state advance), captured at the first
 * step on a private stream of the handle and launched on the caller's stream
 * afterwards; the slope upload and the read-back of the means stay ordinary
 * copies around it.  Every kernel reads the frame's state from the device
 * (ring slot, frame counter), so the graph is replayed unchanged.  While
 * kernel timing is enabled, letkf_step launches the kernels one by one. */
#define LETKF_FLAG_GRAPH 0x4u
/* LETKF_BF16 only, opt-in: the Jacobi rotations run in FP32 instead of FP64
 * (L rounded to FP32 in LDS, rotated to the path's tolerance 1e-4, widened
 * back for lambda, wbar and W, which stay FP64).  A departure from the FP64
 * eigensolve: each rotation rounds at ~6e-8, far below the tolerance, and it
 * is faster where several workgroups share a CU.  Instances with the flag
 * form a batch class of their own in the server.  LETKF_EINVAL with any
 * other precision. */
#define LETKF_FLAG_FP32_ROTATIONS 0x8u

typedef struct letkf_handle letkf_handle;
typedef struct letkf_server letkf_server;

typedef struct letkf_dims {
  int32_t n_act;  /* valid actuators (state n = 2 n_act) */
  int32_t n_sub;  /* valid subapertures (slopes p = 2 n_sub) */
  int32_t m;      /* ensemble members, 2..256 (above 128: FP64 only) */
} letkf_dims;

typedef struct letkf_model {
  const double* a1;        /* host [n_act]: AR coefficient of phi_k */
  const double* a2;        /* host [n_act]: AR coefficient of phi_{k-1} (0 gives AR(1)) */
  double sigma_v;          /* model-noise std added to phi_{k+1}; >= 0 */
  const double* r_inv;     /* host [p]: diagonal of R^-1 (inverse slope-noise variance); >= 0 */
  int32_t d_nnz;           /* nonzeros of D */
  const int32_t* d_rowptr; /* host [p+1]: CSR row pointers of D (p x n_act) */
  const int32_t* d_col;    /* host [d_nnz]: actuator index of each nonzero */
  const double* d_val;     /* host [d_nnz] */
  double inflation;        /* rho > 0; 1 = no inflation */
  uint64_t seed;           /* Philox key of the model noise */
  int32_t obs_instant;     /* which instant the slopes observe (Sec. 2.1: the state holds two):
                              0 = phi_k, H = [D 0] (pseudo-open-loop slopes of the current
                              instant); 1 = phi_{k-1}, H = [0 D]; other values LETKF_EINVAL */
} letkf_model;

typedef struct letkf_domain_map {
  int32_t n_domains;
  const int32_t* est_ptr;   /* host [n_domains+1]: CSR into est_act/est_w */
  const int32_t* est_act;   /* host: actuators of each estimation domain (both instants updated) */
  const double* est_w;      /* host: merge weight of each (domain, actuator); for every actuator
                               the weights of the domains covering it sum to 1 (|sum-1| <= 1e-9) */
  const int32_t* obs_ptr;   /* host [n_domains+1]: CSR into obs_sub/obs_taper */
  const int32_t* obs_sub;   /* host: subapertures of each observation region (x and y slope used) */
  const double* obs_taper;  /* host: localisation weight in [0,1], multiplies R^-1 of both slopes */
} letkf_domain_map;

/* ---- single instance -------------------------------------------------- */

/* Bytes of device workspace letkf_create needs for this problem. */
int letkf_workspace_size(const letkf_dims* dims, const letkf_model* model,
                         const letkf_domain_map* map, int precision, uint32_t flags,
                         size_t* bytes);

/* Validates everything, lays the problem out in the caller's device
 * workspace (>= letkf_workspace_size bytes, 256-byte aligned; owned by the
 * caller and never freed by the library), uploads D, the map, the model and
 * the initial ensemble X0 (host, n x m FP64, converted to the path's
 * storage precision) on `stream`, and returns a handle.  Frame counter = 0. */
int letkf_create(const letkf_dims* dims, const letkf_model* model, const letkf_domain_map* map,
                 int precision, uint32_t flags, const double* X0, void* workspace,
                 size_t workspace_bytes, void* stream, letkf_handle** out);

/* Releases host-side state (pinned staging, tables).  Waits for the
 * handle's outstanding work.  The workspace stays the caller's. */
int letkf_destroy(letkf_handle* h);

/* Analysis of the resident forecast ensemble with slopes y (p values, FP64;
 * host pointer if y_on_device == 0, else device).  Host y is copied before
 * return.  If mean_out (host [n_act]) is non-NULL the analysis mean of
 * phi_k is written there and the call waits for the stream; otherwise the
 * call is asynchronous on `stream`.  Non-finite host slopes: LETKF_ENUMERIC. */
int letkf_analyse(letkf_handle* h, const double* y, int y_on_device, double* mean_out, void* stream);

/* AR forecast of the resident ensemble to the next frame (asynchronous on
 * `stream`); advances the frame counter. */
int letkf_forecast(letkf_handle* h, void* stream);

/* One frame of the plain path: analyse(y) then forecast.  If pred_out (host
 * [n_act]) is non-NULL it receives the prediction mean of phi_{k+1} and the
 * call waits for completion. */
int letkf_step(letkf_handle* h, const double* y, int y_on_device, double* pred_out, void* stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid allocation): one frame of the
 * plain path, like letkf_step with device slopes, that allocates nothing -
 * no device memory, no pinned staging, no host synchronisation.  y_dev
 * (device [p] FP64) is read by the frame's kernels; pred_dev (device
 * [n_act] FP64) receives the prediction mean of phi_{k+1}; both are the
 * caller's and must stay valid until the stream reaches the frame.
 * Asynchronous on `stream`.  The frame's scratch (slope perturbations,
 * innovation, per-domain analysis rows, the copies of A on the FP64 path,
 * analysis means, and the descriptor copies that point the kernels there)
 * lives in a static device array of the library, 32 MiB per GPU, held until
 * the process ends, instead of the instance workspace: LETKF_EINVAL when the
 * frame needs more (e.g. 84x84 subapertures with m = 64 needs about 26 MB in
 * FP64, 10 MB in FP32/BF16) or m > 128.  Every such call on one GPU shares
 * that array, so calls that overlap on one GPU (other streams, other
 * threads) race and must be ordered by the caller.  The first call on a GPU
 * looks the array's address up (make it outside a graph capture).  Device
 * slopes are not checked for non-finite values; letkf_last_means does not
 * see these frames. */
int letkf_step_noalloc(letkf_handle* h, const double* y_dev, double* pred_dev, void* stream);

/* Copies the ensemble (host [n x m] FP64, rows [phi_k; phi_{k-1}]) and the
 * frame counter out (frame_out may be NULL); waits for the stream. */
int letkf_get_state(letkf_handle* h, double* X_out, uint64_t* frame_out, void* stream);

/* Replaces the ensemble (host [n x m] FP64) and the frame counter. */
int letkf_set_state(letkf_handle* h, const double* X, uint64_t frame, void* stream);

/* Per-domain intermediates of the last analysis (needs LETKF_FLAG_DEBUG):
 * C_out [m x m] (C = Y'^T diag(r) Y', no (m-1)/rho I), lam_out [m]
 * (ascending eigenvalues of A), T_out [m x m] (W + wbar 1^T), sweeps_out
 * (Jacobi sweeps used), cycles_out [5] (shader-clock cycles spent by the
 * domain's workgroup in: gather + C/b, Cholesky, Jacobi, wbar/W/T, update).
 * Any output may be NULL.  Waits for the stream. */
int letkf_debug_domain(letkf_handle* h, int32_t domain, double* C_out, double* lam_out,
                       double* T_out, int32_t* sweeps_out, double* cycles_out, void* stream);

/* Where each domain's analysis ran in the last analysis (needs
 * LETKF_FLAG_DEBUG; m <= 128): hw_id_out the workgroup's HW_ID register
 * (shader engine, shader array, CU and SIMD fields, as the ISA defines
 * them), xcc_id_out its XCC_ID register (the XCD), workgroup_out the
 * index of the analysis workgroup that took it, start_clock_out the shader
 * clock when it started (comparable within one XCD).  A tool for
 * studying how the analysis workgroups are spread over the CUs.  Any output
 * may be NULL.  Waits for the stream. */
int letkf_debug_placement(letkf_handle* h, int32_t domain, uint32_t* hw_id_out, uint32_t* xcc_id_out,
                          int32_t* workgroup_out, double* start_clock_out, void* stream);

/* Shader-clock cycles of the sub-steps of the wbar/W/T phase of a domain in
 * the last analysis (needs LETKF_FLAG_DEBUG; m <= 128): cycles_out [4] =
 * {lambda and U from the columns of L J, wbar = U Lambda^-1 U^T b, its
 * refinement, T}.  Waits for the stream. */
int letkf_debug_substeps(letkf_handle* h, int32_t domain, double* cycles_out, void* stream);

/* Number of domains whose eigensolver hit the sweep cap in the last analysis
 * (0 when all converged); waits for the stream. */
int letkf_unconverged_domains(letkf_handle* h, int32_t* count, void* stream);

/* The means the last plain-path frame wrote (host [n_act] each, either may
 * be NULL): amean_out the analysis mean of phi_k (letkf_analyse or
 * letkf_step), pmean_out the prediction mean of phi_{k+1} (letkf_forecast or
 * letkf_step).  A two-frame-delay controller extrapolates with both, e.g.
 * phi_{k+2|k} = a1 pmean + a2 amean (eq. (1) applied to the means).  Waits
 * for the stream. */
int letkf_last_means(letkf_handle* h, double* amean_out, double* pmean_out, void* stream);

/* Kernel timing of the plain path: while enabled, analyse/forecast/step
 * record HIP events on their stream around each kernel.  enable = 1 clears
 * and starts, 0 stops.  ms_out (nullable, [3]) receives the accumulated
 * milliseconds of {slope synthesis, domain analysis, merge/forecast} and
 * frames_out (nullable) the number of timed frames; reading waits for the
 * recorded events.  At most 65536 frames are timed per enable. */
int letkf_kernel_times(letkf_handle* h, int enable, double* ms_out, uint64_t* frames_out);

/* Order in which an instance's domains become work items of the analysis
 * launch (workgroup b takes the b-th first, further ones are claimed in
 * order). */
#define LETKF_ORDER_MAP 0   /* the domain map's order */
#define LETKF_ORDER_COST 1  /* decreasing cost (actuators + subapertures): the default */
#define LETKF_ORDER_XCD 2   /* the map's order cut into 8 contiguous chunks, position b from chunk b % 8: \
                               workgroup b runs on XCD b % 8, so neighbouring domains share an L2 */
#define LETKF_ORDER_BALANCED 3 /* plain instances only, placed by measured cost: the Jacobi sweeps    \
                                  of each domain so far (summed over every analysis of the instance). \
                                  When every domain's workgroup is resident at once: LETKF_ORDER_XCD  \
                                  with each XCD's domains re-placed among its CUs so that the costliest \
                                  run alone on a CU or with the cheapest company; otherwise longest    \
                                  first.  Computed when applied (letkf_autotune, letkf_set_tuning),    \
                                  from the sweeps at that time */

/* Result of an autotuning run of the domain-analysis launch. */
typedef struct letkf_tuning {
  int32_t grid;           /* analysis workgroups per launch chosen (persistent: they share the items) */
  int32_t order;          /* LETKF_ORDER_* */
  int32_t blocks_per_cu;  /* analysis workgroups of this class one CU holds at once */
  int32_t candidates;     /* configurations timed */
  float best_us;          /* mean analysis launch time of the choice (microseconds) */
  float default_us;       /* same for the default: LETKF_ORDER_COST, grid = min(domains, blocks_per_cu x CUs) */
} letkf_tuning;

/* Picks the analysis launch shape of this instance by timing it on its own
 * resident data: the grid of the persistent analysis kernel (how many
 * domains run on a CU at once: ceil(k x CUs / 2) workgroups, k = 1 ..
 * 2 x blocks_per_cu, or one per domain; capped at the domain count) and the
 * order in which the domains are claimed (LETKF_ORDER_*).  Each
 * candidate is timed over `reps` launches (1..100) after one warm-up, with
 * HIP events on `stream`.  The fastest candidate is chosen, except that the
 * best LETKF_ORDER_XCD or LETKF_ORDER_BALANCED candidate wins when it is
 * within 2 % of it (they read less from HBM for the same time); the choice is
 * kept by the handle (a captured LETKF_FLAG_GRAPH frame is re-captured).  The
 * balanced order is placed by the sweeps of the analyses so far including
 * the tuning launches, which all analyse the current frame.  The instance's
 * state (ensemble, frame and sweep counters, per-domain sweep sums) is
 * unchanged; letkf_debug_domain reads the
 * tuning runs' intermediates until the next analysis.  Results of later
 * frames do not depend on the choice: every domain's analysis is computed
 * the same way whichever workgroup runs it.  `out` may be NULL.  Waits for
 * the stream. */
int letkf_autotune(letkf_handle* h, int32_t reps, letkf_tuning* out, void* stream);

/* Applies a launch shape chosen earlier (say a letkf_tuning kept from a
 * letkf_autotune run on the same GPU model and domain map): grid in
 * [1, 65535] workgroups (more than the domain count acts as the domain
 * count) and order (LETKF_ORDER_*; LETKF_ORDER_BALANCED is placed by the
 * sweeps of the analyses so far, so applying it again after some frames
 * re-balances); the other fields are ignored.  Waits for the stream.
 * LETKF_EINVAL for out-of-range fields. */
int letkf_set_tuning(letkf_handle* h, const letkf_tuning* t, void* stream);

/* Totals since create (or set_state): Jacobi sweeps over all domain solves,
 * and the number of domain solves.  Waits for the stream. */
int letkf_sweep_stats(letkf_handle* h, uint64_t* sweeps, uint64_t* domain_solves, void* stream);

/* ---- serving: many resident instances, batched frames ----------------- */

/* Completion callback: called once per submitted frame from the server's
 * completion thread (holding no server lock), after pred_out has been
 * written.  status is LETKF_OK or a negative code.  It may submit further
 * frames; it must not call letkf_server_drain, _remove or _destroy. */
typedef void (*letkf_done_fn)(void* user, uint64_t frame_id, int status);

/* A server sub-allocates instance workspaces from the caller's device arena
 * (arena_bytes = the HBM budget, 256-byte aligned; letkf_server_reserved_bytes
 * of it hold the server's own tables and staging) and runs one scheduler
 * thread.  Instances fall into classes (padded ensemble size 16/32/64/128 x
 * arithmetic variant: the precision, with LETKF_FLAG_FP32_ROTATIONS a variant
 * of its own); a batch holds the oldest pending frame of several instances of
 * one class (at most max_batch), every domain of which is one work item of
 * one analysis launch.  Up to 8 batches run at once, each on a stream of its
 * own, so the batches of different classes overlap on the GPU.  An instance
 * has at most one frame in flight; its frames run in submission order.
 * A batch's analysis runs in the persistent kernel with the class's grid
 * (letkf_server_autotune; by default as many workgroups as the GPU holds at
 * once, at most one per domain item).  While batches can overlap (more
 * admitted instances than max_batch, or instances of several classes), the
 * grid of a class that fits two or more analysis workgroups on a CU is capped
 * one workgroup per CU below that, so the slope and merge kernels of the
 * batches beside it start at once.  flags: 0 or LETKF_SERVER_GRAPHS. */
int letkf_server_create(void* arena, size_t arena_bytes, int32_t max_batch, uint32_t flags,
                        letkf_server** out);

/* Server flag: each batch's kernels (slope synthesis, analysis, pistons,
 * merge + forecast, state advance) are replayed from a hipGraph captured on
 * the first batch of the same shape (class, analysis grid, pistons, and the
 * power-of-two buckets of its slope rows, domains and actuators) on the same
 * staging slot; the uploads of the batch header and slopes and the download
 * of the means stay ordinary copies around the replay.  The kernels read the
 * batch's composition from the slot's header, so one graph serves every
 * batch of that shape. */
#define LETKF_SERVER_GRAPHS 0x1u

/* Times the analysis launch of every class with admitted instances on their
 * resident data (a batch of up to max_batch of them, as letkf_autotune does
 * for one instance) and keeps the fastest grid per class (within the cap on
 * overlapping batches described at letkf_server_create); the instances'
 * domain orders are set to the fastest order.  out (nullable) has
 * LETKF_SERVER_CLASSES (16) entries, one per class: padded size 16/32/64/128
 * x arithmetic variant, index variant x 4 + size, with variant = precision
 * (FP64 0, FP32 1, BF16 2) or 3 for LETKF_BF16 with
 * LETKF_FLAG_FP32_ROTATIONS; classes without instances are zeroed.  Only while
 * idle: LETKF_EAGAIN when frames are queued or in flight.  Frames submitted
 * during the call wait until it returns.  Instance states are unchanged. */
#define LETKF_SERVER_CLASSES 16
int letkf_server_autotune(letkf_server* s, int32_t reps, letkf_tuning* out);

/* Sets the analysis grid of class cls (index variant x 4 + size, as in
 * letkf_server_autotune's output) and the domain order of its admitted
 * instances (instances admitted later keep the default order).  Only while
 * idle (LETKF_EAGAIN otherwise); LETKF_EINVAL for out-of-range fields and
 * for LETKF_ORDER_BALANCED (a batch's workgroup placement depends on the
 * batch). */
int letkf_server_set_tuning(letkf_server* s, int32_t cls, const letkf_tuning* t);

/* Bytes of a server's arena taken by its own instance table and staging
 * buffers (independent of the instances admitted). */
size_t letkf_server_reserved_bytes(void);

/* Admits one instance (same arguments as letkf_create).  LETKF_ENOMEM when
 * the remaining arena cannot hold its workspace. */
int letkf_server_add(letkf_server* s, const letkf_dims* dims, const letkf_model* model,
                     const letkf_domain_map* map, int precision, uint32_t flags, const double* X0,
                     letkf_handle** out);

/* Removes an idle instance (no frame in flight) and returns its workspace to
 * the arena.  LETKF_EAGAIN while it still has frames in flight. */
int letkf_server_remove(letkf_server* s, letkf_handle* h);

/* Queues one frame of instance h: y (host [p] FP64) is copied before return;
 * the frame is analyse(y) then forecast, and pred_out (host [n_act], owned by
 * the caller, valid until cb fires) receives the prediction mean of phi_{k+1}.
 * Frames of one instance run in submission order.  LETKF_EAGAIN when the
 * instance's queue (64 frames) is full. */
int letkf_submit_frame(letkf_handle* h, const double* y, uint64_t frame_id, double* pred_out,
                       letkf_done_fn cb, void* user);

/* As letkf_submit_frame, with the slopes already in device memory: y_dev
 * ([p] FP64, on the server's GPU) is read by the batch's kernels directly and
 * must stay unchanged until cb fires.  Device slopes are not checked for
 * non-finite values. */
int letkf_submit_frame_device(letkf_handle* h, const double* y_dev, uint64_t frame_id, double* pred_out,
                              letkf_done_fn cb, void* user);

/* Blocks until every submitted frame has completed. */
int letkf_server_drain(letkf_server* s);

/* Batching window (default 100 us): a class is launched as soon as every
 * idle instance of it (no frame in flight) has a pending frame; otherwise its
 * oldest pending frame waits at most this long for the others.  0 launches
 * every frame as soon as it arrives. */
int letkf_server_set_window(letkf_server* s, uint32_t window_us);

/* Counters since create: frames completed, batches launched, sum of batch
 * sizes (any pointer may be NULL). */
int letkf_server_stats(letkf_server* s, uint64_t* frames, uint64_t* batches, uint64_t* batched_frames);

/* Drains, stops the scheduler and frees host state; instance handles of the
 * server become invalid.  The arena stays the caller's. */
int letkf_server_destroy(letkf_server* s);

/* ---- errors, build ------------------------------------------------------ */
const char* letkf_strerror(int status);
/* Hash of the sources the library was built from (16 hex digits). */
const char* letkf_build_id(void);
const char* letkf_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LETKF_H */
