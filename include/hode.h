/*
 * hode — explicit Runge-Kutta time stepping on one AMD Instinct MI355X.
 *
 * C ABI of libhode.so.  Every function returns an int status (HODE_OK = 0,
 * negative on error) unless stated otherwise; no C++ exception crosses this
 * boundary.  After an error, hode_last_error() describes it.
 *
 * Concepts follow the paper's description of Odeint ("Architecture and
 * nomenclature of Boost Odeint"; "The distributed OpenFPM state type and
 * algebra"; the Reuse-potential listings):
 *   - a *state* (the solution vector at time t) is initialised by the caller
 *     and updated in place;
 *   - a *System* right-hand side F(t, u) is selected from a closed set
 *     (exponential, sigmoidal/logistic, 3D Gray-Scott);
 *   - a *stepper* is chosen by type (classical RK4, Runge-Kutta-Dopri5 of
 *     Table 1), and the state is advanced by do_step, integrate_n_steps
 *     (integrate_const) or integrate_adaptive with a tolerance, which returns
 *     the number of steps performed;
 *   - adaptive steppers bound the error with the L-infinity norm of the
 *     embedded error estimate.
 *
 * Ownership: the context owns every device buffer it allocates.  Pointers
 * passed in are borrowed for the duration of the call only (data is copied).
 * Threading: one context per host thread; calls on one context must not
 * overlap.  All device work runs on the context's stream; every call returns
 * after that stream has synchronised.
 *
 * State layout: element-wise systems hold n independent components (nfields
 * 1, ndim 1, shape {n}).  Gray-Scott holds two fields on an N^3 periodic grid
 * (nfields 2, ndim 3, shape {N, N, N}), field-major (u then v), each field
 * with x fastest: element (f, z, y, x) at f*N^3 + x + N*(y + N*z).
 * dtype selects the state precision; time, step size, step control and the
 * error-norm reduction are always FP64.
 */
#ifndef HODE_H
#define HODE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hode_ctx hode_ctx;

enum { HODE_F32 = 1, HODE_F64 = 2 };
enum { HODE_RHS_EXP = 1, HODE_RHS_LOGISTIC = 2, HODE_RHS_GRAYSCOTT3D = 3 };
/* Steppers (the paper's Table 1): classical Runge-Kutta 4; Dormand-Prince
 * 5(4) ("Dopri5", 7 stages, first same as last); Cash-Karp 5(4) (6 stages,
 * Cash & Karp 1990); explicit Euler and the modified midpoint method (Gragg,
 * two substeps of h/2: z1 = y + (h/2) f(y), z2 = y + h f(z1), y_new =
 * (z2 + z1 + (h/2) f(z2)) / 2; fixed steps only); Runge-Kutta-Fehlberg
 * 7(8) (13 stages, Fehlberg 1968; carries the 8th-order solution); and the
 * multi-step Adams-Bashforth methods with s = 1 .. 8 steps, HODE_AB1 + s - 1
 * (fixed steps only; y_{n+1} = y_n + h sum_j beta_j f_{n-j} over the last s
 * right-hand sides, the first s - 1 steps of a fresh history taken by the
 * Fehlberg 7(8) step).  The 5(4) pairs carry the 5th-order solution. */
enum { HODE_RK4 = 1, HODE_DOPRI5 = 2, HODE_CASHKARP54 = 3, HODE_EULER = 4, HODE_FEHLBERG78 = 5, HODE_MIDPOINT = 6 };
enum { HODE_AB1 = 11, HODE_AB2, HODE_AB3, HODE_AB4, HODE_AB5, HODE_AB6, HODE_AB7, HODE_AB8 };
/* Adams-Bashforth-Moulton with s = 1 .. 8 steps, HODE_ABM1 + s - 1 (fixed
 * steps only; the paper's Table 1 multi-step pair): per step f_n = f(y_n),
 * the Adams-Bashforth prediction p, f(p), and the Adams-Moulton correction
 * y_{n+1} = y_n + h (gamma_0 f(p) + sum_{j>=1} gamma_j f_{n+1-j}) over s
 * right-hand sides (order s; two System evaluations per step); history and
 * start-up as for Adams-Bashforth. */
enum { HODE_ABM1 = 21, HODE_ABM2, HODE_ABM3, HODE_ABM4, HODE_ABM5, HODE_ABM6, HODE_ABM7, HODE_ABM8 };
enum { HODE_CTRL_PI = 1, HODE_CTRL_I = 2, HODE_CTRL_MLP = 3 };
enum {
  HODE_OK = 0,
  HODE_EINVAL = -1,        /* bad argument */
  HODE_ESTATE = -2,        /* call out of order: no state / RHS set, or buffer too small */
  HODE_EHIP = -3,          /* HIP runtime error (text in hode_last_error) */
  HODE_ENOMEM = -4,        /* device allocation failed */
  HODE_EDT_UNDERFLOW = -5, /* adaptive step fell below 1e-12 * max(1, |t|) */
  HODE_EMAXSTEPS = -6,     /* attempt budget exhausted before t1 */
  HODE_ENONFINITE = -7     /* step underflow while the error norm was NaN/inf */
};

/* Result of an adaptive integration (also filled for fixed-step runs). */
typedef struct {
  int64_t accepted;  /* steps performed (the paper's return value) */
  int64_t rejected;  /* rejected attempts */
  int64_t rhs_evals; /* System evaluations per element */
  double t;          /* time reached */
  double dt_next;    /* proposed next step */
  double last_err;   /* error norm of the last attempt */
  int32_t status;    /* HODE_OK or the error that ended the run */
  int32_t pad;
} hode_stats;

/* Creates a context on HIP device `device`: the holder of one state, its
 * System and stepper (the objects a user creates before integrating, Reuse
 * potential, main-program listing).  `stream` is a hipStream_t to run on
 * (borrowed, must outlive the context) or NULL for a context-owned stream.
 * *out receives the context (NULL on error). */
int hode_create(hode_ctx **out, int device, void *stream);

/* Frees every device buffer and the context (the end of the objects'
 * lifetime in the same listing).  NULL is ignored. */
void hode_destroy(hode_ctx *ctx);

/* Selects the System.  HODE_RHS_GRAYSCOTT3D takes params = {Du, Dv, F, k, L}
 * (diffusivities, feed, kill, box edge; the paper's Gray-Scott equation with
 * the System listing's +u v^2 - (F+k) v term) with nparams = 5; the
 * element-wise systems take none (params may be NULL).  Invalidates the
 * cached first stage. */
int hode_set_rhs(hode_ctx *ctx, int rhs, const double *params, int nparams);

/* Allocates the state and its stage buffers and copies `src` in (host memory
 * if src_on_device == 0, else device memory).  Element-wise: nfields 1,
 * ndim 1, shape {n}, n >= 0.  Gray-Scott: nfields 2, ndim 3, shape {N,N,N},
 * 1 <= N <= 2048.  The RHS must be set first (HODE_ESTATE otherwise). */
int hode_init_state(hode_ctx *ctx, int dtype, int nfields, int ndim, const int64_t *shape, const void *src,
                    int src_on_device);

/* Copies the current state out (the state the caller reads after
 * integrate_adaptive returns, Reuse potential, main-program listing), in the
 * layout of hode_init_state, to host memory (dst_on_device == 0) or device
 * memory; dst_bytes must be at least the state size (HODE_ESTATE
 * otherwise).  The caller owns dst. */
int hode_read_state(hode_ctx *ctx, void *dst, size_t dst_bytes, int dst_on_device);

/* Size of the state in bytes (0 before init): 2 N^3 or n elements of the
 * state precision (layout above). */
size_t hode_state_bytes(const hode_ctx *ctx);

/* Absolute and relative tolerance of the error norm
 * max_i |e_i| / (atol + rtol * max(|y_i|, |ynew_i|)) (the predefined
 * tolerance adaptive steppers keep the embedded estimate within, measured in
 * the L-infinity norm: Architecture and nomenclature of Boost Odeint).
 * Both >= 0, not both 0 (HODE_EINVAL).  Defaults: 1e-6, 1e-6. */
int hode_set_tolerances(hode_ctx *ctx, double atol, double rtol);

/* Step-size controller for adaptive runs: HODE_CTRL_PI (default,
 * Gustafsson PI), HODE_CTRL_I (elementary), or HODE_CTRL_MLP with `weights`
 * the packed bf16 parameters of the 16-64-64-1 network (nbytes = 2 * 5313:
 * W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3), copied in.  The PI
 * proposal remains the fallback and retry rule. */
int hode_set_controller(hode_ctx *ctx, int kind, const void *weights, size_t nbytes);

/* One fixed step of size dt from time t, in place (Odeint do_step); any
 * stepper. */
int hode_do_step(hode_ctx *ctx, int method, double t, double dt);

/* n fixed steps (Odeint integrate_const with n = (tf - t0)/dt):
 * t_n = t0 + n dt.  *t_end (may be NULL) receives t_n.
 * Adams-Bashforth keeps its history of right-hand sides in the context, as an
 * Odeint stepper object does: a call with the same s and dt continues it (n
 * steps in several calls equal n in one); a different s or dt, any other
 * stepping call, hode_set_rhs or hode_init_state starts a fresh history.
 * Its ring of s right-hand sides (and, Gray-Scott, the 12 Fehlberg stage
 * arrays for the start-up) is allocated on first use. */
int hode_integrate_n_steps(hode_ctx *ctx, int method, double t0, double dt, int64_t n, double *t_end);

/* Embedded pair of the adaptive calls (hode_try_step,
 * hode_integrate_adaptive, hode_integrate_times): HODE_DOPRI5 (default),
 * HODE_CASHKARP54 or HODE_FEHLBERG78.  All use the same error norm; the
 * controller's exponents follow the embedded order (k = 5 for the 5(4)
 * pairs, 8 for Fehlberg 7(8): alpha = 0.7/k, beta = 0.4/k, reject factor
 * 0.9 err^(-1/k)).  The learned controller (trained on the 5(4) pairs) is
 * refused with Fehlberg 7(8) (HODE_EINVAL at the integrate call).  Not for
 * ensemble contexts (they step with Dopri5). */
int hode_set_stepper(hode_ctx *ctx, int method);

/* One error-controlled attempt of size *dt from *t.  On acceptance *t
 * advances and the state is updated; either way *dt receives the proposed
 * next step and *accepted 0/1.  Controller history carries over between
 * calls until the next integrate call. */
int hode_try_step(hode_ctx *ctx, double *t, double *dt, int *accepted);

/* Error-controlled integration from t0 to t1 with the adaptive stepper
 * (Odeint integrate_adaptive), first
 * trial step dt0, at most max_steps attempts.  The last step is clipped to
 * land on t1 exactly.  Returns HODE_OK or the status that ended the run; the
 * state holds the last accepted step either way.  `out` may be NULL. */
int hode_integrate_adaptive(hode_ctx *ctx, double t0, double t1, double dt0, int64_t max_steps, hode_stats *out);

/* Odeint integrate_times with a recording observer: the state at times[0]
 * is the current one; the adaptive stepper then advances to times[1],
 * times[2], ... (strictly increasing) in turn, each step clipped to land on
 * them exactly, carrying the proposed step and the controller's memory from
 * one to the next.  dst receives n_times states back to back (layout as
 * hode_read_state; host or device memory, dst_bytes >= n_times * state
 * bytes).  max_steps bounds the attempts of the whole call; at the first
 * failing status the call stops (later slots are not written) and returns
 * it.  `out` (may be NULL) receives the summed stats; traces keep the last
 * interval's attempts. */
int hode_integrate_times(hode_ctx *ctx, const double *times, int64_t n_times, double dt0, int64_t max_steps,
                         void *dst, size_t dst_bytes, int dst_on_device, hode_stats *out);

/* Dense output (Odeint's dense-output Dopri5 with integrate_times): Dopri5
 * error-controlled steps from times[0] to times[n_times-1], exactly those of
 * hode_integrate_adaptive over that interval (only the last step clipped,
 * to land on the end; same counts and final state), while the state at each
 * intermediate times[i] comes from the continuous extension of the accepted
 * step that covers it (Dormand & Prince 1986, 4th order: the quartic through
 * y_n and y_{n+1} with end slopes k1 and k7 plus a correction from all
 * stages).  Slot i of dst (n_times states, as for hode_integrate_times)
 * receives the state at times[i]; slot 0 the current state, the last slot
 * the end state.  The device loop pauses between graph chunks after the
 * step that reaches the next requested time, interpolates there and goes
 * on.  Gray-Scott keeps k6 for it (one more array, allocated on first use;
 * stage 6 then writes it); the element-wise families evaluate the step's
 * stages again in registers.  Adaptive stepper HODE_DOPRI5 only
 * (HODE_EINVAL otherwise).  Returns as hode_integrate_times does. */
int hode_integrate_times_dense(hode_ctx *ctx, const double *times, int64_t n_times, double dt0, int64_t max_steps,
                               void *dst, size_t dst_bytes, int dst_on_device, hode_stats *out);

/* Statistics of the last run (accepted steps are the step count that
 * integrate_adaptive returns, Reuse potential; rejected attempts and System
 * evaluations beside it). */
int hode_get_stats(hode_ctx *ctx, hode_stats *out);

/* Checkpoint of the step control (with the state from hode_read_state, what
 * a restarted run needs to continue an error-controlled step sequence).
 * Layout of the blob, version 1: */
typedef struct {
  uint32_t magic;          /* HODE_CKPT_MAGIC */
  uint32_t version;        /* 1 */
  double t;                /* time reached */
  double dt_next;          /* proposed next step */
  double err_prev;         /* PI memory: the last accepted error norm (1 before any) */
  int32_t last_rejected;   /* the last attempt was rejected (no growth on the next accept) */
  int32_t hist_n;          /* attempts in the learned controller's history (<= 4) */
  double hist_lerr[4], hist_lh[4], hist_acc[4];  /* that history, newest first */
  int64_t accepted, rejected, rhs_evals;           /* counters of the last call */
} hode_checkpoint;
#define HODE_CKPT_MAGIC 0x48434b50u

/* Writes the control state at the end of the last stepping call into blob
 * (*nbytes in: its size; out: the size written, sizeof(hode_checkpoint)).
 * blob == NULL only reports the size.  HODE_ESTATE before any stepping. */
int hode_get_ctrl(hode_ctx *ctx, void *blob, size_t *nbytes);

/* Restores a checkpoint: the next hode_try_step continues its controller
 * memory (err_prev, last_rejected, history), so try_step sequences split by
 * a checkpoint and a restore (into this or a fresh context, after
 * hode_init_state with the saved state) equal the unsplit sequence bitwise
 * when called with the saved t and dt_next.  hode_integrate_adaptive and
 * the multi-step histories start afresh as always.  HODE_EINVAL for a blob
 * of another size, magic or version. */
int hode_set_ctrl(hode_ctx *ctx, const void *blob, size_t nbytes);

/* Doubles per trace record: h, err, accepted, t after, dt proposed, PI
 * log-ratio, learned log-ratio or NaN, landed-on-t1 flag, then for accepted
 * attempts the 16 learned-controller features, else NaN.  A trace buffer
 * for cap records holds cap * HODE_TRACE_W doubles. */
#define HODE_TRACE_W 24

/* Records one HODE_TRACE_W-double entry per adaptive attempt (the accept /
 * reject history the step control produces, the training data of the learned
 * controller) for the next runs, up to `capacity` attempts (0 disables).  The
 * trace is device memory owned by the context. */
int hode_set_trace(hode_ctx *ctx, int64_t capacity);

/* Copies up to `cap` recorded entries (cap * HODE_TRACE_W doubles) to host
 * `dst` (owned by the caller; NULL with cap 0 only queries); *n receives
 * the number of attempts of the last run (may exceed cap). */
int hode_read_trace(hode_ctx *ctx, double *dst, int64_t cap, int64_t *n);

/* Evaluates the System at the current state into dst (same layout/dtype as
 * the state). */
int hode_eval_rhs(hode_ctx *ctx, void *dst, size_t dst_bytes, int dst_on_device);

/* Launch mode of the integration loop: enable != 0 (default) replays
 * captured hipGraph chunks of attempts; 0 enqueues every stage and control
 * kernel on the stream instead (same kernels and results; for comparing
 * launch overhead on small, launch-bound grids). */
int hode_set_graphs(hode_ctx *ctx, int enable);

/* Gray-Scott tile configuration: ry in {1, 2, 4} rows per wavefront (tile of
 * 64*vw x nw*ry cells per workgroup of nw wavefronts), zc >= 1 z-planes per
 * workgroup, for every stage kind.  Element-wise: `ry` is ignored and zc is
 * the workgroup count cap. */
int hode_set_tile(hode_ctx *ctx, int ry, int zc);
int hode_get_tile(const hode_ctx *ctx, int *ry, int *zc);  /* the widest stage's tile */

/* Gray-Scott wavefronts per workgroup for the tiles set next and now: 4
 * (default) or 8.  Eight-wavefront tiles (twice the rows per tile, so half
 * the halo rows per row of the grid) exist for the RK4, Dopri5, Cash-Karp
 * and Euler stage kinds with ry <= 2 and 16-byte lanes (vw 4 for FP32, 2
 * for FP64); every other kind keeps 4.  Results are bitwise the same. */
int hode_set_tile_waves(hode_ctx *ctx, int nw);

/* The tile of one stage kind (numbered as for hode_time_kernel): rows per
 * wavefront, planes per workgroup, wavefronts per workgroup (HODE_ESTATE
 * before a Gray-Scott state exists). */
int hode_get_kind_tile(const hode_ctx *ctx, int kind, int *ry, int *zc, int *nw);

/* Gray-Scott cells per lane (1, 2 or 4; fp64 at most 2; must divide N), or 0
 * for the widest that divides N (16-byte loads where possible). */
int hode_set_vector_width(hode_ctx *ctx, int vw);

/* Times `reps` launches of one stage kernel (Gray-Scott: kind 0..50 as D1,
 * R2, R3, R4, D2..D7, D7F, C4, C5, C6, C6F, E1, D6F, F1..F13, F13F,
 * AB1..AB8, D6K, ABC1..ABC8 (the Adams-Moulton correctors, which write the
 * state), MM1..MM3; element-wise: kind = method) on the context's
 * stream with HIP events and returns the mean duration in milliseconds.
 * The state is left unchanged for Gray-Scott non-final kinds only; timing an
 * Adams-Bashforth kind ends the Adams-Bashforth history. */
int hode_time_kernel(hode_ctx *ctx, int kind, int reps, double *avg_ms);

/* Gray-Scott: runs `reps` attempts of `method` (RK4: stages D1 R2 R3 R4;
 * DOPRI5: stages D2..D7 of an adaptive attempt; CASHKARP54: D1 D2 D3 C4 C5
 * C6; FEHLBERG78: F1..F13; HODE_AB<s>: its one kernel) with the control
 * kernel in a no-op timing mode, HIP events around every stage kernel on the
 * context's stream, and writes the mean duration of each stage in
 * milliseconds to ms[0 .. stages-1] (ms holds at least 13).  The current
 * state is left unchanged (and k1 = f(y)); Adams-Bashforth ends its history. */
int hode_profile_attempt(hode_ctx *ctx, int method, int reps, double *ms);

/* Gray-Scott: times one attempt of `method` for every tile configuration
 * (ry in {1,2,4}; zc the powers of two 8 .. 256 and ceil(N / k) for k = 1 ..
 * 12, at least 8; 4 or, where the kind has them, 8 wavefronts per workgroup)
 * with hode_profile_attempt and keeps, for every stage kernel
 * of the attempt, its fastest configuration (the first k1 and the fixed-step
 * stage variants take those of their shape twins); returned are the widest
 * stage's (stage 6 of Dopri5 and Cash-Karp, stage 4 of RK4, stage 13 of
 * Fehlberg 7(8), the one kernel of Adams-Bashforth) and the sum of the stages'
 * best times (ms); any output pointer may be NULL.  Results are bitwise
 * identical for every tile.  hode_set_tile sets one tile for all stages. */
int hode_autotune(hode_ctx *ctx, int method, int reps, int *best_ry, int *best_zc, double *best_ms);

/* Testing aid: fills every buffer the library may use as scratch (the spare
 * state buffer, the stage arrays, the extra arrays, the first-same-as-last
 * slot unless it holds a valid k1, the Adams ring unless a history is live)
 * with NaN bit patterns, so a kernel that read one before writing it in the
 * same call would spoil its result.  Leaves the state and every carried
 * quantity intact. */
int hode_debug_poison(hode_ctx *ctx);

/* hode_autotune with a persistent cache: the tiles of every stage kind are
 * read from the text file at cache_path when it holds an entry for this
 * device architecture, precision, method, grid edge and cells-per-lane
 * setting (the last such entry wins), else found with hode_autotune and
 * appended to the file as one line ("hode-tune-v2 <arch> <dtype> <method>
 * <N> <vw>" and ry:zc:nw for every kind).  cache_path NULL: the environment
 * variable HODE_TUNE_CACHE; without either no file is used.  *from_cache
 * (may be NULL) receives 1 when the tiles came from the file.  HODE_EINVAL
 * if the file cannot be written. */
int hode_autotune_cached(hode_ctx *ctx, int method, int reps, const char *cache_path, int *from_cache);

/* Measurement reference: copies `bytes` (a multiple of 16) from device
 * buffer src to device buffer dst (both 16-byte aligned; HODE_EINVAL
 * otherwise, and for reps < 1) with a plain 16-byte-per-lane streaming
 * kernel, `reps` times after one warm-up, on a stream of its own; returns the
 * mean duration per copy in milliseconds.  Used as the achievable-bandwidth
 * ceiling and to calibrate HBM traffic counters. */
int hode_stream_copy(void *dst, const void *src, size_t bytes, int reps, double *avg_ms);

/* ---- batched ensemble ------------------------------------------------------
 * n independent Gray-Scott instances (uneven grid edges and parameters), each
 * with its own adaptive Dopri5 step control (the paper's integrate_adaptive,
 * Reuse potential), stepped together by a persistent kernel captured once in
 * a hipGraph.  By default one launch carries the whole integration: every
 * unfinished instance advances in lock step, one attempt per round; a round
 * is six stage phases and one control phase separated by grid-wide
 * barriers; in a stage phase the workgroups claim tiles (rows and planes of
 * one instance) from eight per-XCD queues, their own XCD's first, so every
 * phase is balanced dynamically; finished instances skip their tiles, and
 * the launch ends when every instance is done.  Each time the number of
 * running instances has halved, the kernel re-cuts the running ones into
 * tiles sized for them (ensembles of up to 2048 instances), so the last,
 * largest instances still spread over every workgroup.  Every instance's arithmetic
 * and step decisions are those of the single-grid path, so results are
 * bitwise those of running the instance alone. */

/* Creates an ensemble context: instance i has grid edge edges[i] (1..1024) and
 * params[5*i .. 5*i+4] = {Du, Dv, F, k, L}; dtype HODE_F32 or HODE_F64.  All
 * instance buffers are allocated here (9 arrays of 2 N^3 elements each). */
int hode_ensemble_create(hode_ctx **out, int device, void *stream, int n, const int64_t *edges,
                         const double *params, int dtype);
int hode_ensemble_size(const hode_ctx *ctx);

/* Copies instance i's initial state in (layout as hode_init_state). */
int hode_ensemble_init_state(hode_ctx *ctx, int i, const void *src, int src_on_device);
int hode_ensemble_read_state(hode_ctx *ctx, int i, void *dst, size_t dst_bytes, int dst_on_device);

/* Per-attempt work estimates (> 0, any common unit), one per instance, used
 * to deal the instances to the per-XCD tile queues (default: the cells the
 * instance's tiles cover, rows padded to the 64-lane tile width). */
int hode_ensemble_set_weights(hode_ctx *ctx, const double *w);

/* Split the integration into launches: at most `first` attempts per
 * instance in the first launch and `rest` in every later one (1 .. 4096),
 * the host relaunching with the instances still running (a resumed
 * instance keeps its first-same-as-last stage, so results are unchanged).
 * Both 0 (the default): one launch for the whole integration. */
int hode_ensemble_set_epoch(hode_ctx *ctx, int first, int rest);

/* Polls a grid barrier of the persistent ensemble kernel makes before it
 * gives up (at least 1; default 2^24: each poll sleeps briefly and re-reads
 * the barrier's device-scope counter, so a wait that no legitimate phase
 * needs ends in seconds, not minutes).  A barrier that gives
 * up sets an error flag on which every workgroup leaves the kernel, and the
 * integration returns HODE_EHIP; the instances' states are then undefined
 * until they are initialised again.  This bounds every wait of the kernel
 * (failure detection if workgroups were ever not all resident) and lets a
 * test force that path from the host. */
int hode_ensemble_set_barrier_limit(hode_ctx *ctx, int64_t polls);

/* The last integration's summed kernel durations (HIP events around every
 * launch, in ms) and its number of launches; either pointer may be NULL. */
int hode_ensemble_timing(hode_ctx *ctx, double *kernel_ms, int *launches);

/* Cells per lane of instance i's tiles: 1, 2 or 4 (fp64: 1 or 2), dividing N.
 * With 16-byte lanes (4, fp64 2) and rows of at most 32 lanes, the tiles
 * pack one row per segment of a wavefront (the default for such grids). */
int hode_ensemble_set_vector_width(hode_ctx *ctx, int i, int vw);

/* Planes per tile of instance i's tiles (>= 1, kept for the whole
 * integration; 0, the default: sized so a phase has about half a tile per
 * workgroup, and re-sized as instances finish), and the tile of instance i:
 * vector width and planes per tile. */
int hode_ensemble_set_plane_chunk(hode_ctx *ctx, int i, int zc);
int hode_ensemble_get_tile(const hode_ctx *ctx, int i, int *vw, int *zc);

/* Per-instance attempt traces, HODE_TRACE_W doubles per attempt with the
 * fields of hode_set_trace; capacity is per instance.  read_trace copies up
 * to cap records (cap * HODE_TRACE_W doubles) of instance i to host dst and
 * stores the instance's attempt count of the last run in *n. */
int hode_ensemble_set_trace(hode_ctx *ctx, int64_t capacity);
int hode_ensemble_read_trace(hode_ctx *ctx, int i, double *dst, int64_t cap, int64_t *n);

/* Tile autotuner of the ensemble: times the persistent kernel on a twin of
 * the whole ensemble (same edges and parameters, started from this
 * ensemble's current states; this ensemble is unchanged; the twin's buffers
 * are allocated for the call) for `reps` attempts per candidate.  Edge by
 * edge, largest total cells first, every cells-per-lane width dividing the
 * edge is tried for that edge's instances (16-byte lanes give segmented rows
 * where rows are at most 32 lanes, narrower widths 64-lane rows) with the
 * other edges at their current choice, and the width with the shortest
 * kernel time is kept.  The instances' planes per tile are reset to 0 (sized
 * from the running cells, re-cut as instances finish).  With the environment
 * variable HODE_TUNE_CACHE naming a text file, choices recorded there for
 * this architecture, precision, instance count, workgroup count and edge
 * list are used without timing, and new ones are appended (one line per
 * edge: "hode-ens-tune-v2 <arch> <dtype> <n> <workgroups> <edge-list hash>
 * <N> <vw> <ms>").  vw_out (n entries, may be NULL) receives each
 * instance's width; ms_out (n entries, may be NULL) the twin's kernel time
 * in ms of the last edge's chosen candidate, the same for every instance. */
int hode_ensemble_autotune(hode_ctx *ctx, int reps, int *vw_out, double *ms_out);

/* Integrates every instance from t0 to t1 (first trial step dt0, at most
 * max_steps attempts each; tolerances and controller of the context), each
 * with its own integrate_adaptive step control (Reuse potential).
 * per_instance (may be NULL) receives n stats.  Returns HODE_OK, the first
 * failing instance's status, or HODE_EHIP if a HIP call failed or a wait of
 * the persistent kernel gave up (hode_ensemble_set_barrier_limit). */
int hode_ensemble_integrate_adaptive(hode_ctx *ctx, double t0, double t1, double dt0, int64_t max_steps,
                                     hode_stats *per_instance);

/* ---- learned step-size controller: network kernels --------------------------
 * The 16-64-64-1 tanh network of HODE_CTRL_MLP (packed parameters as in
 * hode_set_controller, 5313 values).  All pointers are device memory owned by
 * the caller; work runs on `stream` (a hipStream_t, NULL = default stream) and
 * the calls return after it synchronised.  Arithmetic: bf16 weights, inputs
 * and first-layer activations, fp32 accumulation on the matrix cores, as in
 * the controller's own evaluation.
 *   X: rows of 16 features (fp32, row-major); T: one target per row; Wt:
 *   one sample weight per row; idx: B row indices (int64, each a valid row
 *   of X, T and Wt) giving minibatch sample b = row idx[b], or NULL for
 *   rows 0 .. B-1 (the kernels gather the rows as they load them);
 *   Wb: bf16 bits of the parameters; Wm: fp32 master parameters;
 *   grad, m, v: 5313 fp32 each; acc: 2 doubles of scratch. */
int hode_mlp_forward(const uint16_t *Wb, const float *X, float *Y, int64_t B, void *stream);
/* Wb = bf16 rounding (to nearest, ties to even) of Wm. */
int hode_mlp_quantize(const float *Wm, uint16_t *Wb, void *stream);
/* grad = d/dparams of sum_b Wt_b (y_b - T_b)^2 / sum_b Wt_b over the B
 * minibatch samples (B >= 1); *loss_out (may be NULL) receives the loss. */
int hode_mlp_loss_grad(const uint16_t *Wb, const float *X, const float *T, const float *Wt, const int64_t *idx,
                       int64_t B, float *grad, double *acc, double *loss_out, void *stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, step >= 1, learning rate
 * lr) on Wm from the gradient at Wb over the minibatch; refreshes Wb;
 * *loss_out receives the loss before the step. */
int hode_mlp_train_step(const float *X, const float *T, const float *Wt, const int64_t *idx, int64_t B, float *Wm,
                        uint16_t *Wb, float *m, float *v, float *grad, double *acc, int64_t step, float lr,
                        double *loss_out, void *stream);

/* hode_mlp_train_step for callers that cannot allocate (code under HIP
 * graph capture, tight training or serving loops, harnesses that forbid
 * allocation): no gradient or scratch argument, and the call allocates
 * nothing.  The gradient (5313 fp32) and the two loss sums live in a
 * library-owned device array of 21.5 KB per GPU (the GPU running `stream`,
 * the current device for NULL), set up on the first call on that GPU and
 * held until the process ends; every call clears it before use.  Calls on
 * one GPU share that array: calls that overlap on one GPU (other streams,
 * other host threads) race and must be serialised by the caller.  B is 1 ..
 * HODE_MLP_NOALLOC_MAX_B samples (HODE_EINVAL otherwise); other arguments
 * and results as hode_mlp_train_step. */
#define HODE_MLP_NOALLOC_MAX_B 2147483647LL
int hode_mlp_train_step_noalloc(const float *X, const float *T, const float *Wt, const int64_t *idx, int64_t B,
                                float *Wm, uint16_t *Wb, float *m, float *v, int64_t step, float lr,
                                double *loss_out, void *stream);

/* Text of the last error on this context (valid until the next call on it;
 * owned by the context). */
const char *hode_last_error(const hode_ctx *ctx);

/* HODE_TRACE_W of the built library (for bindings that cannot read this
 * header). */
int hode_trace_width(void);

#ifdef __cplusplus
}
#endif

#endif /* HODE_H */
