/*
 * swe.h - C ABI of the MI355X shallow-water step library (libswe.so).
 *
 * The library advances the 2-D nonlinear shallow-water equations of Madden,
 * Marras & Suckale (arXiv 2301.12010), Methods, Eqs. (1)-(3), in the vector
 * form u_t + F_x + G_y = S of Eq. (4) with u = (h, hu, hv):
 *   - fifth-order WENO reconstruction at every half-step face (Methods, WENO
 *     paragraph) of the Lax-Friedrichs split fluxes F+- = (F +- alpha u~)/2,
 *     u~ = (h + m, hu, hv), with alpha the global maximum characteristic
 *     speed of each RK stage (Methods, Lax-Friedrichs paragraph, Eq. (6));
 *   - the pressure flux 1/2 g (h^2 - m^2) and the bed source
 *     -g (h + m) grad b, centred at the cell, its face values of b
 *     reconstructed with the normal-momentum flux's WENO weights, and the
 *     explicit Manning friction -g n^2 |q| q / h^(7/3) (Eqs. (2)-(3), (7)).
 *     m = min(b, 0) takes the bed relative to the datum (the still-water
 *     level 0): below it this is the printed form with b, and on land
 *     (m = 0) the depth form 1/2 g h^2, -g h grad b, under which dry land
 *     carries no flux and still water at the datum stays at rest exactly;
 *   - the three-stage TVD Runge-Kutta update of Eq. (8).
 * Options (off by default): point-implicit friction in place of the explicit
 * term (SWE_OPT_FRICTION_IMPLICIT) and a compensated FP32 level
 * (SWE_OPT_COMPENSATED).
 * All arithmetic of the state is FP32 on the GPU; FP64 is kept for time and
 * the mass diagnostics.  No call takes or returns a torch type.  Device
 * memory comes from hipMalloc or from a caller allocator
 * (swe_set_allocator).
 *
 * Arrays are row-major [ny][nx] float32 with x fastest (element (i, j) at
 * j * nx + i).  Input and output pointers may be host or device memory; the
 * runtime's unified addressing tells them apart.  Callers keep ownership of
 * every array they pass; the library copies inputs and owns its device
 * buffers.  No function throws; each returns an SWE_* code.
 */
#ifndef SWE_H
#define SWE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ------------------------------------------------------- */
#define SWE_OK 0
#define SWE_EINVAL (-1)     /* bad argument: sizes, spacing, non-finite or negative field */
#define SWE_ENOMEM (-2)     /* device allocation failed or the memory budget is exceeded */
#define SWE_EDEVICE (-3)    /* a HIP runtime call failed */
#define SWE_ENONFINITE (-4) /* a wave speed became non-finite; the state is poisoned */
#define SWE_EBUSY (-5)      /* the server's request queue is full */
#define SWE_ENOTFOUND (-6)  /* unknown ticket or scenario index */

/* ---- boundary kinds (per side: west, east, south, north) ---------------- */
/* REFLECT: three mirrored ghost layers, normal momentum odd (the free-slip,
 *          no-penetration walls of Section 2.4 and the reflective walls of the
 *          dam-break workload).
 * FIXED:   ghost (h, hu, hv) frozen at the create-time values of the nearest
 *          interior cell, bed extended linearly: the constant-height zero-flux
 *          (Section 2.1), Dirichlet (Section 2.2) and inflow/outflow
 *          (Section 2.3) conditions of the verification problems. */
#define SWE_BC_REFLECT 0
#define SWE_BC_FIXED 1

/* Problem parameters (plain data, copied by the library). */
typedef struct swe_params {
    int32_t nx, ny;    /* cells in x and y; each >= 3 */
    double dx, dy;     /* cell sizes [m], > 0 */
    double g;          /* gravity [m/s^2]; the paper uses 9.81 */
    double cfl;        /* > 0: dt = cfl / (alpha_x/dx + alpha_y/dy) from u^n;
                          <= 0: fixed dt = dt_fixed (the paper's runs use 5e-3) */
    double dt_fixed;   /* used when cfl <= 0; must then be > 0 */
    double h_dry;      /* wet/dry threshold [m]: wet <=> h > h_dry */
    double weno_eps;   /* WENO5 epsilon added to the smoothness indicators */
    double kappa_cap;  /* > 0: friction rate capped at kappa_cap/dt; <= 0: no cap */
    int32_t bc[4];     /* SWE_BC_* for west, east, south, north */
} swe_params;

/* Diagnostics returned with a read. */
typedef struct swe_stats {
    double t;          /* simulated time [s] (FP64 sum of the step sizes) */
    int64_t step;      /* completed RK3 steps */
    double mass;       /* sum of h dx dy over the grid (FP64 sum of the FP32 state) */
    double clamp_mass; /* mass added by clamping h < 0 to 0, weighted by how much
                          of each stage's clamp reaches u^(n+1) (1/6, 2/3, 1) */
    double dt;         /* step size of the next step (from the current state) */
    float alpha_x;     /* global max |u| + sqrt(g h) of the current state */
    float alpha_y;     /* global max |v| + sqrt(g h) */
    float runup;       /* max bed elevation b > 0 of any wet cell so far (0 if none) */
    int32_t status;    /* SWE_OK or SWE_ENONFINITE */
} swe_stats;

/* ---- single scenario ---------------------------------------------------- */
typedef struct swe_ctx swe_ctx;

/* Create a scenario on the current HIP device: the inputs of the paper's
 * problem statement (Methods: bathymetry b, Manning n, the initial state
 * (h, hu, hv), the resolution; Sections 2.1-2.4 for the boundary kinds).
 * b is the bed elevation [m] relative to the datum (the still-water level),
 * manning_n the Manning coefficient per cell, (h0, hu0, hv0) the initial
 * state; all [ny][nx] float32, host or device.  hip_stream is a hipStream_t
 * (NULL: the library creates its own); every later call of this context is
 * ordered on it.  Errors: SWE_EINVAL for nx or ny < 3, a grid of 2^30 or
 * more elements once rows are padded to multiples of 64, dx or dy <= 0,
 * cfl <= 0 with dt_fixed <= 0, an unknown boundary kind, or any non-finite
 * value, h0 < 0 or manning_n < 0; SWE_ENOMEM, SWE_EDEVICE otherwise.  On
 * error *out is NULL. */
int swe_create(const swe_params *p, const float *b, const float *manning_n,
               const float *h0, const float *hu0, const float *hv0,
               void *hip_stream, swe_ctx **out);

/* Enqueue nsteps RK3 steps (Methods, Eqs. (7)-(8): three stage launches
 * each, every stage the WENO5 / Lax-Friedrichs operator with the bed and
 * Manning sources; dt from the CFL condition, computed on the device).
 * Asynchronous; never blocks; a non-finite state surfaces at the next
 * swe_read.  nsteps < 0 is SWE_EINVAL; 0 is a no-op. */
int swe_step(swe_ctx *ctx, int32_t nsteps);

/* Wait for the context's stream, then copy the state (any of h, hu, hv may
 * be NULL) and the diagnostics (stats may be NULL): the solution fields the
 * paper's runs write out (Section 3), with the time, the mass (Section 2,
 * conservation) and the runup (Section 2.4).  Returns SWE_ENONFINITE once a
 * wave speed became non-finite (the copies are still made). */
int swe_read(swe_ctx *ctx, float *h, float *hu, float *hv, swe_stats *stats);

/* Release the context's device memory.  NULL-safe. */
void swe_destroy(swe_ctx *ctx);

/* Context options (swe_set_option keys). */
#define SWE_OPT_GRAPH_STEPS 1 /* steps per captured hipGraph segment; 0 = plain launches (default 32) */
#define SWE_OPT_TILE 2        /* tile variant index, see swe_tile_info; -1 = automatic (default) */
/* 1: keep the FP32 rounding residual of the stored level in three more
 * planes (12 bytes per cell) and combine the RK stages with error-free sums,
 * so that increments below half an ulp of the level are kept; removes the
 * FP32 mass drift of shallow wet/dry runs (up to 6e-10 of the mass per step
 * otherwise; about 1e-13 with it).  Costs 8-12 more bytes of traffic per
 * cell and stage and about 4% more time per step.  0 (default): off.  Can
 * be switched at any time (the residual then starts at zero; the captured
 * graph is dropped).  Returns SWE_EINVAL for other values, SWE_ENOMEM when
 * the planes cannot be allocated (the option is then off).  Batches take it
 * through swe_batch_set_option and servers through swe_server_set_option. */
#define SWE_OPT_COMPENSATED 3
/* 1: point-implicit Manning friction (Methods: the paper keeps friction
 * explicit and names an implicit treatment as the alternative it declines).
 * Each RK stage takes its own friction term backward in time with the rate
 * kappa = g n^2 |q| / h^(7/3) of the stage input, uncapped (kappa_cap is
 * ignored): q_out = [a_n q^n + a_w (q + dt L')] / (1 + a_w dt kappa), L' the
 * right-hand side without friction, (a_n, a_w) = (0, 1), (3/4, 1/4),
 * (1/3, 2/3).  Stable for any friction stiffness; first order in dt where the
 * friction dominates.  0 (default): the explicit term of the paper.  Can be
 * switched at any time (the captured graph is dropped); other values are
 * SWE_EINVAL.  Batches and servers take it through swe_batch_set_option and
 * swe_server_set_option. */
#define SWE_OPT_FRICTION_IMPLICIT 4
/* 1: local Lax-Friedrichs splitting (Methods, Lax-Friedrichs paragraph: the
 * paper splits with the global maximum speed of each stage).  Each face
 * takes the largest normal speed |u_n| + sqrt(g h+) over the six cells its
 * two reconstructions read and splits those cells with it; the face flux
 * stays single-valued (conservative) and still water stays at rest.  Less
 * viscosity where the flow is slow (wet/dry fronts); the time step stays
 * global.  Each face then reconstructs its own split values (no sharing
 * between neighbouring faces), about twice the arithmetic.  0 (default):
 * the global speed.  Can be switched at any time (the captured graph is
 * dropped); other values are SWE_EINVAL.  Batches and servers take it
 * through swe_batch_set_option and swe_server_set_option. */
#define SWE_OPT_LOCAL_SPLIT 5
int swe_set_option(swe_ctx *ctx, int32_t key, int64_t value);

/* Device addresses of the context's live state (depth h, hu, hv of u^n) and
 * the row pitch in elements, for callers that keep results on the GPU.  The
 * library stores the level h + min(b, 0) rather than h (precise surface
 * elevation in deep water); the h plane returned is a depth copy that this
 * call refreshes on the context's stream and that stays valid until the next
 * swe_step or swe_time_stages.  hu and hv are the live planes and change only
 * through those two calls. */
int swe_state_device(swe_ctx *ctx, float **h, float **hu, float **hv, int64_t *pitch);

/* Measurement: run nsteps steps with plain launches, bracketing every stage
 * kernel with HIP events on the context's stream; ms[0..2] receive the mean
 * device duration of the stage-1, -2 and -3 launches.  Blocks until done.
 * The steps advance the state as swe_step does (requested outputs are taken,
 * a tracked maximum-depth map is updated). */
int swe_time_stages(swe_ctx *ctx, int32_t nsteps, double *ms);

/* ---- outputs during a run ------------------------------------------------
 * The paper's runs write the state at chosen output times while the solver
 * advances (Section 3, host orchestration of the replicated computation);
 * here snapshots are taken on the device and streamed to the host on a copy
 * stream, and a maximum-depth (inundation) map is kept on the device. */

/* Request snapshots at n output times (simulated seconds, finite,
 * non-decreasing).  Output k is the state at the end of the first step,
 * enqueued after this call, whose time t >= times[k]; a step that passes
 * several output times serves all of them.  A snapshot is copied on the
 * device when taken and then copied to library-owned pinned host memory on
 * a copy stream while later steps run (the transfer is enqueued by the next
 * swe_step or swe_output_get call after the snapshot's step has finished).
 * Memory: 12 bytes per cell and output, on the device and on the host.
 * Replaces any previous request; n = 0 clears.  Errors: SWE_EINVAL for
 * n < 0 or n > 65536, times NULL with n > 0, non-finite or decreasing times;
 * SWE_ENOMEM. */
int swe_set_outputs(swe_ctx *ctx, const double *times, int32_t n);

/* Output k (0 <= k < n of the last swe_set_outputs).  Returns 1 after
 * copying it into the caller's [ny][nx] arrays (any of h, hu, hv, t, step
 * may be NULL); 0 if it is not available: with wait = 0, not yet on the
 * host; with wait != 0, the steps enqueued so far do not reach times[k]
 * (the call first waits for them and for the transfer).  SWE_EINVAL for k
 * out of range. */
int swe_output_get(swe_ctx *ctx, int32_t k, int32_t wait, float *h, float *hu, float *hv,
                   double *t, int64_t *step);

/* Maximum-depth map: with enable != 0, keep for every cell the maximum of h
 * over the state at the call and the state after every later step (updated
 * inside the last RK stage's store); enable = 0 drops the map.  Enabling
 * again restarts it.  SWE_ENOMEM if the plane cannot be allocated. */
int swe_track_max_depth(swe_ctx *ctx, int32_t enable);

/* Wait for the context's stream, then copy the maximum-depth map ([ny][nx]).
 * SWE_EINVAL if the map is not being kept or hmax is NULL. */
int swe_read_max_depth(swe_ctx *ctx, float *hmax);

/* ---- the same run without allocation -------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.
 * swe_run_noalloc computes what swe_create + swe_step(nsteps) + swe_read
 * compute for one scenario (bitwise the same state and diagnostics; the
 * tile variant is the automatic one), but on the caller's device arrays and
 * without any allocation: the scenario's working storage (swe_footprint
 * bytes) is a fixed device array of the library, SWE_NOALLOC_MAX_BYTES long,
 * that every GPU the library runs on holds until the process ends.
 *   b, manning_n: bed and Manning n, [ny][nx] float32 device arrays (read).
 *   h, hu, hv: the initial state on entry, the state after nsteps steps on
 *     return, [ny][nx] float32 device arrays, advanced in place; time starts
 *     at 0 and the FIXED ghosts are frozen at the entry state.
 *   hip_stream: the hipStream_t every kernel is enqueued on (NULL: the null
 *     stream).
 *   stats: NULL makes the call asynchronous: kernels only, no copy, no
 *     synchronisation, so it can be captured into a graph and replayed.
 *     Non-NULL waits for the stream and fills the diagnostics of swe_read.
 * Errors: SWE_EINVAL for invalid parameters (as swe_create), nsteps < 0, a
 * NULL or non-device array, a scenario whose footprint exceeds
 * SWE_NOALLOC_MAX_BYTES (about 1.5 million cells: 1024 x 1024 fits), or,
 * with stats, input fields that are non-finite or have h < 0 or n < 0 (the
 * arrays then hold no meaningful state); SWE_EDEVICE for a failed runtime
 * call; with stats, SWE_ENONFINITE as swe_read.  All calls on one GPU share
 * its array and each leaves its contents behind: calls that overlap on one
 * GPU (on different streams or host threads) race and must be serialised by
 * the caller. */
#define SWE_NOALLOC_MAX_BYTES (64ull << 20)
int swe_run_noalloc(const swe_params *p, const float *b, const float *manning_n, float *h,
                    float *hu, float *hv, int32_t nsteps, void *hip_stream, swe_stats *stats);

/* ---- tile variants and autotuning --------------------------------------- */
/* Tile variants of the stage kernel: tile width tx, height ty, cells per
 * thread along a sweep r, threads per block. Results are bitwise identical
 * across variants.  Returns SWE_ENOTFOUND past the last variant. */
int swe_tile_info(int32_t index, int32_t *tx, int32_t *ty, int32_t *r, int32_t *threads);
int swe_tile_count(void);

/* Time every tile variant on a synthetic nx-by-ny problem and return the
 * fastest.  With cache_path non-NULL the result is looked up in / added to
 * that JSON file, keyed by (nx, ny, gfx arch). */
int swe_autotune(int32_t nx, int32_t ny, const char *cache_path, int32_t *best_tile,
                 double *best_ms_per_step);

/* ---- batched scenarios (one launch sequence for all) -------------------- */
typedef struct swe_batch swe_batch;

/* Empty batch bound to hip_stream (NULL: own stream). */
int swe_batch_create(void *hip_stream, swe_batch **out);

/* Add a scenario with its own grid, fields and step count (>= 0); *index
 * receives its position.  Same validation as swe_create. */
int swe_batch_add(swe_batch *bt, const swe_params *p, const float *b, const float *manning_n,
                  const float *h0, const float *hu0, const float *hv0, int32_t nsteps,
                  int32_t *index);

/* Advance every scenario by min(max_steps, its remaining steps) in one run:
 * one persistent launch, or one launch per stage round (see
 * swe_batch_set_mode); max_steps < 0 runs to completion.  Asynchronous. */
int swe_batch_run(swe_batch *bt, int32_t max_steps);

/* Wait, then copy scenario `index` (pointers may be NULL). */
int swe_batch_read(swe_batch *bt, int32_t index, float *h, float *hu, float *hv, swe_stats *stats);

/* Launch modes of swe_batch_run (swe_batch_set_mode).  Default: ROUNDS
 * captured as one hipGraph per run (the faster mode on MI355X). */
#define SWE_BATCH_PERSISTENT 0 /* one persistent kernel, tile tickets, per-scenario barriers */
#define SWE_BATCH_ROUNDS 1     /* one launch per stage covering every active scenario */
int swe_batch_set_mode(swe_batch *bt, int32_t mode, int32_t use_graph);
/* Tile variant used by the batch's launches (-1: automatic: the 128 x 16
 * tile once the batch's tiles fill the GPU, 256 such tiles or more, else
 * the choice for the scenario with most cells).  All variants give bitwise
 * identical states. */
int swe_batch_set_tile(swe_batch *bt, int32_t tile);
/* Batch options, 0 or 1, for every scenario of the batch from the next
 * swe_batch_run on: SWE_OPT_FRICTION_IMPLICIT (Methods, the friction variant
 * described at that key), SWE_OPT_LOCAL_SPLIT (Methods, the splitting
 * variant described at that key) and SWE_OPT_COMPENSATED (residual planes, 12 bytes
 * per cell, for every scenario present and added later; switching it on
 * starts the residuals at zero, off releases them).  A scenario then
 * advances bitwise as a context with the same options.  Other keys or values
 * are SWE_EINVAL; SWE_ENOMEM if residual planes cannot be allocated (the
 * option is then off for every scenario). */
int swe_batch_set_option(swe_batch *bt, int32_t key, int64_t value);
/* Maximum-depth map of scenario `index`, as swe_track_max_depth for a
 * single scenario: with enable != 0 keep per cell the maximum of h over its
 * state at the call and after every later step of this batch (the map is
 * updated inside the batch's own stage launches); enable = 0 drops it.
 * SWE_ENOTFOUND for a bad index, SWE_ENOMEM if the plane cannot be
 * allocated.  swe_batch_read_max_depth waits for the batch's stream and
 * copies the map ([ny][nx]); SWE_EINVAL if it is not being kept. */
int swe_batch_track_max_depth(swe_batch *bt, int32_t index, int32_t enable);
int swe_batch_read_max_depth(swe_batch *bt, int32_t index, float *hmax);
void swe_batch_destroy(swe_batch *bt);

/* ---- serving: continuous batching of scenario requests ------------------ */
typedef struct swe_server swe_server;

#define SWE_PENDING 0
#define SWE_DONE 1
#define SWE_FAILED 2
#define SWE_CANCELLED 3

typedef struct swe_result {
    int32_t status;   /* SWE_PENDING, SWE_DONE, SWE_FAILED or SWE_CANCELLED */
    int32_t error;    /* SWE_OK or the error that failed the request */
    double t;         /* simulated time at completion */
    double mass;
    float runup;
    int64_t steps;
    double t_submit;  /* host monotonic seconds: submit, admission, result ready */
    double t_admit;
    double t_done;
} swe_result;

typedef struct swe_server_stats {
    int64_t submitted, completed, failed, cancelled;
    int64_t queued;  /* waiting for admission */
    int64_t active;  /* admitted: resident, or being uploaded to join the next segment */
    size_t mem_in_use, mem_high_water, mem_budget;
    int64_t segments;  /* segments run so far */
} swe_server_stats;

/* Start a server on `device` with a device-memory budget for scenario state
 * (bytes; 0 = half of the device's free memory), at most max_slots resident
 * scenarios, and segment_steps steps per segment (one batched run of every
 * resident request) between admissions.  The server runs segments, uploads
 * and read-backs on three streams of its own; a process that also uses other
 * streams should allow HIP enough hardware queues (GPU_MAX_HW_QUEUES, 8 or
 * more) to keep them on separate queues, or uploads wait behind segments. */
int swe_server_create(int32_t device, size_t mem_budget, int32_t max_slots,
                      int32_t segment_steps, swe_server **out);

/* Queue a request; inputs are copied before return.  Returns SWE_EINVAL for
 * bad input, SWE_ENOMEM if it can never fit the budget, SWE_EBUSY if the
 * queue is full. */
int swe_submit(swe_server *sv, const swe_params *p, const float *b, const float *manning_n,
               const float *h0, const float *hu0, const float *hv0, int32_t nsteps,
               uint64_t *ticket);

/* Non-blocking.  Fills r; when r->status is DONE the state is copied into
 * the non-NULL h, hu, hv (host memory).  A ticket is released after a final
 * status (DONE, FAILED, CANCELLED) has been returned once; afterwards it is
 * SWE_ENOTFOUND. */
int swe_poll(swe_server *sv, uint64_t ticket, swe_result *r, float *h, float *hu, float *hv);

/* Flags of swe_submit_ex. */
#define SWE_SUBMIT_MAX_DEPTH 1 /* keep the request's maximum-depth (inundation) map */

/* swe_submit with flags.  SWE_SUBMIT_MAX_DEPTH keeps, on the device, the
 * per-cell maximum of the depth over the starting state and the state after
 * every step (as swe_track_max_depth does for one scenario; Section 3 output
 * of the paper's runs), adding one plane (4 bytes per cell) to the request's
 * footprint.  Unknown flags: SWE_EINVAL. */
int swe_submit_ex(swe_server *sv, const swe_params *p, const float *b, const float *manning_n,
                  const float *h0, const float *hu0, const float *hv0, int32_t nsteps, int32_t flags,
                  uint64_t *ticket);

/* swe_poll that also copies the maximum-depth map ([ny][nx], host memory)
 * into hmax when the request is DONE.  hmax may be NULL; a non-NULL hmax for
 * a request submitted without SWE_SUBMIT_MAX_DEPTH returns SWE_EINVAL and
 * leaves the ticket unchanged. */
int swe_poll_ex(swe_server *sv, uint64_t ticket, swe_result *r, float *h, float *hu, float *hv,
                float *hmax);

/* Launch mode of the server's segments (SWE_BATCH_ROUNDS, the default, or
 * SWE_BATCH_PERSISTENT); takes effect at the next segment. */
int swe_server_set_mode(swe_server *sv, int32_t mode);
/* Server options, 0 or 1, for every request: SWE_OPT_FRICTION_IMPLICIT,
 * SWE_OPT_LOCAL_SPLIT and SWE_OPT_COMPENSATED (each request's footprint then includes its three
 * residual planes); settable before the first submit only (SWE_EBUSY after
 * it), so that all requests share one treatment.  Other keys or values are
 * SWE_EINVAL. */
int swe_server_set_option(swe_server *sv, int32_t key, int64_t value);

/* Cancel a queued or running request (it ends as SWE_CANCELLED). */
int swe_cancel(swe_server *sv, uint64_t ticket);

int swe_server_get_stats(swe_server *sv, swe_server_stats *st);

/* Stop the server thread and free its memory.  NULL-safe. */
void swe_server_destroy(swe_server *sv);

/* ---- misc ----------------------------------------------------------------- */
const char *swe_strerror(int code);

/* Bytes of device memory one nx-by-ny scenario occupies. */
size_t swe_footprint(int32_t nx, int32_t ny);

/* Caller allocator for the library's device memory, so that a framework's
 * caching allocator (torch's, for one) owns and accounts for it (plumbing,
 * not an operation of the method).  It covers every device allocation:
 * contexts (state, outputs, maximum-depth map, compensated planes), batches
 * (scenarios, schedule tables) and servers (arena, schedule tables).  Pinned
 * host memory for snapshots is not routed.
 *   alloc(bytes, device, user) returns device memory of at least `bytes` on
 *     HIP device `device`, aligned to 256 bytes, or NULL (the library call
 *     then fails with SWE_ENOMEM; misaligned memory is handed back and the
 *     call fails with SWE_EINVAL).
 *   release(ptr, device, user) takes back what alloc returned.  The library
 *     waits for the device to finish all work before it calls release, so
 *     the allocator may reuse the memory at once.
 * Both NULL restores hipMalloc/hipFree (the default); exactly one NULL is
 * SWE_EINVAL.  Process-wide and thread-safe; it applies to allocations made
 * after the call, and each allocation is released through the allocator that
 * made it, even after another one is set, so the callbacks and `user` must
 * stay valid until that memory is freed.  The callbacks run on the thread
 * that called into the library, or on a server's own thread (its schedule
 * tables), and must not call back into it. */
typedef void *(*swe_alloc_fn)(size_t bytes, int32_t device, void *user);
typedef void (*swe_release_fn)(void *ptr, int32_t device, void *user);
int swe_set_allocator(swe_alloc_fn alloc, swe_release_fn release, void *user);

#ifdef __cplusplus
}
#endif
#endif /* SWE_H */
