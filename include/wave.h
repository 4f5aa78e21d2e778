/*
 * wave.h -- C ABI of libwave.so, an MI355X (gfx950) propagator for the 3-D
 * constant-density acoustic wave equation.
 *
 * What one step computes (paper, Section III: Eq. 1, Eq. 2 and the 25-point
 * Laplacian; Algorithm 1 for the time loop; Section IV-C for counting the
 * centre once; Section IV-D for the source), in single precision:
 *
 *   lap(u)   = sum_{a in x,y,z} (1/h_a^2) [ c0 u + sum_{m=1..4} c_m (u(+m e_a) + u(-m e_a)) ]
 *              with the 8th-order weights c = (-205/72, 8/5, -1/5, 8/315, -1/560);
 *   u^{n+1}  = G (2 u^n - G u^{n-1} + k lap(u^n)),  k = V^2 dt^2 per cell,
 *              G = gx(x) gy(y) gz(z) a Cerjan sponge (G = 1 with no sponge,
 *              where this is Eq. 2 exactly);
 *   u^{n+1}[src] += s_n                (value supplied by the caller);
 *   trace[n][r]   = u^{n+1}[rec_r]     (after the source is added).
 *
 * The paper gives no programming interface; this one is designed for a GPU
 * that owns the fields.  Conventions for every call:
 *   - return value: WAVE_OK (0) or a negative WAVE_E* code; nothing throws;
 *     wave_strerror() names a code, wave_last_error() gives the message of
 *     the last failure on a context;
 *   - "device pointer" = memory allocated on the context's GPU by the caller
 *     (hipMalloc, a torch tensor); the library never frees caller memory;
 *   - host arrays are only read during the call;
 *   - a context is not thread-safe; distinct contexts are independent;
 *   - work is enqueued on the context's stream and returns before it runs;
 *     wave_sync() waits for it and reports asynchronous GPU errors.
 *
 * Field layout (every wave field and k share it; see wave_layout):
 *   planes [nz+8] x rows [ny+8] x pitch_x elements, x fastest.  A ghost layer
 *   of 4 cells surrounds the interior on every face (paper Section IV-B
 *   extends each column by 4 cells on both sides; here the same is done on
 *   all three axes).  Interior point (z, y, x), 0 <= x < nx etc., is element
 *       ((z + 4) * (ny + 8) + (y + 4)) * pitch_x + x_offset + x.
 *   Ghost cells must be zero in u fields (zero Dirichlet boundary) and stay
 *   so: the library writes nothing but zero into them (when nx is not a
 *   multiple of 4, a row's last 4-cell group, which ends in right-ghost
 *   cells, is stored whole).  The tiled step kernels take ghost rows,
 *   columns and planes as zero without reading them; they read only the
 *   right-ghost cells inside a row's last 4-cell group, which must hold zero
 *   (the naive cross-check kernel reads every ghost cell it reaches).
 *   x_offset makes every interior row start on a 128-byte boundary.
 */
#ifndef WAVE_H
#define WAVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define WAVE_OK 0
#define WAVE_EINVAL (-1)    /* bad argument; nothing was enqueued */
#define WAVE_EUNSTABLE (-2) /* k too large for the leapfrog stability limit */
#define WAVE_ESTATE (-3)    /* call not valid in the context's current state */
#define WAVE_ENOMEM (-4)    /* host or device allocation failed */
#define WAVE_EHIP (-5)      /* a HIP runtime call or a kernel failed */

/* storage types: FP32, or 16-bit with FP32 arithmetic.  A 16-bit field
 * holds x * 2^-e with one exponent e per time level, chosen on the device
 * each step from the previous maxima so that |x| * 2^-e < 2^14; k is kept
 * by the library in the same format with a fixed exponent.
 *   WAVE_F16, WAVE_BF16        the two time levels u^n, u^{n-1} (8 bytes
 *                              of traffic per cell and step);
 *   WAVE_F16_UV, WAVE_BF16_UV  u^n and the step change d^n = u^n - u^{n-1}
 *                              (10 bytes per cell and step).  d is stored
 *                              to its own relative precision instead of as
 *                              the difference of two rounded levels, which
 *                              at small Courant numbers is several times
 *                              (FP16) to ten times (BF16) more accurate.  The
 *                              library keeps d in a buffer of its own. */
#define WAVE_F32 0
#define WAVE_F16 1
#define WAVE_BF16 2
#define WAVE_F16_UV 3
#define WAVE_BF16_UV 4

typedef struct wave_layout_t {
    int64_t pitch_x;  /* elements per row (a multiple of 128 bytes) */
    int64_t rows;     /* rows per plane = ny + 8 */
    int64_t planes;   /* planes = nz + 8 */
    int64_t x_offset; /* element offset of interior x = 0 within a row */
    int64_t plane;    /* elements per plane = pitch_x * rows */
    int64_t elems;    /* elements per field = plane * planes */
    int64_t bytes;    /* bytes per field */
} wave_layout_t;

typedef struct wave_params_t {
    int32_t nx, ny, nz;   /* interior size, each >= 1 */
    double dx, dy, dz;    /* grid spacing (> 0), same unit as V dt */
    int32_t sponge_width; /* W >= 0 cells on every face; 0 = no sponge */
    double sponge_alpha;  /* g(d) = exp(-(alpha (W - d))^2) for distance d < W */
    int32_t dtype;        /* WAVE_F32, WAVE_F16, WAVE_BF16, WAVE_F16_UV or WAVE_BF16_UV */
} wave_params_t;

typedef struct wave_ctx wave_ctx;

/* Host arithmetic only: layout of a field of interior size nx x ny x nz.
 * Returns WAVE_EINVAL for sizes < 1, an unknown dtype, a NULL out, or a
 * plane of 2^31 elements or more. */
int wave_layout(int32_t nx, int32_t ny, int32_t nz, int32_t dtype, wave_layout_t *out);

/*
 * Create a context on the current device.
 *   p         grid, spacing, sponge and storage type;
 *   k         device, V^2 dt^2 per cell as FP32 in the FP32 layout (interior
 *             read, ghosts ignored).  With FP32 storage the library reads it
 *             every step (keep it alive); with 16-bit storage it is read
 *             once here and encoded into a library-owned 16-bit copy;
 *   u_cur     device, [layout of dtype] u^n   (ghost cells zero; all zero
 *             for 16-bit storage, whose first exponent is 0);
 *   u_prev    device, [layout of dtype] u^{n-1} (ghost cells zero); it is
 *             overwritten by u^{n+1} in the first step (two time levels,
 *             paper Section IV-B);
 *   src_zyx   host, 3 interior indices of the point source, or NULL for none;
 *   rec_zyx   host, [nrec][3] interior indices of the receivers (may repeat);
 *   nrec      >= 0;
 *   stream    hipStream_t for all work of this context (NULL = default stream).
 * Validates all arguments before touching the device (WAVE_EINVAL), builds
 * the sponge profiles and receiver tables on the device, then reads k once
 * and returns WAVE_EUNSTABLE if max(k) * (2048/315) * sum_a 1/h_a^2 > 4 or
 * WAVE_EINVAL if k holds a negative or non-finite value (this read
 * synchronises the stream).  The step counter starts at 0.  *out is owned
 * by the library until wave_destroy.
 */
int wave_init(wave_ctx **out, const wave_params_t *p, const void *k, void *u_cur,
              void *u_prev, const int32_t *src_zyx, const int32_t *rec_zyx, int32_t nrec,
              void *stream);

/* Attach a device trace buffer [nt_capacity][nrec] (FP32): the step with
 * counter n writes row n.  NULL detaches.  Steps whose row would reach
 * nt_capacity are rejected with WAVE_EINVAL before anything is enqueued. */
int wave_record(wave_ctx *ctx, float *traces_dev, int32_t nt_capacity);

/* Enqueue one step with source value src_value; the counter advances by 1
 * and the two field buffers swap roles. */
int wave_step(wave_ctx *ctx, float src_value);

/* Enqueue nsteps >= 0 steps; step j (0-based within this call) adds
 * src_dev[j] (device FP32 array of >= nsteps values), or nothing if
 * src_dev is NULL. */
int wave_run(wave_ctx *ctx, int32_t nsteps, const float *src_dev);

/* Graph replay of wave_run (on != 0): a run's launches are captured once as
 * a HIP graph and replayed by later runs that start from the same state --
 * same step counter, buffer roles, source array, trace buffer and nsteps,
 * e.g. the same shot again after wave_reset; any other run is captured
 * anew (the last capture is kept).  Meant for small grids, where a
 * launch costs more than the step it runs (the time loop of Algorithm 1 is
 * one launch per step).  Needs a stream other than the legacy default
 * stream (WAVE_EINVAL).  Results are bit for bit those of eager launches. */
int wave_set_graph(wave_ctx *ctx, int32_t on);

/* Current roles: *cur holds u^n and *prev u^{n-1}, with n = *step.  Any
 * output pointer may be NULL. */
int wave_fields(const wave_ctx *ctx, void **cur, void **prev, int64_t *step);

/* Decode u^n (which = 0) or u^{n-1} (which = 1, the level stored by the
 * step before; u-and-change storage keeps it too, though its steps read
 * d^n instead) into dst, an FP32 field in
 * the FP32 layout (interior written, ghosts untouched); enqueued on the
 * context's stream.  With FP32 storage this is a copy. */
int wave_export(wave_ctx *ctx, int32_t which, float *dst);

/* Reset the counter to 0 and the roles to those given at init, and clear
 * the 16-bit scale history and (u-and-change storage) the library's d
 * field; the caller re-initialises the contents of its own fields. */
int wave_reset(wave_ctx *ctx);

/* Replace the stream used by later calls. */
int wave_set_stream(wave_ctx *ctx, void *stream);

/*
 * Kernel selection (tuning and cross-checks).  variant 0 = automatic;
 * 1 .. wave_variant_count()-1 name compiled kernels (wave_variant_name);
 * zchunk = planes per work-group along z (0 = automatic).  Takes effect
 * from the next step; rebuilds the receiver tables.
 */
int wave_configure(wave_ctx *ctx, int32_t variant, int32_t zchunk);
int32_t wave_variant_count(void);
const char *wave_variant_name(int32_t variant);
/* Variant and z-chunk in use, and the work-groups one step launches. */
int wave_config(const wave_ctx *ctx, int32_t *variant, int32_t *zchunk, int32_t *workgroups);

/* Watchdog: counts the non-finite values (infinity, NaN) of the current
 * field u^n (interior) and of the trace rows written so far.  Either count
 * pointer may be NULL.  Synchronises the context's stream; a run that went
 * unstable (for instance a k edited after init) shows up here. */
int wave_check(wave_ctx *ctx, int64_t *field_nonfinite, int64_t *trace_nonfinite);

/* wave_check for callers that cannot allocate device memory (a loop that
 * checks the run every few steps, harnesses that forbid hipMalloc): the
 * same counts, with the two counters held in a fixed device array of the
 * library (64 ints, 256-byte aligned, one per GPU, kept until the process
 * ends; its address is looked up by wave_init) instead of a buffer
 * allocated and freed per call.  Allocates nothing; clears the counters
 * with a kernel, then synchronises the context's stream as wave_check
 * does.  Every context on one GPU shares the array: calls that overlap on
 * one GPU (from several host threads or streams) race and may report each
 * other's counts.  WAVE_EHIP if the array's address cannot be obtained or
 * a launch or copy fails. */
int wave_check_noalloc(wave_ctx *ctx, int64_t *field_nonfinite, int64_t *trace_nonfinite);

/* Wait for all work enqueued on the context's stream; WAVE_EHIP if it or
 * any earlier launch failed. */
int wave_sync(wave_ctx *ctx);

/*
 * Gradient with respect to k (FP32 storage only).  The paper gives only the
 * forward time loop (Eq. 2, Algorithm 1); what follows is the exact discrete
 * adjoint of that loop as this library runs it (sponge included, source
 * values held fixed).  For a scalar J of the traces of nt steps, with
 * g_n = dJ/d trace[n] (one row per step), it returns
 *
 *   dJ/dk = sum_{m=1..nt} lambda^m G lap(a^{m-1}),
 *   lambda^m = R^T g_{m-1} + 2 G lambda^{m+1} + lap(k G lambda^{m+1}) - G^2 lambda^{m+2},
 *
 * (lambda^{nt+1} = lambda^{nt+2} = 0, a^m the forward field after step m,
 * a^0 and a^{-1} the fields the run started from, R^T adding each
 * receiver's value at its cell).  On the device the adjoint field is kept
 * as phi = k lambda, so that the adjoint step is the forward stencil update
 * applied to G phi; every forward level a^{m-1} is recomputed segment by
 * segment from checkpoints (a^{c-1}, a^c) taken every C steps, and the sum
 * is accumulated in FP64.  wave_adjoint_velocity returns dJ/dv = 2 v dt^2
 * dJ/dk instead.
 */

/* Run nt forward steps from the current state, exactly as wave_run (same
 * traces, fields and step counter afterwards), and keep what the adjoint
 * run needs: checkpoints every `every` steps (0: the library picks the
 * largest segment that fits in half of the free device memory -- all levels
 * of the run when they fit, so that nothing is recomputed) and the levels
 * of the last segment.  src_dev: nt FP32 device values (copied; NULL = no
 * source).  Library-owned device memory: (2 ceil(nt / C) + C) field levels
 * of wave_layout bytes each, kept until the next call or wave_destroy.
 * WAVE_ENOMEM when it cannot be allocated, WAVE_EINVAL for 16-bit storage. */
int wave_forward_checkpointed(wave_ctx *ctx, int32_t nt, const float *src_dev, int32_t every);

/* Adjoint run of the last wave_forward_checkpointed run.
 *   trace_grad_dev  FP32 device array [nt][nrec]: dJ/d trace (row n belongs
 *                   to step n of that run; may be NULL without receivers);
 *   grad_dev        FP64 device array [nz][ny][nx] (dense, x fastest):
 *                   receives dJ/dk, or has it added when accumulate != 0.
 * Receivers sharing a cell contribute the sum of their derivatives.  May be
 * called again for another trace_grad of the same run (levels are then
 * recomputed).  Library-owned device memory: two FP32 fields and one FP64
 * field of the layout, kept until wave_destroy.  The context's fields,
 * traces and step counter are left as the forward run left them. */
int wave_adjoint(wave_ctx *ctx, const float *trace_grad_dev, double *grad_dev, int32_t accumulate);

/* The same adjoint run with the result taken to velocity, for a context
 * whose k was made from a velocity model v as k = (v dt)^2 (see
 * wave_velocity_to_k): dJ/dv = 2 dt^2 v dJ/dk.
 *   v_dev                 FP32 device array [nz][ny][nx] (dense, x
 *                         fastest): the velocity that gave the context's k;
 *   dt                    the time step of k = (v dt)^2 (> 0);
 *   source_scales_with_k  0: the injected source values are held fixed, as
 *                         in wave_adjoint.  Non-zero: they were k at the
 *                         source cell times fixed values (Eq. 2 scales the
 *                         source term by dt^2 V^2 at the source cell), and
 *                         dJ/dk there gains sum_m lambda^m s_{m-1} / k_src,
 *                         the derivative through the source values;
 *   grad_v_dev            FP64 device array [nz][ny][nx]: receives dJ/dv,
 *                         or has it added when accumulate != 0.
 * trace_grad_dev, memory, state and errors as for wave_adjoint;
 * WAVE_EINVAL also for a NULL v_dev or dt <= 0. */
int wave_adjoint_velocity(wave_ctx *ctx, const float *trace_grad_dev, const float *v_dev, double dt,
                          int32_t source_scales_with_k, double *grad_v_dev, int32_t accumulate);

/* Eq. 2's per-cell coefficient k = V^2 dt^2 from a velocity model: each of
 * the n FP32 values of v_dev (device) is multiplied by dt and squared in
 * FP64, and the result rounded once to FP32 into k_dev (device, n values,
 * same indexing; the two arrays must not overlap).  Enqueued on `stream`.
 * WAVE_EINVAL for a NULL pointer, n < 0 or dt <= 0; WAVE_EHIP if the launch
 * fails. */
int wave_velocity_to_k(const float *v_dev, int64_t n, double dt, float *k_dev, void *stream);

/* The adjoint run normally makes phi^{m-1} and adds the imaging term of
 * phi^m in one pass over the grid (36 instead of 44 bytes per cell and
 * step); on = 0 selects two separate passes.  Both give the same result
 * bit for bit; the switch exists for that cross-check. */
int wave_set_adjoint_fusion(wave_ctx *ctx, int32_t on);

/* Steps, segment length, segments and bytes of checkpoint/level storage of
 * the last checkpointed forward run (nt = 0 when there is none). */
int wave_grad_info(const wave_ctx *ctx, int32_t *nt, int32_t *every, int32_t *segments, int64_t *bytes);

/* Least-squares misfit of n trace values: *misfit_dev = 0.5 sum (t - d)^2,
 * summed in FP64 in a fixed order (deterministic); residual_dev (FP32, may
 * be NULL) receives t - d, which is dJ/d trace for this J.  All pointers
 * are device memory; enqueued on `stream`. */
int wave_misfit(const float *traces_dev, const float *observed_dev, int64_t n, float *residual_dev,
                double *misfit_dev, void *stream);

/*
 * Batched runs: many shots (contexts) advanced together, one launch per
 * time step for every group of shots that share a kernel variant and
 * storage type (a work-group finds its shot through a per-launch table).
 * Shots may differ in size, model, source, receivers and tile choice.
 *   ctxs       nshots distinct contexts, configured (wave_configure) before
 *              the batch is created and not reconfigured afterwards; the
 *              naive kernel and u-and-change storage are not batched;
 *   stream     the stream of every batched run (the contexts' own streams
 *              are not used by it); required when use_graph != 0, and then
 *              it must not be the legacy default stream;
 *   use_graph  capture a run's launches once as a HIP graph (schedule 1:
 *              one graph per stream) and replay it for later runs of the
 *              same length.
 * The batch holds pointers to the contexts: destroy it before them.
 */
typedef struct wave_batch wave_batch;
int wave_batch_create(wave_batch **out, wave_ctx *const *ctxs, int32_t nshots, void *stream,
                      int32_t use_graph);

/* Enqueue nsteps steps of every shot.  All contexts must be at the same
 * step counter (WAVE_ESTATE otherwise).  src_dev: host array of nshots
 * device pointers (FP32, >= nsteps values each; a NULL entry injects
 * nothing for that shot), or NULL for no source at all.  Traces, step
 * counters and buffer roles of every context advance exactly as if each
 * had called wave_run.  When the run's descriptors differ from the last
 * run's (another starting step, other buffers or sources), the call first
 * waits for the batch stream, then uploads them. */
int wave_batch_run(wave_batch *b, int32_t nsteps, const float *const *src_dev);

/* How a batched run is launched.
 *   schedule 0  one persistent launch per step for every group of shots
 *               sharing a kernel (work items taken by ticket), the default;
 *   schedule 1  every shot's steps launched with its own kernel
 *               configuration, the shots dealt, largest first, to the least
 *               loaded (in cells) of nstreams (1..16) streams of the library
 *               that fork from and join back to the batch stream; with
 *               use_graph each stream's share of the run is captured as a
 *               graph of its own, replayed on that stream (so the streams
 *               run concurrently) while the shots' states, sources, trace
 *               buffers and nsteps repeat.  Shots large enough to
 *               fill the GPU alone run best this way, each with the tiling
 *               that suits its own shape;
 *   schedule 2  SWITCHED OFF (returns WAVE_EINVAL): its first GPU run did not
 *               complete and the cause is not yet known.  Design: FP32
 *               only; one launch for every step of every shot of a
 *               group (shots sharing a tile shape), each shot pinned to one
 *               of the 8 XCDs (largest first to the least loaded) and its
 *               tiles and chunks started as soon as the ones their stencil
 *               reads have finished the step before (per-tile step
 *               counters in place of the launch boundary between steps).
 *               nstreams is ignored;
 *   schedule 3  one cooperative launch per group of shots (shots sharing a
 *               kernel and storage type) for the whole run: every step is
 *               schedule 0's work (items taken by ticket from per-XCD
 *               ranges), and a grid-wide barrier takes the place of the
 *               launch boundary between steps (agent-scope release on
 *               arrival, acquire on departure, so no assumption about which
 *               XCD runs which work-group).  As many work-groups as the GPU
 *               holds at once.  A barrier wait that runs past a wall-clock
 *               limit (2 s plus 0.1 ms per step and 0.1 ns per cell update)
 *               stops the launch and wave_batch_sync returns WAVE_EHIP.  The
 *               launch is made directly, not captured (use_graph has no
 *               effect).  nstreams is ignored.  WAVE_EINVAL if the device
 *               cannot launch cooperative kernels.
 * All give the same results bit for bit as the shots run alone.  Waits for
 * the batch stream; drops a captured graph.  WAVE_EINVAL for another
 * schedule, a stream count out of range, or schedule 1 with graph replay on
 * the legacy default stream, or schedule 2 with shots not stored in FP32;
 * WAVE_EHIP if the library's streams or events cannot be created or the
 * schedule-3 launch shape cannot be determined, and WAVE_ENOMEM if the
 * schedule-2 tables cannot be allocated; the batch is then left on
 * schedule 0. */
int wave_batch_set_schedule(wave_batch *b, int32_t schedule, int32_t nstreams);

/* Schedule 2: how many times one dependency wait polls (about 50 ns apart)
 * before it gives up; the default is 2^24.  Schedule 3 bounds its barrier
 * waits by wall-clock time instead and reads only the sign: a negative value
 * makes every barrier wait give up at once (the same test hook).  A wait only ever waits for work
 * already running, so it ends; the limit is a safety net.  A wait that gives
 * up stops the whole launch, and wave_batch_sync then returns WAVE_EHIP.  A
 * negative value makes every wait after a launch's first step give up (a
 * hook for testing that failure path).  Waits for the batch stream and drops
 * a captured graph. */
int wave_batch_set_wait_limit(wave_batch *b, int32_t polls);

/* Launch groups, work-groups and interior points of one batched step. */
int wave_batch_info(const wave_batch *b, int32_t *groups, int64_t *workgroups_per_step,
                    int64_t *points_per_step);

/* Wait for the batch stream; WAVE_EHIP if a batched launch failed or, with
 * schedule 2 or 3, a dependency or barrier wait gave up. */
int wave_batch_sync(wave_batch *b);

int wave_batch_destroy(wave_batch *b);
const char *wave_batch_last_error(const wave_batch *b);

/* Free library-owned memory (host and device); caller buffers are kept.
 * NULL is accepted. */
int wave_destroy(wave_ctx *ctx);

const char *wave_strerror(int code);
const char *wave_last_error(const wave_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* WAVE_H */
