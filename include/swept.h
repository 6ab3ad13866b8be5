/*
 * swept.h -- C ABI of the MI355X swept-rule stencil library (libswept.so).
 *
 * The library advances 1D periodic explicit stencil PDEs in time on one AMD
 * Instinct MI355X (gfx950).  Two schedules produce the same bits:
 *
 *  - swept_advance: the swept rule (paper, Section 3).  Each workgroup owns a
 *    tile of W = 2k points (the paper's node, which owns an even number of
 *    points).  It first computes the shrinking space-time triangle that its
 *    own points determine, then, in every later stage, the diamond whose
 *    domain of dependence is covered by the V formed by two swept leading
 *    edges.  Only those edges (two points per sub-timestep and side) travel
 *    between workgroups, through HBM, once per stage of k sub-timesteps.
 *  - swept_naive_advance: the straight decomposition (paper, Sections 1 and
 *    4), one kernel launch per time step (or per sub-timestep).
 *
 * The local code -- what one sub-timestep does to one point -- is selected by
 * a stencil id (the paper's Section 5 separates it from the global, swept
 * ordering code; here it is compiled in rather than called back).
 *
 * Conventions for every entry point:
 *  - Return 0 (SWEPT_OK) on success or a negative swept_status.  Nothing
 *    aborts or throws across the ABI; swept_last_error() returns a message
 *    for the last failure of the calling thread.
 *  - Pointers named u are DEVICE pointers to nx contiguous elements of the
 *    stencil's type (double for *_F64, float for *_F32, three interleaved
 *    doubles per cell for SWEPT_EULER_F64), owned by the caller.  They are
 *    updated in place to the state after nsteps full time steps.
 *  - Work is enqueued on the library's current stream (swept_set_stream) and
 *    is asynchronous: the caller keeps u alive until that stream is
 *    synchronised.  Errors raised by kernels that are still running surface
 *    at swept_sync().
 *  - params points to HOST memory and is read during the call only.
 *  - The library owns its scratch (edge buffers of the swept path, a second
 *    field for the naive path, checkpoints of the adjoints, the tables of a
 *    batch).  It grows on demand, synchronising the current stream first,
 *    and is released by swept_finalize().  Work still running on another
 *    stream when the scratch grows is the caller's to finish first.
 *  - The library keeps one context per process (device, stream, tuning,
 *    scratch): calls from several host threads must be serialised by the
 *    caller.  Calls that overlap on the device (two streams) must not share
 *    the library's scratch, so use one stream at a time.
 *  - swept_advance and swept_naive_advance enqueue only kernels (and, on the
 *    naive path, one device copy) once the scratch is large enough, so a
 *    caller may capture them into a HIP graph after one eager call of the
 *    same size and replay the graph; the captured kernels keep the scratch
 *    addresses of that moment, so the graph must not outlive a later call
 *    that grows the scratch, nor swept_finalize().  Capture with stage
 *    profiling off.
 */
#ifndef SWEPT_H
#define SWEPT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SWEPT_OK = 0,
    SWEPT_EINVAL = -1,        /* bad argument: null pointer, nx < 3, nsteps < 0, bad id, bad params */
    SWEPT_ENOTINIT = -2,      /* swept_init was not called (or failed) */
    SWEPT_ENOMEM = -3,        /* device allocation of scratch failed */
    SWEPT_EHIP = -4,          /* a HIP runtime call or kernel launch failed */
    SWEPT_EUNSUPPORTED = -5,  /* valid request the library cannot run (e.g. tiling impossible) */
    SWEPT_ETIMEOUT = -6       /* a bounded device-side wait gave up (persistent batch,
                                 reported by swept_sync) */
} swept_status;

/*
 * Stencil ids.  Each defines one time step as a sequence of radius-1
 * sub-timesteps (paper, Section 2) and the parameters it reads:
 *
 * SWEPT_HEAT_F64 / SWEPT_HEAT_F32: heat equation u_t = u_xx by the 3-point
 *   forward-Euler finite difference, one sub-timestep per step (the paper's
 *   Section 4 "3 FLOPs" scheme):  u' = u + r*((u[i-1] + u[i+1]) - 2*u[i]),
 *   evaluated in that association in binary64 / binary32 without fused
 *   multiply-add.  params = { r } (nparams >= 1); for F32, r is rounded to
 *   float once.
 *
 * SWEPT_KS_F64: Kuramoto-Sivashinsky u_t = -u u_x - u_xx - u_xxxx by central
 *   differences and the RK2 midpoint rule (paper, Section 6; RK2 as
 *   sub-timesteps, Section 2), four sub-timesteps per step:
 *     w = D2(u);  v = u + h*F(u,w);  z = D2(v);  u' = u + dt*F(v,z)
 *   with D2(a) = ((a[i-1]+a[i+1]) - 2a[i])*c2, D1(a) = (a[i+1]-a[i-1])*c1,
 *   F(a,b) = -(((a*D1(a)) + b) + D2(b)), c1 = 1/(2dx), c2 = 1/(dx*dx),
 *   h = dt/2, all in binary64.  params = { dt, dx } (nparams >= 2, dx > 0).
 *
 * SWEPT_EULER_F64: the 1D Euler equations of gas dynamics by second-order
 *   finite volumes (paper, Section 7: minmod limiter, interface flux with
 *   scalar dissipation proportional to the spectral radius of the Roe
 *   matrix, midpoint Runge-Kutta; Section 2: a slope sub-timestep and a
 *   flux-difference sub-timestep per Runge-Kutta stage), four sub-timesteps
 *   per step:  s = slope(q);  r = q - ch*dF(q,s);  s = slope(r);
 *   q' = q - cf*dF(r,s),  ch = (dt/2)/dx, cf = dt/dx.  slope is the minmod of
 *   the one-sided differences; dF the difference of the two face fluxes
 *   F = (f(qL) + f(qR))/2 - (|u| + c)/2 (qR - qL), u and c at the Roe average
 *   of the states qL = v[i] + s[i]/2, qR = v[i+1] - s[i+1]/2.  A cell is
 *   three binary64 values (rho, rho*u, E), interleaved: u points to 3*nx
 *   doubles.  params = { dt, dx, gamma } (nparams >= 3, dx > 0, gamma > 1).
 *   Not available in swept_advance_batch or swept_adjoint.
 *
 * SWEPT_HEAT_F64_FMA / SWEPT_HEAT_F32_FMA / SWEPT_KS_F64_FMA: the same
 *   schemes and parameters with their multiply-adds fused (the contraction-on
 *   build of the schemes; the paper's Section 4 counts the heat sub-timestep
 *   as 3 FLOPs, which is this form):
 *     heat  u' = fma(r, fma(-2, u, u[i-1] + u[i+1]), u)
 *     KS    D2(a) = fma(-2, a, a[i-1] + a[i+1]) * c2,
 *           F(a,b) = -(fma(a, D1(a), b) + D2(b)),
 *           v = fma(h, F(u,w), u),  u' = fma(dt, F(v,z), u)
 *   A fused multiply-add rounds once where the canonical form rounds twice,
 *   so these results agree with the canonical ones to within rounding, not
 *   bit for bit.
 *   swept_advance and swept_naive_advance give the same bits as each other
 *   for these ids.  Not available in swept_advance_batch, swept_adjoint or
 *   swept_naive_substep_advance.
 */
enum {
    SWEPT_HEAT_F64 = 0,
    SWEPT_HEAT_F32 = 1,
    SWEPT_KS_F64 = 2,
    SWEPT_EULER_F64 = 3,
    SWEPT_HEAT_F64_FMA = 4,
    SWEPT_HEAT_F32_FMA = 5,
    SWEPT_KS_F64_FMA = 6
};

/* Schedules for swept_set_tuning. */
enum {
    SWEPT_MODE_AUTO = 0,      /* swept stages when the grid can be tiled, else naive */
    SWEPT_MODE_STAGE = 1,     /* swept: one kernel launch per stage (triangle, diamonds) */
    SWEPT_MODE_NAIVE = 2,     /* one launch per time step */
    SWEPT_MODE_STAGE_BANDED = 3, /* swept stages, every diamond on the banded kernel
                                    (the continuous-band kernel switched off) */
    SWEPT_MODE_STAGE_LANE = 4,   /* swept stages on the lane-frame kernel (one lane per
                                    column, W <= 64): for few, latency-bound tiles */
    SWEPT_MODE_STAGE_RAGGED = 5  /* swept stages on unequal tiles: T-1 tiles of 2k points
                                    and one of the remainder (odd nx on its two-fold
                                    cover); k = tile_w/2, or the target depth if 0 */
};

/*
 * Select the device and reset the stream to the null stream.  Must precede
 * every other call except swept_last_error.  Calling it again with another
 * device releases the scratch of the previous one.
 */
int swept_init(int device);

/* Enqueue all later work on this hipStream_t (NULL = the null stream). */
int swept_set_stream(void *hip_stream);

/*
 * Tuning of the swept path.  tile_w: points per tile W (even, W divides nx);
 * 0 = automatic.  pairs_per_lane: 1, 2, 4 or 8 (0 = automatic; the KS
 * stencil takes at most 4, and swept_advance fails with SWEPT_EUNSUPPORTED
 * for 8); each lane of a tile's wavefront carries that many adjacent point
 * pairs.  mode: one of
 * SWEPT_MODE_*.  The values persist until changed.  Results do not depend on
 * the tuning, bit for bit.
 */
int swept_set_tuning(int32_t tile_w, int32_t pairs_per_lane, int32_t mode);

/*
 * How swept_advance, swept_advance_noalloc and swept_advance_batch evaluate
 * SWEPT_HEAT_F64 and SWEPT_HEAT_F32 (the heat sub-timestep of the paper's
 * Section 4).  Both forms give the canonical bits defined above.
 *  - SWEPT_FORM_AUTO (the default): the stage kernels compute
 *    (u[i-1] + u[i+1]) - 2*u[i] as one fused multiply-add,
 *    fma(-2, u[i], u[i-1] + u[i+1]), in the field's precision.  2*u[i] is
 *    exact whenever it is finite, so the subtraction rounds the same exact
 *    difference once, as the fused multiply-add does: four operations per
 *    point instead of five.  The kernels take this form when 0 <= r <= 1/2
 *    (r as rounded to the field's type), the run is at most 1e15 steps
 *    (binary64) or 1e6 steps (binary32), and a check of the initial field on
 *    the device (one extra read of u, enqueued with the stages) finds no
 *    finite |u| above a sixteenth of the type's largest finite value (MAX).
 *    For such r each update is a convex combination of its three inputs, so
 *    no point comes near MAX/2, the only place where the two forms differ
 *    (2*u overflows, the fused form does not); a non-finite value only
 *    produces non-finite values, alike in both forms.  Otherwise the
 *    kernels evaluate the five operations as written.  A batch takes one
 *    decision for all its heat instances: every one must meet the
 *    conditions (its r, its step count, its field), else all of them run
 *    the five operations; each launch of a batch checks its fields again.
 *  - SWEPT_FORM_CANONICAL: always the five operations as written.
 * The setting persists until changed.  Other stencil ids, swept_naive_advance
 * and the adjoints always evaluate their schemes as written.
 */
enum {
    SWEPT_FORM_AUTO = 0,
    SWEPT_FORM_CANONICAL = 1,
    SWEPT_FORM_FUSED = 2
};
int swept_set_heat_form(int32_t form);

/*
 * The form the last swept_advance or swept_advance_noalloc call with
 * SWEPT_HEAT_F64 or SWEPT_HEAT_F32, or the last swept_advance_batch call with
 * a heat instance, evaluated (SWEPT_FORM_FUSED or SWEPT_FORM_CANONICAL; the
 * naive schedule counts as canonical), or 0 before any such call.  It
 * synchronises the library's stream to read the device-side check.
 */
int swept_last_heat_form(int32_t *form);

/*
 * Plan the swept run swept_advance would use for these arguments, without
 * running it.  out[0..5] = { tile_w, depth_k, tiles, stages, pairs_per_lane
 * (0 on the lane-frame kernel), mode_used }.  For SWEPT_MODE_STAGE_RAGGED
 * tile_w = 2k is the width of the full tiles and tiles counts the tiles of
 * the ring (the two-fold cover for odd nx).  Returns SWEPT_EINVAL for
 * invalid arguments.
 */
int swept_plan(int64_t nx, int64_t nsteps, int32_t stencil_id, int64_t *out);

/*
 * Advance u (device, nx points of the stencil's type, periodic) by nsteps
 * time steps with the swept rule.  nsteps == 0 is a no-op.  The automatic
 * plan tiles every grid: with equal tiles of the largest even width W that
 * divides nx, up to min(1024, nx/16) points, when W is at least half that
 * target; otherwise (odd nx, or an even nx without such a divisor) with
 * SWEPT_MODE_STAGE_RAGGED's unequal tiles at the target depth, odd nx on its
 * two-fold cover.  Grids whose target depth is below 4 points (nx < 128)
 * without a good equal tiling use the naive schedule.  Every plan gives the
 * same bits.
 */
int swept_advance(void *u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                  const double *params, int32_t nparams);

/*
 * For callers that cannot allocate device memory -- code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc: the same
 * as swept_advance (same arguments, plan, kernels and bits), with the scratch
 * in a fixed array of SWEPT_NOALLOC_SCRATCH_BYTES that the library holds on
 * each GPU it runs on (from swept_init until the process ends) instead of
 * memory it allocates.  The call allocates nothing.  It needs
 * 3 * nx * (point size) bytes on the swept path with equal tiles (point
 * size: 8 for heat f64, 4 for heat f32, 24 for KS, 72 for Euler; heat f64 up
 * to 5,592,405 points, KS up to 1,864,135), 6 * nx * (point size) + 2 * nx
 * field elements on the unequal tiling of an odd nx, and nx field elements
 * on the naive path; larger requests fail with SWEPT_EINVAL before any work
 * is enqueued.  Every call on a GPU shares that GPU's array, which keeps the
 * last call's contents: calls that overlap on one GPU (two streams, or two
 * threads) race and must be serialised by the caller.  Stage profiling is
 * ignored during the call.
 */
#define SWEPT_NOALLOC_SCRATCH_BYTES (128u << 20)
int swept_advance_noalloc(void *u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                          const double *params, int32_t nparams);

/*
 * Advance u by nsteps time steps with one kernel launch per time step
 * (KS: the four sub-timesteps of a step fused in one launch, the halo of
 * each block recomputed).  Same arguments and results as swept_advance.
 */
int swept_naive_advance(void *u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                        const double *params, int32_t nparams);

/*
 * KS only: one kernel launch per sub-timestep (four per step), the paper's
 * straight decomposition that communicates every sub-timestep.  Same
 * results as swept_naive_advance.
 */
int swept_naive_substep_advance(void *u, int64_t nx, int64_t nsteps, int32_t stencil_id,
                                const double *params, int32_t nparams);

/*
 * Advance count independent instances at once (binary64 stencils only:
 * SWEPT_HEAT_F64, SWEPT_KS_F64).  u[j] (a HOST array of DEVICE pointers) is
 * instance j's field of nx[j] points, advanced in place by nsteps[j] steps of
 * stencil_id[j] with parameters params[2j], params[2j+1] (heat reads the
 * first).  Every instance gets exactly the bits its own swept_advance would.
 *
 * Each instance of 2h points (h = nx/2 for even nx) is tiled by T = ceil(h/k)
 * tiles: T-1 of width 2k and one of the remainder 2(h - (T-1)k) (k =
 * tile_w/2 of swept_set_tuning if set, else the depth swept_autotune_batch
 * chose for the stencil, else 256), so any even length tiles without
 * remainder.  The regions between two full tiles are k x k squares (those
 * below the target level run on the continuous-band schedule); the regions
 * next to the short tile are rectangles of k_t pairs by k_{t+s} steps.  An
 * odd length runs on its two-fold cover
 * (the field repeated twice, which the scheme keeps repeated).
 *
 * Schedule (swept_set_batch_schedule).  SWEPT_BATCH_PERSISTENT, the default:
 * one persistent kernel launch per stencil runs every region of every stage
 * of every instance.  Its workgroups (as many as the GPU holds at once)
 * take regions from device counters, in stage-major order with the
 * instances with the most stages first, and a region waits only for the two
 * regions of the previous stage it reads (its own tile's and the next
 * tile's) -- the paper's point-to-point communication stage, in which a
 * node needs only the edge it kept and the edge its neighbour sends
 * (Section 3) -- so instances and tiles run ahead of one another as far as
 * their data allows.  A wait that exceeds the spin limit gives up: the
 * launch ends early, the fields are left partly advanced, and the next
 * swept_sync returns SWEPT_ETIMEOUT (SWEPT_EHIP if a queue was left
 * unserved, which a check after the launch detects).  SWEPT_BATCH_STAGED:
 * all tiles of all instances advance one stage per kernel launch (two
 * launches per stage, heat and KS).
 * Either way the launches of a batch are captured into one HIP graph, which
 * is reused when the same batch (same sizes, steps, parameters and
 * pointers) is advanced again.  Uses library scratch for the tables, the
 * edges (three copies of each ring) and, on the persistent schedule, one
 * flag per tile and one task number per region (below 2^31, else
 * SWEPT_EUNSUPPORTED).
 */
int swept_advance_batch(void *const *u, const int64_t *nx, const int64_t *nsteps,
                        const int32_t *stencil_id, const double *params, int64_t count);

/* Schedules for swept_set_batch_schedule. */
enum {
    SWEPT_BATCH_PERSISTENT = 0,   /* one persistent launch for the whole batch (default) */
    SWEPT_BATCH_STAGED = 1        /* one launch per stage and stencil */
};

/*
 * Select the schedule of later swept_advance_batch calls (the results are the
 * same bits either way) and tune the persistent one:
 *  - spin_limit: microseconds after which a wait gives up (0: the default,
 *    60 s; a wait normally lasts at most a few regions' run times);
 *  - chunk: task numbers a workgroup takes per claim (0: the default, 2);
 *    each run of them inside one stage shares one wait for its inputs;
 *  - queues: independent schedules per stencil, whole instances spread over
 *    them by work, each with its own counter.  0, the default: one queue
 *    per XCD, served only by the workgroups running on that XCD (so one L2
 *    holds every exchange of an instance and the hand-over needs no L2
 *    write-back), when a probe of the XCC_ID values tells the XCDs apart,
 *    else 32 queues; and a batch whose instances cannot be spread evenly
 *    (a queue with more than 1.25 times the mean work: a few large
 *    instances, which would leave XCDs idle) runs one launch per stage
 *    instead.  A positive number: that many queues, always persistent,
 *    workgroup w serving queue w mod queues, the hand-over at agent scope.
 * Needs no device; kept until swept_finalize.  SWEPT_EINVAL for an unknown
 * schedule, a limit below 0 or above 2^40 us, a chunk outside [0, 32] or
 * queues outside [0, 1024].
 */
int swept_set_batch_schedule(int32_t schedule, int64_t spin_limit, int32_t chunk,
                             int32_t queues);

/*
 * The naive schedule for a batch, the baseline of swept_advance_batch: one
 * launch per time step and stencil advances every instance that still has
 * steps to go (heat: one thread per point; KS: the fused RK2 step of
 * swept_naive_advance, per block of 256 points of one instance).  Same
 * arguments and same bits as swept_advance_batch.  Uses library scratch for
 * a second copy of every field (8 bytes per point) and synchronizes the
 * stream once to upload its tables.
 */
int swept_naive_advance_batch(void *const *u, const int64_t *nx, const int64_t *nsteps,
                              const int32_t *stencil_id, const double *params, int64_t count);

/*
 * Autotuner for swept_advance (paper, Section 4: Eq. (1) and its optimum
 * n* = sqrt(2 tau / s)).  With W-point tiles a sub-timestep costs
 * max(W s1, nx s_full) + 2 tau / W, where tau is the cost of a stage
 * boundary (end of a launch, edge round trip, next launch), s1 the time one
 * wavefront alone spends per point-substep and s_full the whole GPU's time
 * per point-substep; all three are measured with short runs of the stencil
 * on zero fields.  The prior W0 = max(nx s_full / s1, sqrt(2 tau / s1))
 * centres the candidates: the valid tile widths (even, dividing nx, within
 * the LDS budget) nearest W0/8, W0/4, W0/2, W0, 2 W0 and 4 W0 (the model
 * leaves out that wider tiles hold more LDS and so share a CU with fewer
 * others) and the width the untuned plan would take, each with 1, 2 or 4
 * pairs per lane (64 x pairs <= W/2), the two widest widths of at most 64
 * points on the lane-frame kernel (SWEPT_MODE_STAGE_LANE), and the naive
 * schedule.  Each tiling
 * is timed (best of three) over sixteen of its stages (at most
 * nsteps steps) on as many of its tiles as fill the GPU four times over (at
 * most nx points), the naive schedule over at most 256 steps of all nx
 * points, and the highest rate in point-steps per second is kept.  Later
 * swept_advance calls of the same stencil with floor(log2 nx) equal to this
 * one's, in SWEPT_MODE_AUTO with tile width and pairs per lane left at 0,
 * use it whenever the chosen width divides their nx.  Results never depend
 * on the choice.
 *
 * report (host, may be NULL) receives 8 doubles: tau [s], s1 [s], s_full [s],
 * n* = sqrt(2 tau / s1) [points], W0 [points], the chosen W (0 = naive), the
 * chosen pairs per lane (0 = the lane-frame kernel), the fastest probe's
 * rate [point-steps/s].  The call
 * allocates and frees its own probe fields and synchronizes the stream.
 */
int swept_autotune(int64_t nx, int64_t nsteps, int32_t stencil_id, const double *params,
                   int32_t nparams, double *report);

/*
 * Autotuner for swept_advance_batch: times the batch's own shapes (zero
 * fields; every step count scaled by one factor so that the longest instance
 * runs 6144 sub-timesteps, the others in proportion) under the current
 * schedule, best of two runs each, choosing the depth k in {128, 256, 384,
 * 512} for KS and then for heat (each with the other's depth set, since the
 * two stencils' launches overlap), and keeps the choice for later batches.  depth_out (host, 3 entries indexed by stencil id)
 * receives the chosen depth, 0 for a stencil not in the batch.  Allocates
 * and frees its own probe fields; synchronizes the stream.
 */
int swept_autotune_batch(const int64_t *nx, const int64_t *nsteps, const int32_t *stencil_id,
                         const double *params, int64_t count, int64_t *depth_out);

/* Forget every choice made by swept_autotune and swept_autotune_batch. */
int swept_clear_tuning(void);

/*
 * Per-stage timing.  With profiling enabled, swept_advance records a HIP
 * event on the current stream before its first and after every stage
 * launch.  swept_stage_times waits for those events and returns, for the
 * most recent swept_advance, the duration of each stage launch in
 * milliseconds (ms_out[i]) and which kernel ran it (kind_out[i]: 0 = banded
 * kernel -- the triangle or a stage capped at the target level, 1 =
 * continuous-band diamond kernel, 2 = lane-frame kernel, 3 = the unequal
 * tiling's kernel, which runs every stage of SWEPT_MODE_STAGE_RAGGED).  At most cap
 * entries are written; *count
 * receives the number of stages.  Either output array may be NULL.
 * Returns SWEPT_EINVAL if profiling is off or no swept run was recorded.
 */
int swept_set_profiling(int enable);
int swept_stage_times(double *ms_out, int32_t *kind_out, int64_t cap, int64_t *count);

/*
 * Gradient by the swept discrete adjoint (SWEPT_HEAT_F64, SWEPT_KS_F64).
 * For the objective
 *
 *   J(u0) = window_weight * sum_{j = window_first}^{nsteps} sum_i (u_i^j)^2
 *           + sum_i cot_final[i] * u_i^nsteps
 *
 * where u^j is the field after j time steps of the stencil, writes dJ/du0 to
 * grad_u0.  u0, grad_u0 and cot_final (NULL = 0) are DEVICE pointers to nx
 * elements; window_first > nsteps leaves out the window term.  The
 * derivative is that of the scheme's sub-timesteps in real arithmetic (each
 * sub-timestep's transposed Jacobian, applied in reverse order), evaluated
 * in a fixed order.
 *
 * A forward swept pass keeps the V edges of every stage (one checkpoint per
 * sweep, 2*nx points per stage; u0 is only read); the stages then run in
 * reverse, each region recomputing its forward values from its checkpoint
 * inside its wavefront.  Tiles: W = 2k, the largest k <= 32 with W dividing
 * nx (tile_w of swept_set_tuning, if set, caps k at tile_w/2).  Scratch
 * grows to about 2*nx*(stages)*sizeof(point) bytes, stages = 1 +
 * ceil(4*nsteps/k) for KS (24-byte points; 2^16 points and 20,000 steps at
 * k = 32: 7.9 GB).  Asynchronous on the current stream, like swept_advance.
 */
int swept_adjoint(const void *u0, void *grad_u0, int64_t nx, int64_t nsteps, int32_t stencil_id,
                  const double *params, int32_t nparams, int64_t window_first,
                  double window_weight, const void *cot_final);

/*
 * The same gradient by the straight decomposition of the discrete adjoint,
 * the baseline of swept_adjoint: a forward pass of one launch per time step
 * that keeps the field of every step, then one launch per time step
 * backwards (each recomputes that step's sub-timestep levels on a halo and
 * applies their transposes).  Same arguments and same bits as
 * swept_adjoint.  Scratch: (nsteps + 3) fields of nx points (KS at 2^16
 * points and 20,000 steps: 10.5 GB); SWEPT_ENOMEM if that cannot be had.
 */
int swept_naive_adjoint(const void *u0, void *grad_u0, int64_t nx, int64_t nsteps,
                        int32_t stencil_id, const double *params, int32_t nparams,
                        int64_t window_first, double window_weight, const void *cot_final);

/*
 * The objective of swept_adjoint, evaluated by the library (SWEPT_HEAT_F64,
 * SWEPT_KS_F64 and their _FMA forms):
 *
 *   J = window_weight * sum_{j = max(window_first, 0)}^{nsteps} sum_i (u_i^j)^2
 *       + sum_i cot_final[i] * u_i^nsteps
 *
 * written as one double to J_out (a DEVICE pointer), asynchronously on the
 * current stream.  u0 and cot_final (NULL = 0) are DEVICE pointers to nx
 * doubles; u0 is only read.  A copy of u0 advances by the swept schedule to
 * the step before the window, then one naive launch per step of the window
 * (the sum needs every one of its fields).  Each step's sum is formed on the
 * device in a fixed order and the steps are accumulated with compensated
 * (two-sum) addition, so J does not depend on timing and its relative
 * rounding error is a few units of 1e-16 rather than growing with the number
 * of steps -- what a finite-difference check of the gradient differences.
 * Uses its own device buffer (nx doubles and 8 KiB), grown on demand.
 */
int swept_window_objective(const void *u0, int64_t nx, int64_t nsteps, int32_t stencil_id,
                           const double *params, int32_t nparams, int64_t window_first,
                           double window_weight, const void *cot_final, void *J_out);

/*
 * Wait for the current stream; report asynchronous kernel errors, and
 * SWEPT_ETIMEOUT if a persistent batch launched since the last call gave up
 * a wait (the flag is then cleared).
 */
int swept_sync(void);

/* Message for the last failure on this thread ("" if none).  Never NULL. */
const char *swept_last_error(void);

/* Release scratch and forget the device.  Safe to call more than once. */
void swept_finalize(void);

#ifdef __cplusplus
}
#endif

#endif /* SWEPT_H */
