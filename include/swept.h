/*
 * swept.h -- C ABI of the MI355X (gfx950) swept time-space decomposition
 * library for explicit 1-D periodic stencils.
 *
 * Method: Magee & Niemeyer, "An initial investigation of the performance of
 * GPU-based swept time-space decomposition" (arXiv 1612.02495).  A workgroup
 * advances one spatial tile ("node", Sec. 4.2) through many tiers of the
 * space-time plane without leaving on-chip memory: an up-triangle phase, then
 * diamond phases whose tiling is shifted by half a tile each time
 * (the zig-zag of Sec. 4.2), then a closing down-triangle phase that emits the
 * full solution row.  Only the two outermost stencil-radius bands of every
 * tier ("edges", Sec. 4.2 Figs. firstorder/collection; four values per side
 * per sub-step for the five-point stencil, Sec. 4.3) pass through HBM between
 * launches.  The swept rule does not change the numerical scheme (Sec. 2), so
 * every entry point below returns exactly what the plain timestepper returns
 * for the same precision and operation order.
 *
 * Checking aid: with SWEPT_DEBUG_POISON set (to anything but "" or "0")
 * when a plan, batch or adjoint plan is created, its edge slots (and the
 * adjoints' checkpoints and lambda slots) are filled with quiet NaNs before
 * each run, and each tile's LDS buffers (band buffer, staging row, tier rows,
 * halo exchange words) are filled with quiet NaNs when the tile starts, so an
 * entry read before a phase or tile wrote it shows up as NaN in the result.
 * Results are unchanged otherwise; the fill costs one pass over the workspace
 * per run.
 *
 * Schemes (Sec. 4.1 and Appendix; periodic boundaries, index (i+k) mod n,
 * except for the insulated rod):
 *   SWEPT_HEAT_FTCS  T_i^{m+1} = Fo (T_{i+1}^m + T_{i-1}^m) + (1 - 2 Fo) T_i^m,
 *                    Fo = alpha dt / dx^2                       (Eq. HeatDisc)
 *   SWEPT_KS_RK2     Kuramoto-Sivashinsky, 5-point central differences
 *                    (Eq. KSDisc) advanced by the RK2 midpoint rule
 *                    (predictor with dt/2, then final with dt).
 *   SWEPT_HEAT_INSULATED  the heat scheme on a rod of n nodes with insulated
 *                    ends (Sec. 4.1; Appendix): mirror ghosts about the end
 *                    nodes, T_{-1} = T_1 and T_n = T_{n-2}.  The rod is laid
 *                    on the same ring of tiles; only the tiles that hold node
 *                    0 or n-1 (where the ring closes) use the ghost values.
 * Rounding (the paper states no operation order): IEEE round to nearest even,
 * constants formed on the host in double (rounded once to float for FP32
 * plans), divisions replaced by products with host-formed inverses (Sec. 5).
 * The heat update is fma(Fo, T_{i+1} + T_{i-1}, (1 - 2 Fo) T_i), one rounding
 * of the product-sum.  The KS right-hand side sums its terms left to right,
 * with the multiples 2u_i, 4u_{i+-1} and 6u_i of the difference numerators
 * fused into the sums they join and u_{i+1}^2 - u_{i-1}^2 unfused; each RK2
 * stage is one fused multiply-add, u + (dt/2) f and u + dt f.
 *
 * Conventions shared by all entry points
 *   - Return value: SWEPT_OK (0) or a negative swept status code.  Nothing
 *     crosses the ABI as an exception.  The message of the last failure on
 *     the calling thread is available from swept_last_error().
 *   - Argument validation happens before any HIP call: an invalid call
 *     touches neither the device nor the caller's buffers.
 *   - Device pointers are HIP device allocations owned by the caller,
 *     contiguous, of the plan's dtype, aligned to the element size.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Runs are enqueued asynchronously on it; the caller synchronises.
 *   - A plan owns its device workspace (edge strips and the naive ping-pong
 *     buffer), allocated by swept_plan_create and freed by swept_plan_destroy.
 *     A plan must not be used on two streams at the same time.
 *   - The current HIP device at swept_plan_create is the plan's device; later
 *     calls make it current for their duration.
 */
#ifndef SWEPT_H
#define SWEPT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* status codes */
#define SWEPT_OK 0
#define SWEPT_EINVAL -1        /* bad argument                               */
#define SWEPT_EUNSUPPORTED -2  /* valid request this build cannot tile       */
#define SWEPT_ENOMEM -3        /* device allocation failed                   */
#define SWEPT_EDEVICE -4       /* HIP runtime error (message in last_error)  */
#define SWEPT_ENONFINITE -5    /* the opt-in check found a non-finite value  */
/* There is no time-out status: no kernel of this library waits on another
   workgroup or on the host (the batched kernel's workgroups only take work
   from a counter and never spin), so every launch ends on its own. */

/* check flags (swept_plan_set_checks, swept_batch_set_checks) */
#define SWEPT_CHECK_NONFINITE 1 /* after each run, scan the grid for NaN/Inf */

/* stencil kinds */
#define SWEPT_HEAT_FTCS 0
#define SWEPT_KS_RK2 1
#define SWEPT_HEAT_INSULATED 2 /* heat, rod with insulated ends: plans with
                                  tile_width 512 or 1024 (n a multiple of
                                  it), swept on the compacted engine; not in
                                  the batched or adjoint entry points       */

/* element types */
#define SWEPT_F32 0
#define SWEPT_F64 1

/* phase engines (swept_plan_set_engine) */
#define SWEPT_ENGINE_AUTO 0 /* compacted engine where it applies, else the
                               register engine, else LDS                      */
#define SWEPT_ENGINE_LDS 1  /* tile in LDS, two tier rows, one thread block    */
#define SWEPT_ENGINE_WAVE 2 /* tile in the registers of one wave64, DPP halos   */
#define SWEPT_ENGINE_COMPACT 3 /* wave64 per tile, V/Lambda compacted onto the
                                  lanes: R points per lane as the part grows or
                                  shrinks, bands in LDS                         */
#define SWEPT_ENGINE_RESIDENT 4 /* batched runs only: grids of at most 16384
                                   points whole in one workgroup's registers,
                                   the rest as compacted tiles                 */

typedef struct swept_plan_s* swept_plan;

/*
 * swept_plan_create -- build a plan for one periodic grid of n points.
 *   out             receives the plan handle (host pointer, required).
 *   n               number of grid points: a multiple of the tile width, or,
 *                   for tile width 512 or 1024 and n >= 32 (periodic kinds),
 *                   any n -- then the ring is cut into tiles of uneven width
 *                   (two halves of at most tile_width / 2 points each, all
 *                   but one half a multiple of 4 s points; the edge passing
 *                   of Sec. 4.2 needs no equal tiles), run on the compacted
 *                   engine; the phase height is then at most the smallest
 *                   half's triangle.
 *   kind, dtype     SWEPT_HEAT_FTCS / SWEPT_KS_RK2 / SWEPT_HEAT_INSULATED,
 *                   SWEPT_F32 / SWEPT_F64.
 *   dt, dx          timestep and grid spacing (finite, dx != 0).
 *   alpha           diffusivity (heat kinds only; ignored for KS).
 *   tile_width      points per tile ("node", Sec. 4.2): a multiple of 2s
 *                   (s = 1 heat, 2 KS) and of 8 for KS, 4..4096; 0 picks one:
 *                   the autotuned configuration for (kind, dtype, n) when
 *                   one is known (see swept_autotune; used only together with
 *                   steps_per_cycle = 0), else the largest power of two up to
 *                   1024 dividing n if it is at least 256, else the uneven
 *                   tiling at 1024 (n >= 32).
 *   steps_per_cycle timesteps per full phase: 1..w/2 (heat), 1..w/8 (KS);
 *                   0 = the pure triangle height (w/2 heat, w/8 KS).
 * Discretisation constants are formed once on the host in double and, for
 * SWEPT_F32, rounded once to float: Fo = (alpha*dt)/(dx*dx), 1-2Fo,
 * 1/(4dx), 1/dx^2, (1/dx^2)^2, dt, dt/2 (inverses instead of divisions,
 * Sec. 5).  Size limit: a phase launches one workgroup per tile and a
 * dispatch counts at most 2^32 - 1 work-items, so n / tile_width tiles times
 * the engine's work-items per tile (64 for the register engines, up to 256
 * for LDS) must stay below 2^32 -- e.g. n < 2^36 at tile width 1024; the
 * plan fails with EUNSUPPORTED otherwise (naive_run takes any n).  Indices
 * are 64-bit throughout.  Errors: EINVAL (bad argument), EUNSUPPORTED (n not
 * tileable with a supported width, or too many tiles), ENOMEM / EDEVICE
 * (allocation).
 */
int swept_plan_create(swept_plan* out, int64_t n, int kind, int dtype, double dt, double dx,
                      double alpha, int tile_width, int steps_per_cycle);

/*
 * swept_run -- advance u (device, n elements, in/out) by `steps` timesteps
 * with the swept decomposition (Sec. 4.2-4.3): one up-triangle launch,
 * diamond launches, one down-triangle launch; the last phase is a flattened
 * (trapezoid) phase when steps is not a multiple of steps_per_cycle.
 * steps == 0 is a no-op.  Result is bit-identical to naive_run.
 */
int swept_run(swept_plan p, void* u, int64_t steps, void* stream);

/*
 * swept_run_noalloc -- swept_run without a plan, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Arguments n .. steps_per_cycle are those
 * of swept_plan_create and are validated the same way, except that
 * tile_width = 0 takes the default width (as swept_plan_create without an
 * autotuned entry) and never the autotuner's table; u, steps and stream are those
 * of swept_run, and the result is the same, bit for bit.  Nothing is
 * allocated: the edge slots live in a static array in the library's device
 * memory, 32 MiB per GPU (held by each GPU the library runs on until the
 * process ends; its address is looked up on the first call on each device).
 * A grid whose edge slots need more, 2 (n / tile_width) (tile_width + 2 s)
 * values (about 16 bytes per point in FP64, so n up to about 2^21 at tile
 * width 1024), fails with EUNSUPPORTED before anything is launched.  Every call
 * on one GPU uses that GPU's one array, and nothing in it needs to start at
 * zero (each phase writes every slot entry before the next phase reads it);
 * calls that overlap on one GPU (on two streams, or from two threads) race on
 * it and must be serialised by the caller.  The current HIP device is the
 * device the call runs on.
 */
int swept_run_noalloc(int64_t n, int kind, int dtype, double dt, double dx, double alpha, int tile_width,
                      int steps_per_cycle, void* u, int64_t steps, void* stream);

/*
 * naive_run -- the classic decomposition (Sec. 4.4): one kernel launch per
 * sub-timestep reading and writing global memory, ping-ponging with the
 * plan's buffer.  Same arguments and result as swept_run.
 */
int naive_run(swept_plan p, void* u, int64_t steps, void* stream);

/*
 * swept_plan_info -- report the plan's tile width, timesteps per full phase
 * and device workspace size in bytes.  Any output pointer may be NULL.
 */
int swept_plan_info(swept_plan p, int* tile_width, int* steps_per_cycle, size_t* workspace_bytes);

/*
 * swept_plan_set_engine -- choose the kernel that runs the phases:
 * SWEPT_ENGINE_AUTO, _LDS, _WAVE or _COMPACT.  _WAVE requires tile_width =
 * 64*P with P in {2, 4, 8, 16} for heat and {4, 8, 16} for KS; _COMPACT
 * requires P in {8, 16} for either kind; a plan of uneven tiles (tile width
 * not dividing n) runs on _COMPACT (or AUTO) only; otherwise the call fails
 * with EUNSUPPORTED and the plan keeps its engine.  Every engine computes the
 * same values bit for bit and leaves the same edge slots, so the choice
 * changes only the speed.  An engine whose launch would exceed the size limit
 * of swept_plan_create also fails with EUNSUPPORTED.
 */
int swept_plan_set_engine(swept_plan p, int engine);

/*
 * swept_plan_set_checks -- opt-in checks of the plan's runs (0 = none, the
 * default).  With SWEPT_CHECK_NONFINITE, swept_run and naive_run enqueue,
 * after their phases, a scan of the n values of u that sets a plan-owned
 * device flag when any value is NaN or infinite (the scheme itself never
 * makes one from finite data unless it is unstable, e.g. Fo > 1/2), then wait
 * for their stream and return SWEPT_ENONFINITE if the flag is set; u holds
 * the run's result either way.  With the check on, runs are therefore
 * synchronous and cannot be captured into a graph.  The first call with the
 * flag allocates the 4-byte flag.  Errors: EINVAL (NULL plan, unknown flags),
 * ENOMEM.
 */
int swept_plan_set_checks(swept_plan p, int flags);

/* swept_plan_destroy -- free the plan and its workspace (NULL is a no-op). */
void swept_plan_destroy(swept_plan p);

/* swept_last_error -- message of the last failure on this thread ("" if none). */
const char* swept_last_error(void);

/*
 * swept_schedule -- host-only query of the phase schedule swept_run uses.
 * Writes the heights (in tiers: timesteps for heat, sub-steps for KS) of the
 * edge sets passed between consecutive launches into heights[0..cap) and
 * their number into *count; swept_run makes (*count + 1) launches.  Every
 * height equals the full phase height except possibly the last.
 * tile_width and steps_per_cycle as for swept_plan_create (0 = default for
 * steps_per_cycle; tile_width must be given).  No device is touched.
 */
int swept_schedule(int kind, int tile_width, int steps_per_cycle, int64_t steps, int32_t* heights,
                   int64_t cap, int64_t* count);

/*
 * swept_tile_geometry -- host-only query of the per-tile sizes the kernels
 * use for a kind and tile width w (any output pointer may be NULL):
 *   full_tiers       tiers of a full triangle: w/2 (heat), w/4 (KS), i.e. the
 *                    triangle of Sec. 4.2 whose tier k holds w - 2 s k values;
 *   row_values       values per LDS tier row, w + 2s (the two-row matrix of
 *                    Sec. 4.2 holds 2 (w + 2) values for the 3-point stencil);
 *   edge_slot_values values per edge slot in HBM, (w/2 + s) positions x 2.
 * Errors: EINVAL for an unknown kind or an invalid width.  No device is touched.
 */
int swept_tile_geometry(int kind, int tile_width, int* full_tiers, int* row_values,
                        int* edge_slot_values);

/* ------------------------------------------------------------ autotuner -- */

/* One timed candidate of swept_autotune. */
typedef struct {
  int32_t tile_width;
  int32_t steps_per_cycle;
  int32_t engine;   /* SWEPT_ENGINE_LDS, _WAVE or _COMPACT */
  int32_t reserved; /* zero */
  double ns_per_cell_update;
} swept_tune_result;

/*
 * swept_autotune -- time the candidate configurations for a grid of n points
 * and remember the fastest for (kind, dtype, n).  Candidates: every
 * power-of-two tile width 64..2048 that divides n (and 512 and 1024 with
 * uneven tiles when they do not), each engine that has a kernel for it, and
 * phase heights of 1, 3/4, 1/2 and 1/4 of the full triangle -- the per-size search
 * of the best launch configuration of Sec. 5, extended to the swept
 * parameters.  Each candidate runs `steps` timesteps (0 = 2048 heat / 512 KS;
 * clamped to 4096 / 1024) on a library-owned zero grid, once to warm up and
 * three times timed with HIP events on a library-owned stream; the best of
 * the three counts.  Argument values dt, dx, alpha only feed the constants
 * (timing does not depend on them).
 *   results/cap/count  optional: every timed candidate (count = how many ran)
 *   tile_width, steps_per_cycle, engine  optional: the winner
 * The winner is stored in the process table and, if the environment variable
 * SWEPT_AUTOTUNE_CACHE names a file, merged into that JSON file.  A later
 * swept_plan_create with tile_width = 0 and steps_per_cycle = 0 for the same
 * (kind, dtype, n) uses it.  Errors: EINVAL, EUNSUPPORTED (no width divides
 * n), ENOMEM / EDEVICE.  Synchronous: returns after the timing finished.
 */
int swept_autotune(int64_t n, int kind, int dtype, double dt, double dx, double alpha, int64_t steps,
                   swept_tune_result* results, int cap, int* count, int* tile_width, int* steps_per_cycle,
                   int* engine);

/*
 * swept_autotune_lookup -- host-only: the remembered configuration for
 * (kind, dtype, n) from the process table or the SWEPT_AUTOTUNE_CACHE file.
 * EUNSUPPORTED when there is none.  Output pointers may be NULL.
 */
int swept_autotune_lookup(int64_t n, int kind, int dtype, int* tile_width, int* steps_per_cycle, int* engine,
                          double* ns_per_cell_update);

/* swept_autotune_forget -- host-only: clear the process table (files untouched). */
void swept_autotune_forget(void);

/* -------------------------------------------------------------- batched -- */

typedef struct swept_batch_s* swept_batch;

/*
 * swept_batch_create -- plan a batch of nprob independent periodic grids of
 * uneven size, all of one kind and dtype, each advanced by `steps` timesteps
 * per swept_batch_run.
 *   n[i]                 points of grid i (host array): any 32 <= n[i] <= 2^30
 *                        (other sizes fail with EUNSUPPORTED)
 *   dt[i], dx[i], alpha[i]  per-grid parameters (host arrays; alpha is read
 *                        for heat only and may be NULL for KS); constants are
 *                        formed as in swept_plan_create
 * The grids live back to back in one device array in input order (offsets
 * from swept_batch_info).  With the default engine (AUTO, the same as
 * RESIDENT), every grid of at most 16384 points runs whole in one workgroup
 * of 1, 4, 8 or 16 waves, 16 points per lane held in registers for all the
 * steps (the last lane holding the n mod 16 remaining points), halos passed
 * between lanes and waves each sub-step: a single tile whose phase is the
 * whole run, with no edge band through HBM; these workgroups run beside the
 * persistent kernel.  Every other grid (every grid with the COMPACT or WAVE
 * engine) is run with the swept rule of swept_run: wave-resident tiles of at
 * most 64 P points (P = 8 points per lane for heat with the COMPACT engine,
 * 16 otherwise) with two halves of uneven width (measured in points; in
 * whole 16-point lanes for WAVE), flattened phases on the wider halves,
 * zig-zag tilings, edge bands through HBM (Sec. 4.2-4.3), by one persistent kernel:
 * each workgroup pulls the next grid, largest first, from a device counter
 * and advances it through all of its phases.  The plan owns the edge slots,
 * the grid descriptors and the counter.  Each resident size class is one
 * launch of one workgroup per grid, so more than 2^32 / (64 x its waves)
 * grids of one class fail with EUNSUPPORTED.  Errors: EINVAL, EUNSUPPORTED,
 * ENOMEM, EDEVICE.
 */
int swept_batch_create(swept_batch* out, int32_t nprob, const int64_t* n, int kind, int dtype, const double* dt,
                       const double* dx, const double* alpha, int64_t steps);

/*
 * swept_batch_run -- advance every grid of u (device, sum n[i] elements,
 * in/out) by the plan's steps.  use_graph != 0: the whole-grid kernel, the
 * counter reset and the persistent kernel are captured once into a HIP graph
 * (re-captured when u changes) and replayed with one graph launch;
 * use_graph == 0: the same launches enqueued directly.  Asynchronous on `stream`.  Results equal
 * naive_run / swept_run of each grid on its own, bit for bit.
 */
int swept_batch_run(swept_batch b, void* u, int use_graph, void* stream);

/*
 * swept_batch_set_engine -- choose how the grids run: SWEPT_ENGINE_RESIDENT
 * (grids of at most 16384 points whole in the register-resident kernels, the
 * rest as compacted swept tiles), SWEPT_ENGINE_COMPACT (every grid as
 * compacted swept tiles: compacted layouts, edge bands in LDS),
 * SWEPT_ENGINE_WAVE (every grid as register-engine swept tiles, every tier
 * over the whole tile; every n[i] must be a multiple of 16, else
 * EUNSUPPORTED) or SWEPT_ENGINE_AUTO (the default, the same as
 * RESIDENT: measured fastest on the 4096-grid heat and KS workloads).  All
 * give the same values bit for bit.  Changing the
 * engine rebuilds the grid descriptors and edge slots, re-sizes the
 * persistent grid (the engines need different LDS) and drops a captured
 * graph, so call it between runs, never while one is in flight.  SWEPT_ENGINE_LDS fails with
 * EUNSUPPORTED, other values with EINVAL; on failure the plan keeps its
 * engine.
 */
int swept_batch_set_engine(swept_batch b, int engine);

/*
 * swept_batch_info -- total points, per-grid offsets into u (host array of
 * nprob entries, may be NULL), edge-slot bytes and persistent grid size.
 */
int swept_batch_info(swept_batch b, int64_t* total_points, int64_t* offsets, size_t* workspace_bytes, int* grid);

/*
 * swept_batch_set_checks -- as swept_plan_set_checks for a batch: with
 * SWEPT_CHECK_NONFINITE the scan of all grids' values is part of each run
 * (of the captured graph too), and swept_batch_run waits for its stream and
 * returns SWEPT_ENONFINITE when any grid holds a NaN or infinite value.
 * Changing the flags drops a captured graph.  Errors: EINVAL, ENOMEM.
 */
int swept_batch_set_checks(swept_batch b, int flags);

/* swept_batch_destroy -- free the plan and its device memory (NULL is a no-op). */
void swept_batch_destroy(swept_batch b);

/* -------------------------------------------------------------- adjoint -- */

typedef struct swept_adjoint_s* swept_adjoint;

/*
 * swept_adjoint_create -- plan the gradient of a functional of u_T for a
 * batch of `batch` periodic heat FTCS grids of n points each (Eq. HeatDisc),
 * all with the same dt, dx and number of steps, each with its own alpha.
 *   batch  1 .. 65535
 *   dtype  SWEPT_F64 (other types fail with EUNSUPPORTED)
 *   n      a positive multiple of 64
 *   steps  >= 1
 * The forward pass runs swept phases of 32 steps on tiles of 64 points and
 * keeps the edge slots every phase writes (the swept state between
 * launches) as checkpoints; the first steps mod 32 run with the classic
 * scheme and keep their grids.  Workspace: about 2.06 n x 8 bytes per grid
 * per phase of checkpoints, (steps mod 32 + 1) grids per grid of classic
 * states, plus O(n) buffers -- all owned by the plan (swept_adjoint_info
 * reports the checkpoint size).  batch x n (n rounded up to 256) must stay
 * below 2^32, the work-items of one classic-step launch; larger requests
 * fail with EUNSUPPORTED.  Errors: EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE.
 */
int swept_adjoint_create(swept_adjoint* out, int32_t batch, int64_t n, int dtype, double dt, double dx,
                         int64_t steps);

/*
 * swept_adjoint_create_segmented -- swept_adjoint_create with two-level
 * checkpointing: the edge state of only every `segment`-th phase (phases
 * K mod segment, K mod segment + segment, .., K - segment, with K = steps / 32
 * phases and `segment` capped at K) is kept by swept_forward_ckpt, and
 * swept_adjoint_run recomputes the edge states of the other phases, segment by
 * segment just before it reverses each, from the kept state below them (from
 * the initial state for the phases below the first kept one) into one reused
 * set of segment - 1 buffers.  The top segment's states are the forward's
 * own, left in those buffers.  Checkpoint memory falls from K sets to
 * floor(K / segment) + segment - 1 sets, at the cost of about one more forward
 * pass in swept_adjoint_run (K - floor(K / segment) - segment + 1 phases); the
 * gradients are the same bits as with every phase kept (the recomputed states
 * are the same bits).  segment = 1 is swept_adjoint_create; segment = 0 picks
 * ceil(sqrt(K)), about 2 sqrt(K) sets (e.g. 64 grids of 2^18 points over 10^4
 * steps: 34 sets, 9.4 GB, instead of 312 sets, 86 GB).  Errors as
 * swept_adjoint_create, and EINVAL for segment < 0.
 */
int swept_adjoint_create_segmented(swept_adjoint* out, int32_t batch, int64_t n, int dtype, double dt, double dx,
                                   int64_t steps, int segment);

/*
 * swept_forward_ckpt -- u_T = A(alpha)^steps u_0 for every grid, storing the
 * checkpoints the reverse sweep restarts from.  u0, uT: device, batch x n
 * doubles, row-major (grid b at b*n), may not alias; alpha: device, batch
 * doubles, read once here (Fo = (alpha dt)/(dx dx) per grid, as in
 * swept_plan_create).  Asynchronous on `stream`.  The result equals
 * swept_run / naive_run of each grid bit for bit.
 */
int swept_forward_ckpt(swept_adjoint a, const void* u0, const double* alpha, void* uT, void* stream);

/*
 * swept_adjoint_run -- reverse sweep after swept_forward_ckpt: given
 * g_uT = dJ/du_T (device, batch x n), writes g_u0 = dJ/du_0 (device,
 * batch x n) and g_alpha = dJ/dalpha (device, batch doubles).  For
 * J = 1/2 ||u_T - y||^2, g_uT = u_T - y.  Each swept phase, last to first,
 * is recomputed from its checkpointed edge slots in LDS and swept backwards
 * (lambda_m = A lambda_{m+1}: A is symmetric) while dJ/dalpha accumulates
 * lambda_{m+1} . (dt/dx^2)(u_{m,i-1} + u_{m,i+1} - 2 u_{m,i}); the sum is
 * reduced in a fixed order (deterministic).  g_u0 equals steps applications
 * of the forward stencil to g_uT, bit for bit.  Asynchronous on `stream`.
 * EINVAL if no forward pass ran on this plan.
 */
int swept_adjoint_run(swept_adjoint a, const void* g_uT, void* g_u0, double* g_alpha, void* stream);

/* swept_adjoint_info -- checkpoint bytes, tile width (64), steps per cycle
 * (32) and the number of leading classic steps (steps mod 32). */
int swept_adjoint_info(swept_adjoint a, size_t* checkpoint_bytes, int* tile_width, int* steps_per_cycle,
                       int64_t* leading_classic_steps);

/* swept_adjoint_destroy -- free the plan and its workspace (NULL is a no-op). */
void swept_adjoint_destroy(swept_adjoint a);

/* ----------------------------------------------------------- KS adjoint -- */

typedef struct swept_ks_adjoint_s* swept_ks_adjoint;

/*
 * swept_ks_adjoint_create -- plan dJ/du_0 for a functional J of u_T, for a
 * batch of `batch` periodic Kuramoto-Sivashinsky grids of n points each,
 * advanced with the RK2 midpoint scheme of Sec. 4.1 (Eq. KSDisc, Appendix):
 * q = u + (dt/2) f(u), u' = u + dt f(q), f the 5-point right-hand side, with
 * the constants of swept_plan_create for SWEPT_KS_RK2.  All grids share dt,
 * dx and the number of steps.
 *   batch  1 .. 65535
 *   dtype  SWEPT_F64 (other types fail with EUNSUPPORTED)
 *   n      a positive multiple of 64
 *   steps  >= 1
 * The forward pass runs swept phases of 8 steps (16 sub-step tiers) on tiles
 * of 64 points and keeps the edge bands every phase writes as checkpoints;
 * the first steps mod 8 run with the classic scheme and keep their grids.
 * Workspace: about 2.1 n x 8 bytes per grid per phase of checkpoints,
 * (steps mod 8 + 1) grids per grid of classic states, plus O(n) buffers --
 * all owned by the plan (swept_ks_adjoint_info reports the checkpoint size).
 * batch x n (rounded up to 256) must stay below 2^32, the work-items of one
 * classic-step launch; larger requests fail with EUNSUPPORTED.
 * Errors: EINVAL, EUNSUPPORTED, ENOMEM.
 */
int swept_ks_adjoint_create(swept_ks_adjoint* out, int32_t batch, int64_t n, int dtype, double dt, double dx,
                            int64_t steps);

/*
 * swept_ks_forward_ckpt -- u_T for every grid, storing the checkpoints the
 * reverse sweep restarts from.  u0, uT: device, batch x n doubles,
 * row-major (grid b at b*n), may not alias.  Asynchronous on `stream`.  The
 * result equals swept_run / naive_run of each grid bit for bit.
 */
int swept_ks_forward_ckpt(swept_ks_adjoint a, const void* u0, void* uT, void* stream);

/*
 * swept_ks_adjoint_run -- reverse sweep after swept_ks_forward_ckpt: given
 * g_uT = dJ/du_T (device, batch x n), writes g_u0 = dJ/du_0 (device,
 * batch x n; may not alias g_uT).  For J = 1/2 ||u_T - y||^2, g_uT = u_T - y.
 * Each step is reversed as mu = dt Jf(q)^T lambda',
 * lambda = (lambda' + mu) + (dt/2) Jf(u)^T mu (the last product-sum one fused
 * multiply-add; Jf(v)^T w gathered at i from v_i and w_{i-1}, w_{i+1}, w_i,
 * w_{i-2}, w_{i+2} in that order, each term after the first fused into the
 * running sum), with q and u recomputed
 * phase by phase from the checkpoints; every swept phase, last to first, is
 * one launch that recomputes its tiles in registers and walks the adjoint
 * back through them.  Deterministic (no atomics, a fixed operation order).
 * Asynchronous on `stream`.  EINVAL if no forward pass ran on this plan.
 */
int swept_ks_adjoint_run(swept_ks_adjoint a, const void* g_uT, void* g_u0, void* stream);

/* swept_ks_adjoint_info -- checkpoint bytes, tile width (64), steps per
 * cycle (8) and the number of leading classic steps (steps mod 8). */
int swept_ks_adjoint_info(swept_ks_adjoint a, size_t* checkpoint_bytes, int* tile_width, int* steps_per_cycle,
                          int64_t* leading_classic_steps);

/* swept_ks_adjoint_destroy -- free the plan and its workspace (NULL is a no-op). */
void swept_ks_adjoint_destroy(swept_ks_adjoint a);

#ifdef __cplusplus
}
#endif

#endif /* SWEPT_H */
