/*
 * sw.h - C ABI of libsw, an MI355X (gfx950) library for the explicit
 * two-step Lax-Wendroff time step of the 2-D shallow-water equations.
 *
 * The operation is the one of the paper's "Shallow Water Model" section:
 * conserved state U = (h, hu, hv) at cell centres of a structured grid with a
 * one-cell halo; per time step
 *   (a) boundary values in the halo, applied outside the stencil kernel;
 *   (b) dt from the CFL bound dt <= dx / (sqrt(g h) + |u|), here recomputed
 *       every step as dt = cfl * min(dx, dy) / max_cells(max(|u|, |v|) + sqrt(g h)),
 *       or a fixed dt (the paper's mode);
 *   (c) step 1: half-step states on every cell face,
 *         U_{i+1/2,j} = (U_i + U_{i+1})/2 - dt/(2 dx) (F(U_{i+1}) - F(U_i))
 *         U_{i,j+1/2} = (U_j + U_{j+1})/2 - dt/(2 dy) (G(U_{j+1}) - G(U_j));
 *   (d) step 2: dimensionally unsplit conservative update
 *         U^{n+1} = U^n - dt/dx (F_{i+1/2} - F_{i-1/2}) - dt/dy (G_{j+1/2} - G_{j-1/2})
 *       with F, G the SWE fluxes evaluated at the face states;
 *   (e) double buffering: inputs are read-only, every output cell is written
 *       by exactly one thread into the other buffer.
 * The half-step sign follows the paper's Fortran face statement (its printed
 * equation has the opposite sign and F in place of G in y).
 *
 * Conventions
 *  - Every call returns sw_status (0 = ok, < 0 = error).  Nothing aborts or
 *    throws across the ABI.  On error, sw_last_error_detail() holds a
 *    thread-local message.
 *  - "device pointer" = memory from hipMalloc (or a torch CUDA tensor) on the
 *    current HIP device; "host pointer" = ordinary process memory.
 *  - Streams are passed as void* (a hipStream_t; NULL = the null stream).
 *    Calls marked async only enqueue work on that stream.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef SW_H
#define SW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SW_OK = 0,
    SW_EINVAL = -1,     /* bad argument: shape, pointer, alignment, option combination */
    SW_ENOTSUP = -2,    /* valid but unsupported (halo width != 1, ...) */
    SW_ENOMEM = -3,     /* host or device allocation failed */
    SW_EHIP = -4,       /* a HIP runtime call failed (detail in sw_last_error_detail) */
    SW_EUNSTABLE = -5   /* sticky: a step produced h <= 0 or a non-finite value */
} sw_status;

typedef enum { SW_F32 = 0, SW_F64 = 1 } sw_dtype;

/* Global boundary conditions (the paper leaves them to the programmer, outside
 * the kernel).  REFLECT: solid wall, ghost = mirror of the edge cell with the
 * wall-normal momentum negated.  PERIODIC: ghost = opposite edge cell.
 * Corner ghosts are the x-then-y composition of the two rules. */
typedef enum { SW_BC_REFLECT = 0, SW_BC_PERIODIC = 1 } sw_bc;

/* SW_SCHEME_PAPER: the paper's step 1 (1-D differences only).
 * SW_SCHEME_TRANSVERSE: step 1 also carries the transverse flux term
 *   - dt/(2 dy) * 1/4 [(G_{i,j+1} + G_{i+1,j+1}) - (G_{i,j-1} + G_{i+1,j-1})]
 * on x faces (and the mirrored F term on y faces): the standard 2-D
 * Lax-Wendroff, linearly stable up to CFL ~0.6 (not in the paper). */
typedef enum { SW_SCHEME_PAPER = 0, SW_SCHEME_TRANSVERSE = 1 } sw_scheme;

typedef struct { int32_t nx, ny; } sw_grid;                    /* interior cells */
typedef struct { int32_t left, right, down, up; } sw_halo;     /* the paper's halo = [left, right, down, up] */

typedef struct {
    sw_dtype dtype;     /* arithmetic and storage type of the state */
    sw_bc bc_x, bc_y;   /* boundary condition on the x walls and on the y walls */
    sw_scheme scheme;
    double dy;          /* <= 0 means dy = dx */
    double cfl;         /* > 0: per-step CFL dt with this Courant number */
    double dt_fixed;    /* > 0: fixed dt.  Exactly one of cfl, dt_fixed is > 0 */
} sw_opts;

/* Device layout of one state plane, chosen by the library.
 * Cell (i, j), i in [-1, nx], j in [-1, ny] (ghosts at -1 and nx / ny) lives at
 * element  origin + j * pitch + i  of the plane.  Rows are 256-byte aligned
 * at the first interior column, so the interior is vector-load aligned.
 *
 * The rows of the three planes of a buffer interleave: a buffer is one
 * allocation of buffer_elems elements, plane k (0 h, 1 hu, 2 hv) starts at
 * element k * plane_offset of it, and row j of h, hu and hv lie next to each
 * other (pitch = 3 * plane_offset).  A step then streams one contiguous region
 * per buffer instead of three distant ones; on MI355X this was measured 2-6 %
 * faster at the same bytes.  Any other placement in which each plane pointer
 * addresses plane_elems elements and no two planes share an element also
 * works, at the speed of whatever it leaves to the memory system. */
typedef struct {
    int64_t pitch;         /* elements from one row of a plane to the next */
    int64_t origin;        /* element offset of interior cell (0, 0) from the plane pointer */
    int64_t plane_elems;   /* elements a plane pointer must address: (ny + 1) * pitch + plane_offset */
    int64_t plane_offset;  /* elements of one plane's row: plane k of a buffer starts k * plane_offset in */
    int64_t buffer_elems;  /* elements to allocate per buffer (three interleaved planes): (ny + 2) * pitch */
    int32_t elem_bytes;    /* 4 (SW_F32) or 8 (SW_F64) */
    int32_t reserved;
} sw_layout;

/* Caller-owned device memory: two buffers (ping-pong) of three planes
 * (h, hu, hv), each a device pointer, 256-byte aligned, addressing
 * layout.plane_elems elements (placed as sw_layout describes).  buf[cur]
 * holds U^n. */
typedef struct {
    void *plane[2][3];
    int32_t cur;
    int32_t reserved;
} sw_state;

typedef struct sw_ctx sw_ctx;   /* opaque; owns device scalars (dt ring, time, flags) */

/* Layout of a plane for a grid and dtype.  Pure host computation.
 * Errors: SW_EINVAL for nx, ny < 1, nx > 2^21, ny > 2^30, an unknown dtype or a
 * NULL out. */
sw_status sw_layout_query(sw_grid grid, sw_dtype dtype, sw_layout *out);

/* Create a solver context for one grid (problem statement: grid, halo, g, dx).
 * opts may be NULL: SW_F32, reflective walls, paper scheme, dy = dx, cfl 0.5.
 * halo must be {1, 1, 1, 1} (the width the scheme needs), else SW_ENOTSUP.
 * Allocates a few hundred bytes of device memory on the current device.
 * Errors: SW_EINVAL (shape, g <= 0, dx <= 0, cfl/dt_fixed not exactly one
 * positive, unknown enum), SW_ENOTSUP, SW_ENOMEM, SW_EHIP. */
sw_status sw_create(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts, sw_ctx **out);
sw_status sw_destroy(sw_ctx *ctx);
sw_status sw_get_layout(const sw_ctx *ctx, sw_layout *out);

/* Async.  Materialise the halo of buf[cur] from its interior by the boundary
 * conditions (paper: BCs applied outside the kernel).  Interior untouched.
 * Errors: SW_EINVAL (NULL / misaligned planes, cur not 0 or 1), SW_EHIP. */
sw_status sw_fill_halo(sw_ctx *ctx, const sw_state *state, void *stream);

/* Async.  Advance buf[cur] by nsteps time steps (nsteps >= 0) on the stream
 * without any host synchronisation; then state->cur ^= (nsteps & 1).  dt is
 * recomputed on the device every step (or fixed).  On return of the work,
 * buf[cur] holds U^{n+nsteps} with its halo filled.  The halo of buf[cur] on
 * entry is ignored (it is refilled first).  A step that produces h <= 0 or a
 * non-finite value sets the context's sticky unstable flag (reported by
 * sw_sync_status); the run continues on garbage.
 * Errors (synchronous): SW_EINVAL, SW_EHIP, SW_ENOMEM (workspace of
 * variant 4 or 5), SW_ENOTSUP (a variant the options exclude). */
sw_status sw_step(sw_ctx *ctx, sw_state *state, int32_t nsteps, void *stream);

/* Synchronise the stream, then report the simulated time, the last dt and the
 * number of steps taken since sw_create / sw_reset_time.  Any output pointer
 * may be NULL.  Returns SW_EUNSTABLE if the sticky flag is set. */
sw_status sw_sync_status(sw_ctx *ctx, void *stream, double *t, double *last_dt, int64_t *steps);

/* Sync.  Diagnostics of the interior of buf[cur] (the conserved quantities
 * of section "Shallow Water Model"): out[0] = sum of h (the mass in cell
 * units), out[1] = sum of hu, out[2] = sum of hv, out[3] = max signal speed
 * max(|u|, |v|) + sqrt(g h) over the cells with finite values and h > 0,
 * out[4] = min h, out[5] = number of cells with a non-finite value.  Sums
 * in FP64 over per-block partials combined in a fixed order, so the same
 * state gives the same bits.  Reads buf[cur] only (the halo is not used);
 * `out` is host memory; synchronises the stream; allocates nothing.
 * Errors: SW_EINVAL (NULL, misaligned planes, cur not 0 or 1), SW_EHIP. */
sw_status sw_diagnostics(sw_ctx *ctx, const sw_state *state, void *stream, double out[6]);

/* Async.  Zero the simulated time and step counter and clear the sticky flag. */
sw_status sw_reset_time(sw_ctx *ctx, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  sw_step
 * without a context: validates (grid, halo, g, dx, opts) as sw_create does,
 * then advances buf[cur] of `state` by nsteps (>= 0) steps with the fused
 * kernel in sw_step's default launch shape, launched eagerly on the stream
 * (no graph), and sets state->cur ^= (nsteps & 1).  The results are bitwise
 * those of sw_create + sw_step with the default tuning.  The device scalars
 * of the step sequence (CFL ring, time, step count, sticky flag; 2 KiB,
 * whatever the grid size) live in a static array of the library, one per
 * device, held until the process ends; each call clears them first with a
 * kernel (no memset), so the time and step count cover this call only.
 * Every call on a device shares that array: calls that overlap on one device
 * (other streams, other threads) race and give wrong dt and status.
 * status: device pointer to 4 doubles (8-byte aligned) or NULL; receives
 * (simulated time, last dt, steps, 1 if a step produced h <= 0 or a
 * non-finite value else 0) of this call.  Calls no hipMalloc / hipFree.
 * Errors (synchronous, before any launch): SW_EINVAL (as sw_create and
 * sw_step, NULL / misaligned / shared planes, nsteps < 0, misaligned status),
 * SW_ENOTSUP (halo other than [1,1,1,1]; current device index >= 64), SW_EHIP. */
sw_status sw_step_noalloc(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts, sw_state *state,
                          int32_t nsteps, double *status, void *stream);

/* Kernel variant used by sw_step: 0 = auto (fastest known), 1 = one thread
 * per cell reading neighbours from global memory (baseline), 2 = fused
 * row-marching kernel (both schemes; the default for both), 3 = temporal blocking: K steps of
 * a tile and its K-cell halo per launch in LDS (paper scheme with a fixed dt
 * only; a CFL dt depends on every cell after each step; nsteps % K remaining
 * steps use the fused kernel), 4 = unfused: the first half-step writes the
 * face states to HBM and a second kernel reads them back (the array
 * temporaries of the paper's generated code), 5 = AoS: the state packed as
 * one (h, hu, hv, 0) vector per cell (the paper's hand-optimised kernel;
 * each sw_step converts the current buffer in and the result back out).
 * Variants 4 and 5 are comparison points for section "Performance
 * Measurements" of the paper (paper scheme, either dt mode); the first
 * sw_step that uses one allocates its workspace (six face planes of
 * (ny + 1) rows, or two AoS copies of a buffer), kept until
 * sw_destroy.  6 = generated: a kernel that the region-expression front
 * end emits from the step written as whole-array statements (the paper's
 * contribution, sections "Region functions" and "Source-To-Source
 * Transformations"), in one of two designs: a row march that keeps each
 * array's rows in registers and shifts x neighbours across lanes (default),
 * or the paper's own, inputs and face temporaries staged in LDS per tile
 * with one thread per cell; boundary values are filled by a separate launch
 * after each step (paper scheme, either dt mode).  Variants 2-5 give bitwise
 * identical states; the baseline and variant 6 agree with them up to
 * rounding order.
 * Errors: SW_EINVAL for an unknown variant; sw_step reports SW_ENOTSUP for a
 * variant the options exclude (also variants 3 and 6 for grids taller than
 * 65535 rows of tiles: tiles of 40-92 rows blocked, 4-16 rows generated). */
sw_status sw_set_variant(sw_ctx *ctx, int32_t variant);

/* Launch shape of the step kernel (what the autotuner searches).  Zero
 * fields mean "library default".  All fused and blocked shapes compute
 * every cell with the same arithmetic, so their results are bitwise
 * identical; the per-cell baseline agrees with them to rounding.  Blocked
 * defaults: K = 5 with 16 waves in SW_F32, with 8 waves in SW_F64. */
typedef struct {
    int32_t variant;    /* 0 auto, 1 per-cell baseline, 2 fused, 3 temporal blocking, 4 unfused, 5 AoS,
                           6 generated from region expressions */
    int32_t rows;       /* fused, AoS: rows per tile (>= 1; fused: (rows + 2) * pitch * elem_bytes < 2^31);
                           blocked: steps per launch K (3, 5; 7 in SW_F32);
                           generated: tile height 4, 8 or 16 (design 1) or rows per wave 4, 8, 16, 32 (design 2) */
    int32_t vec;        /* fused: cells per lane; SW_F32: 1, 2 or 4, SW_F64: 1 or 2; blocked: waves per tile (4, 8, 12, 16);
                           generated: design, 1 = LDS tiles (the paper's), 2 = row march in registers (default) */
    int32_t occupancy;  /* fused: register budget in waves per SIMD: 0 (compiler's choice), 3 or 4 */
    int32_t prefetch;   /* fused, generated row march: rows loaded ahead of the row being updated: 1, 2 or 3
                           (defaults: fused 2, row march 1); generated LDS tiles: 0 */
    int32_t order;      /* fused: tile order: 0 row-block-major per XCD, 1 vertically grouped per XCD, 2 plain */
} sw_tuning;

/* Errors: SW_EINVAL for a NULL argument or an unsupported combination. */
sw_status sw_set_tuning(sw_ctx *ctx, const sw_tuning *tuning);
/* The tuning sw_step will use, with defaults resolved. */
sw_status sw_get_tuning(const sw_ctx *ctx, sw_tuning *out);

/* 1 (default): sw_step replays one hipGraph per (nsteps, current buffer,
 * state planes, launch shape), captured on the first such call (kept up to 8
 * per context); 0: eager launches.  Results are identical either way. */
sw_status sw_set_graph(sw_ctx *ctx, int32_t enable);

/* Pick the fastest launch shape for this context by timing candidates on the
 * stream with the caller's state (steps_per_trial >= 1 steps each), then set
 * it.  buf[cur], its halo and the context's time/flags are saved first and
 * restored afterwards, so the simulation is left where it was.  Allocates
 * (and frees) a temporary copy of one buffer of device memory.  With a
 * fixed dt the blocked kernel is among the candidates.  If cache_path is
 * non-NULL, a cached choice for the same (GPU, dtype, scheme, grid, fixed or
 * CFL dt) is used without timing, and new choices are appended there.
 * best may be NULL.  Synchronises the stream.
 * Errors: SW_EINVAL, SW_ENOMEM, SW_EHIP, SW_ENOTSUP (no candidate ran). */
sw_status sw_autotune(sw_ctx *ctx, sw_state *state, int32_t steps_per_trial, const char *cache_path, void *stream,
                      sw_tuning *best);

/* ---------------------------------------------------------------------------
 * Batched mode: n independent grids of possibly different sizes (same g, dx,
 * options and scheme, either scheme), all advanced together.  Each grid
 * keeps its own CFL dt, simulated time and sticky flag; a grid advanced in a
 * batch is bitwise identical to the same grid advanced alone with the same
 * launch shape.  One kernel launch per time step covers every grid (a tile
 * table over all grids; two launches per step, one per chain of grids, for
 * batches of 4 M cells or more); sw_batch_step replays the whole call as
 * hipGraph launches (captured on first use per (nsteps, buffer, tuning)).
 * The caller owns the arena (device memory); the library owns the tile
 * table, per-grid scalars, graphs, a capture stream and the second chain's
 * stream and events. */
typedef struct sw_batch sw_batch;

/* Validates every grid like sw_create (no HIP call until then), then
 * allocates the per-grid scalars.  Errors: SW_EINVAL, SW_ENOTSUP (halo),
 * SW_ENOMEM, SW_EHIP. */
sw_status sw_batch_create(int32_t n, const sw_grid *grids, sw_halo halo, double g, double dx, const sw_opts *opts,
                          sw_batch **out);
sw_status sw_batch_destroy(sw_batch *batch);
/* Bytes of device memory the caller allocates for the arena. */
sw_status sw_batch_arena_bytes(const sw_batch *batch, size_t *bytes);
/* Attach a 256-byte aligned device arena of sw_batch_arena_bytes bytes.
 * Resets the current buffer to 0.  Errors: SW_EINVAL, SW_EHIP. */
sw_status sw_batch_bind(sw_batch *batch, void *arena);
/* Grid i's planes inside the arena, as an sw_state (cur = the batch's
 * current buffer) plus its layout (may be NULL): for writing initial states
 * and reading results. */
sw_status sw_batch_view(const sw_batch *batch, int32_t i, sw_state *view, sw_layout *layout);
/* Async: materialise every grid's halo of the current buffer. */
sw_status sw_batch_fill_halo(sw_batch *batch, void *stream);
/* Async: advance every grid by nsteps (>= 0); the current buffer flips
 * when nsteps is odd.  A batch of 4 M cells or more per step advances as
 * two chains of grids, the second on a stream the batch owns (default
 * priority), forked from `stream` after the call's first launches and joined
 * back into it at the end: work enqueued on `stream` afterwards sees the
 * whole call, as with one chain.  Errors (synchronous): SW_EINVAL, SW_EHIP. */
sw_status sw_batch_step(sw_batch *batch, int32_t nsteps, void *stream);
/* Synchronise, then per grid (arrays of n entries, each may be NULL): time,
 * steps and the sticky flag.  Returns SW_EUNSTABLE if any grid is flagged. */
sw_status sw_batch_sync_status(sw_batch *batch, void *stream, double *t, int64_t *steps, int32_t *unstable);
sw_status sw_batch_reset_time(sw_batch *batch, void *stream);
/* Async, for batches whose grids all have the same size: copy every grid's
 * interior of the current buffer to (export) or from (import) one dense
 * device array [n][3][ny][nx] of the batch's dtype.  Import leaves the halos
 * stale; sw_batch_step refills them.  Errors: SW_EINVAL (sizes differ, NULL). */
sw_status sw_batch_export(sw_batch *batch, void *dense, void *stream);
sw_status sw_batch_import(sw_batch *batch, const void *dense, void *stream);
/* Launch shape for every grid (variant must be 0 or 2; order: 0 = LPT
 * tile table, largest grids first, one wave per tile; 1 = round-robin over
 * grids, one wave per tile; 2 = the LPT table walked by persistent waves,
 * only the workgroups the device holds at once, each wave taking a
 * contiguous run of tiles).  Every shape gives bitwise the same states. */
sw_status sw_batch_set_tuning(sw_batch *batch, const sw_tuning *tuning);
sw_status sw_batch_get_tuning(const sw_batch *batch, sw_tuning *out);
/* 1 (default): one hipGraph launch per sw_batch_step call; 0: eager launches. */
sw_status sw_batch_set_graph(sw_batch *batch, int32_t enable);
/* Like sw_autotune over the batch (saves/restores the current buffer and
 * the per-grid scalars; allocates a temporary copy of one buffer region). */
sw_status sw_batch_autotune(sw_batch *batch, int32_t steps_per_trial, const char *cache_path, void *stream,
                            sw_tuning *best);

/* ---------------------------------------------------------------------------
 * Learned surrogate (not part of the paper): a residual network that maps
 * U^n to U^{n+jump} on H x W grids, jumping `jump` solver steps at a time:
 *   x = normalise(U^n)  (channel c: (u_c - in_offset_c) / in_scale_c; the
 *       input's one-cell halo holds the boundary ghosts);
 *   A1 = relu(conv1(x)), A_l = A_{l-1} + relu(conv_l(A_{l-1})) for l = 2..5,
 *   delta = conv6(A5): 3x3 "same" convolutions with bias, 3 -> 32 -> 32 ->
 *       32 -> 32 -> 32 -> 3 channels, zero padding in the hidden layers,
 *       BF16 weights and activations, FP32 accumulation;
 *   U^{n+jump} = U^n + delta * out_scale   (residual added in FP32).
 * Parameters: one FP32 master vector (device), layer after layer: weights
 * W[co][tap][ci] (tap = 3 * ky + kx, cross-correlation) then biases b[co];
 * 38 755 values.  Training (sw_surrogate_train_step) minimises the mean
 * squared error of the normalised delta with Adam (beta 0.9 / 0.999, eps
 * 1e-8), gradients by the library's own backward kernels. */
typedef struct {
    int32_t layers;      /* must be 6 */
    int32_t hidden;      /* must be 32 */
    int32_t jump;        /* solver steps replaced by one network application (even, e.g. 8) */
    int32_t bc_x, bc_y;  /* sw_bc of the input ghosts (must match the batch it advances) */
    int32_t reserved;
    uint64_t seed;       /* weight initialisation (He-normal; output layer x 0.1) */
} sw_net_cfg;

/* Gate of a surrogate jump, per grid: the jump is rejected, and the plain
 * solver takes it instead, if |M' - M| / M > mass_rel_tol (M = sum of h),
 * if any depth <= hmin, or if any value is non-finite.  project_mass != 0
 * first removes the mean of the predicted dh, so mass is kept exactly.
 * judge != 0 also runs the plain solver over the whole span from the same
 * start (on a copy the network keeps) and compares: a grid whose relative
 * L2 error of h, ||h - h_solver||_2 / ||h_solver||_2 over the interior,
 * exceeds l2_tol takes the solver's result. */
typedef struct {
    double mass_rel_tol;
    double hmin;
    int32_t project_mass;
    int32_t judge;
    double l2_tol;
} sw_gate;

typedef struct sw_net sw_net;

/* Network for H x W grids (W a multiple of 64), up to max_batch grids per
 * call; allocates its weights and activation / gradient workspace (about
 * 14 * 64 * max_batch * (H + 2) * (W + 2) bytes, e.g. 15 GB for 256 grids of
 * 256 x 256).
 * Errors: SW_EINVAL, SW_ENOTSUP (other depth / width), SW_ENOMEM, SW_EHIP. */
sw_status sw_surrogate_create(const sw_net_cfg *cfg, int32_t H, int32_t W, int32_t max_batch, sw_net **out);
sw_status sw_surrogate_destroy(sw_net *net);
/* Device pointer to the FP32 master parameters and their count.  After
 * writing them (e.g. loading saved weights) call sw_surrogate_sync_weights. */
sw_status sw_surrogate_params(sw_net *net, float **master_dev, int64_t *count);
sw_status sw_surrogate_sync_weights(sw_net *net, void *stream);
/* Host arrays of 3 floats each; scales must be > 0. */
sw_status sw_surrogate_set_norm(sw_net *net, const float in_offset[3], const float in_scale[3],
                                const float out_scale[3]);
/* Async.  u: device FP32 frames [B][3][H][W] (h, hu, hv); delta (device, may
 * be NULL): the normalised prediction as FP32 [B][H][W][4] (4th channel 0). */
sw_status sw_surrogate_forward(sw_net *net, const float *u, int32_t B, float *delta, void *stream);
/* Device pointer to the last forward pass's activations: layer 0 = network
 * input (BF16 NHWC, 8 channels, with halo), 1..5 = hidden layers (BF16 NHWC,
 * 32 channels, with halo), 6 = delta (FP32 [B][H][W][4]).  A rollout's
 * first layer reads the batch's planes directly and leaves layer 0 as the
 * last sw_surrogate_forward / grad / train_step wrote it. */
sw_status sw_surrogate_activation(sw_net *net, int32_t layer, const void **ptr, int64_t *bytes);
/* Async.  Loss (device float, may be NULL) and gradient (device, nparams
 * floats, may be NULL) of the pair (u -> u8), without updating. */
sw_status sw_surrogate_grad(sw_net *net, const float *u, const float *u8, int32_t B, float *grad, float *loss,
                            void *stream);
/* Async.  One Adam step on the pair (u -> u8) with learning rate lr. */
sw_status sw_surrogate_train_step(sw_net *net, const float *u, const float *u8, int32_t B, float lr, float *loss,
                                  void *stream);
/* Async.  Advance every grid of an FP32 batch (all H x W, same boundary
 * conditions) by nsteps (a multiple of jump) in jumps; each jump is gated per
 * grid and rejected grids take jump solver steps instead.  fallbacks (device
 * int32[n], may be NULL) is incremented per rejected jump.  The batch's
 * per-grid time and step counters count only the solver steps taken (a
 * network jump has no time step).  Judge mode (gate->judge): l2 (device
 * double[n], may be NULL) receives each grid's relative L2(h) against the
 * plain solver; a grid above gate->l2_tol takes the solver's state, time,
 * step count and unstable flag, and its fallbacks entry is set to nsteps / jump.  The first
 * judged call on a batch allocates the solver's copy (about the batch's arena
 * size), kept until the network is destroyed or judges another batch.
 * Without the judge, the rollout is captured once into a hipGraph per
 * (batch, its tuning and binding, current buffer, nsteps, gate, fallbacks)
 * and replayed on later calls (kept up to 8 per network; sw_surrogate_set_norm
 * drops them); the judged rollout is launched eagerly.  No host sync. */
sw_status sw_surrogate_advance(sw_net *net, sw_batch *solver, int32_t nsteps, const sw_gate *gate,
                               int32_t *fallbacks, double *l2, void *stream);
/* 1 (default): unjudged rollouts replay captured graphs; 0: eager launches.
 * Results are identical either way.  Errors: SW_EINVAL for a NULL network. */
sw_status sw_surrogate_set_graph(sw_net *net, int32_t enable);
/* Upper bound on the workgroups of the persistent convolution and
 * weight-gradient kernels (each walks a contiguous run of tiles); 0 (the
 * default) launches one workgroup per slot the device holds at once.  A
 * smaller cap only changes how the tiles are split among workgroups: the
 * convolution outputs are bitwise unchanged, the weight gradient's FP32 block
 * partials (summed in FP64) split differently.  Drops captured rollouts.
 * Errors: SW_EINVAL for a NULL network or a cap outside [0, 1024]. */
sw_status sw_surrogate_set_block_cap(sw_net *net, int32_t max_blocks);

/* Form of the rollout's network pass.  1: one launch runs all six layers
 * per output tile with the activations on chip (the state with a 6-pixel
 * border in, the prediction out), and the gate's verdict and the rejected
 * grids' solver steps share one launch: three launches per jump.  0: one
 * launch per layer through activation tensors in device memory, then
 * separate gate and fallback launches.  2 (default): 1 while the batch has
 * at most 2 output tiles of 16 x 32 pixels per compute unit, else 0 (the
 * fused form recomputes each tile's border and wins where launches and HBM
 * traffic dominate, i.e. at small batches).  The predictions are bitwise
 * equal; with project_mass the mean of the predicted dh is summed in a
 * different fixed order (per tile instead of per row segment), so h may
 * differ in the last bits.  Drops captured rollouts.
 * Errors: SW_EINVAL for a NULL network or a mode outside 0..2. */
sw_status sw_surrogate_set_fused(sw_net *net, int32_t mode);

const char *sw_strerror(sw_status status);
const char *sw_last_error_detail(void);

#ifdef __cplusplus
}
#endif
#endif /* SW_H */
