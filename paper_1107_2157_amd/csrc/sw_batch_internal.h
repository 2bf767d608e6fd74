// Internal interface of the batched step (host <-> kernels).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "sw_internal.h"

// Words each CFL ring slot of a batched grid is striped over: one per lane of
// a wave, so that the tiles of a large grid rarely meet on one atomic word.
constexpr int kBatchStripes = 64;

// Per-grid device scalars (CFL ring slots striped over kBatchStripes words,
// time, flag).
struct SwBatchScalars {
    unsigned long long smax[3][kBatchStripes];
    double t;
    double last_dt;
    long long steps;
    unsigned int unstable;
    unsigned int pad;
};

// Per-grid descriptor: plane pointers at interior cell (0, 0) of both buffers.
struct SwBatchGrid {
    const void *plane[2][3];
    int64_t pitch;
    int32_t nx, ny;
};

// One tile of the table: grid, strip, row block.
struct SwBatchTile {
    int32_t grid;
    int32_t s;
    int32_t rb;
    int32_t pad;
};

struct SwBatchLaunch {
    const SwBatchTile *tiles;
    const SwBatchGrid *grids;
    SwBatchScalars *sc;
    int32_t ntiles;
    int32_t cur;      // buffer holding U^n for every grid
    int32_t step;     // ring position
    int32_t rows;     // rows per tile
    double g, dx, dy, cfl, dt_fixed;
    int32_t bc_x, bc_y, dtype, scheme;   // scheme: 0 paper, 1 transverse
    const int32_t *active;   // optional per-grid mask: grids with 0 are skipped entirely
    int32_t ghosts;          // 0: the step leaves the ghost cells unwritten (TileArgs::ghosts)
};

// Gate statistics of a surrogate jump, per grid: mass before and after, the
// least depth, whether any value is non-finite, and the verdict.
struct SwGateStats {
    double mass_old, mass_new;
    float hmin;
    unsigned int nonfinite;
    int fallback;
    int pad;
};
// The gate's rule: reject a jump on mass drift above mass_tol, a depth at or
// below hmin, or a non-finite value.
struct SwFallbackGate {
    SwGateStats *stats;
    double mass_tol, hmin;
    int32_t *fallbacks;   // per-grid count of rejected jumps (may be null)
};

hipError_t sw_batch_launch_reset(SwBatchScalars *sc, int n, int clear_time, hipStream_t s);
hipError_t sw_batch_launch_prologue(const SwBatchLaunch &a, int vec, hipStream_t s);
// persistent = 0: one wave per tile of the table.  persistent = 1: resident
// workgroups only, each wave walking a contiguous run of the table (runs of
// one XCD contiguous); the same cells, dt and bookkeeping.
hipError_t sw_batch_launch_step(const SwBatchLaunch &a, int vec, int minw, int pd, int persistent, hipStream_t s);
// FP32 only: prologue and nsteps steps of every grid g < ngrids with
// a.active[g] != 0, one workgroup per grid, one launch (the other grids
// return at once).  Bitwise the same as reset-free prologue + nsteps step
// launches of those grids.
hipError_t sw_batch_launch_fallback(const SwBatchLaunch &a, int ngrids, int nsteps, hipStream_t s);
// The same with the gate folded in: each grid's workgroup takes the verdict
// from the jump's statistics (recording it in stats[g].fallback and
// fallbacks[g]); an accepted grid returns at once, a rejected one copies
// U^n (buffer cur ^ 1, halos included) over the prediction in buffer cur and
// takes its nsteps steps from there.  Bitwise the gate-and-restore pass
// followed by sw_batch_launch_fallback with the verdicts as the mask.
hipError_t sw_batch_launch_gated_fallback(const SwBatchLaunch &a, const SwFallbackGate &gate, int ngrids, int nsteps,
                                          hipStream_t s);
hipError_t sw_batch_launch_copy(const SwBatchGrid *grids, int cur, int n, int nx, int ny, int dtype, void *dense,
                                int to_dense, hipStream_t s);

// Host-side hooks of the batch object for the surrogate (sw_batch.cpp).
struct sw_batch;
struct SwBatchInfo {
    const SwBatchGrid *d_grids;
    SwBatchScalars *d_sc;
    int n, cur, dtype, bc_x, bc_y;
    int same_nx, same_ny;          // common grid size, or -1 if sizes differ
    uint64_t gen;                  // changes whenever the batch's launch arguments do
};
int sw_batch_internal_info(const sw_batch *b, SwBatchInfo *info);   // returns sw_status
// Resolve the tuning and build the tile table now (it allocates and copies
// synchronously), so that later enqueues only launch kernels.
int sw_batch_internal_prepare(sw_batch *b);
// Eager, one launch: prologue and nsteps steps for the grids with
// active[g] != 0 (device array), starting from the current buffer; the other
// grids are left alone.  FP32 batches.  Does not flip the batch's current
// buffer (nsteps must be even).
int sw_batch_internal_fallback(sw_batch *b, int nsteps, const int32_t *active, hipStream_t s);
// The gated form (sw_batch_launch_gated_fallback) on the batch's current
// buffer, which holds the prediction; U^n is in the other one.
int sw_batch_internal_gated_fallback(sw_batch *b, int nsteps, const SwFallbackGate &gate, hipStream_t s);
// A batch with the same grids, options and tuning as src, bound to an arena
// it allocates (*arena; the caller frees it after sw_batch_destroy).
int sw_batch_internal_clone(const sw_batch *src, sw_batch **out, void **arena);
// Whether a and b hold the same grids with the same options (a clone's test).
bool sw_batch_internal_compatible(const sw_batch *a, const sw_batch *b);
// dst := src's current buffer (whole region, halos included) and current-buffer
// index, with dst's time and step counters cleared.  Compatible batches only.
int sw_batch_internal_copy_state(sw_batch *dst, const sw_batch *src, hipStream_t s);
// Make buffer cur (0 or 1) the batch's current buffer (its contents must
// already hold the state, halos included).
int sw_batch_internal_set_cur(sw_batch *b, int cur);
