// Batched step kernels: many independent grids of uneven sizes advance one
// time step per launch.  A device tile table lists (grid, strip, row block)
// for every grid; each wave takes one tile, reads the tile's grid descriptor
// and that grid's dt, and runs the same per-tile body as the single-grid
// kernel (sw_tile.h), so a grid advanced in a batch is bitwise identical to
// the same grid advanced alone.  Each grid keeps its own CFL ring slots,
// time and sticky flag.
#include <algorithm>

#include "sw_batch_internal.h"
#include "sw_tile_tr.h"

using namespace sw;
using namespace sw::tile;

namespace {

// A slot is read by one wave (a stripe per lane) and indexed with a mask.
static_assert(kBatchStripes <= 64 && (kBatchStripes & (kBatchStripes - 1)) == 0, "stripes: power of two, at most 64");

// dt of grid `grid` for step `step` (wave-wide).
// The grid's dt in two halves (its ring stripe, a load; then the wave max
// and the division), so that the step kernel issues its first row loads in
// between.
__device__ __forceinline__ double batch_dt_stripe(const SwBatchLaunch &a, int grid) {
    if (a.dt_fixed > 0) return 0.0;
    const int lane = threadIdx.x & 63;
    return lane < kBatchStripes ? __longlong_as_double((long long)a.sc[grid].smax[a.step % 3][lane]) : 0.0;
}
__device__ __forceinline__ double batch_dt_finish(const SwBatchLaunch &a, double v) {
    if (a.dt_fixed > 0) return a.dt_fixed;
    return a.cfl * fmin(a.dx, a.dy) / wave_max(v);
}

// Wave-wide: this wave's tile, XCD-aware (block b runs on XCD b % 8; every
// XCD takes a contiguous run of the tile table).
__device__ __forceinline__ int batch_tile_index() {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per_xcd = gridDim.x >> 3;
    return ((((int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3)) << 2) + wave);
}

__device__ __forceinline__ void batch_reduce(const SwBatchLaunch &a, int grid, int slot, int stripe, double smax,
                                             bool bad) {
    smax = wave_max(smax);
    unsigned long long anybad = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&a.sc[grid].smax[slot][stripe & (kBatchStripes - 1)], (unsigned long long)__double_as_longlong(smax));
        if (anybad) atomicOr(&a.sc[grid].unstable, 1u);
    }
}

template <typename T, int VEC, int MINW, int PD, bool TR>
__global__ __launch_bounds__(256, (MINW > 0 ? MINW : 1)) void k_batch_step(SwBatchLaunch a) {
    const int tile = batch_tile_index();
    if (tile >= a.ntiles) return;                 // whole wave leaves: no barriers are used
    const SwBatchTile tt = a.tiles[tile];
    if (a.active && !a.active[tt.grid]) return;
    const SwBatchGrid &gd = a.grids[tt.grid];
    const double stripe = batch_dt_stripe(a, tt.grid);
    TileArgs t;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        t.in[k] = gd.plane[a.cur][k];
        t.out[k] = const_cast<void *>(gd.plane[a.cur ^ 1][k]);
    }
    t.pitch = gd.pitch;
    t.nx = gd.nx;
    t.ny = gd.ny;
    t.bc_x = a.bc_x;
    t.bc_y = a.bc_y;
    t.s = tt.s;
    t.rb = tt.rb;
    t.rows = a.rows;
    t.ghosts = a.ghosts;
    T smax = T(0);
    bool bad = false;
    double dt = 0.0;
    if constexpr (TR)
        fused_tile_tr<T, VEC, PD>(t, [&] { return batch_dt_finish(a, stripe); }, a.g, a.dx, a.dy, smax, bad, dt);
    else
        fused_tile<T, VEC, PD>(t, [&] { return batch_dt_finish(a, stripe); }, a.g, a.dx, a.dy, smax, bad, dt);
    batch_reduce(a, tt.grid, (a.step + 1) % 3, tile, (double)smax, bad);
    if (tt.s == 0 && tt.rb == 0) {               // the grid's first tile keeps its books
        const int lane = threadIdx.x & 63;
        if (lane < kBatchStripes) atomicExch(&a.sc[tt.grid].smax[(a.step + 2) % 3][lane], 0ull);
        if (lane == 0) {
            a.sc[tt.grid].t += dt;
            a.sc[tt.grid].last_dt = dt;
            a.sc[tt.grid].steps += 1;
        }
    }
}

// Persistent form of the step: only resident workgroups are launched and
// each wave walks a contiguous run of the tile table (tiles_per_wave
// entries; the runs of one XCD's waves are contiguous, so a grid's
// neighbouring tiles meet in that XCD's L2).  The next tile's table entry is
// loaded while the current tile runs, the grid's dt is kept while the run
// stays on one grid, and the signal-speed max of consecutive tiles of one
// grid is flushed once per grid.  Every cell, dt and book entry is the one
// k_batch_step computes.
template <typename T, int VEC, int MINW, int PD, bool TR>
__global__ __launch_bounds__(256, (MINW > 0 ? MINW : 1)) void k_batch_step_pers(SwBatchLaunch a, int tiles_per_wave) {
    const int w = batch_tile_index();            // this wave's position among all waves, XCD-aware
    const int t0 = w * tiles_per_wave;
    const int t1 = min(a.ntiles, t0 + tiles_per_wave);
    if (t0 >= t1) return;                         // whole wave leaves: no barriers are used
    SwBatchTile nxt = a.tiles[t0];
    int cur_grid = -1;
    double dt_grid = 0.0;
    T smax = T(0);
    bool bad = false;
    for (int t = t0; t < t1; ++t) {
        const SwBatchTile tt = nxt;
        if (t + 1 < t1) nxt = a.tiles[t + 1];     // in flight during this tile
        if (tt.grid != cur_grid) {                 // a new grid: flush the previous one's max, take this one's dt
            if (cur_grid >= 0) batch_reduce(a, cur_grid, (a.step + 1) % 3, w, (double)smax, bad);
            smax = T(0);
            bad = false;
            cur_grid = tt.grid;
            dt_grid = batch_dt_finish(a, batch_dt_stripe(a, cur_grid));
        }
        if (a.active && !a.active[tt.grid]) continue;
        const SwBatchGrid &gd = a.grids[tt.grid];
        TileArgs ta;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            ta.in[k] = gd.plane[a.cur][k];
            ta.out[k] = const_cast<void *>(gd.plane[a.cur ^ 1][k]);
        }
        ta.pitch = gd.pitch;
        ta.nx = gd.nx;
        ta.ny = gd.ny;
        ta.bc_x = a.bc_x;
        ta.bc_y = a.bc_y;
        ta.s = tt.s;
        ta.rb = tt.rb;
        ta.rows = a.rows;
        ta.ghosts = a.ghosts;
        double dt = 0.0;
        const double dtg = dt_grid;
        if constexpr (TR)
            fused_tile_tr<T, VEC, PD>(ta, [&] { return dtg; }, a.g, a.dx, a.dy, smax, bad, dt);
        else
            fused_tile<T, VEC, PD>(ta, [&] { return dtg; }, a.g, a.dx, a.dy, smax, bad, dt);
        if (tt.s == 0 && tt.rb == 0) {           // the grid's first tile keeps its books
            const int lane = threadIdx.x & 63;
            if (lane < kBatchStripes) atomicExch(&a.sc[tt.grid].smax[(a.step + 2) % 3][lane], 0ull);
            if (lane == 0) {
                a.sc[tt.grid].t += dt;
                a.sc[tt.grid].last_dt = dt;
                a.sc[tt.grid].steps += 1;
            }
        }
    }
    if (cur_grid >= 0) batch_reduce(a, cur_grid, (a.step + 1) % 3, w, (double)smax, bad);
}

// Once per call: ghosts of U^cur for every grid and the max signal speed
// into ring slot 0.  One wave per tile, lanes across the tile's columns.
template <typename T>
__global__ __launch_bounds__(256) void k_batch_prologue(SwBatchLaunch a, int tile_cols) {
    const int tile = batch_tile_index();
    if (tile >= a.ntiles) return;
    const SwBatchTile tt = a.tiles[tile];
    if (a.active && !a.active[tt.grid]) return;
    const SwBatchGrid &gd = a.grids[tt.grid];
    const int lane = threadIdx.x & 63;
    T *P[3] = {(T *)gd.plane[a.cur][0], (T *)gd.plane[a.cur][1], (T *)gd.plane[a.cur][2]};
    const T g = (T)a.g;
    const int j0 = tt.rb * a.rows, j1 = min(j0 + a.rows, gd.ny);
    const int c0 = tt.s * tile_cols, c1 = min(c0 + tile_cols, gd.nx);
    double smax = 0.0;
    bool bad = false;
    for (int j = j0; j < j1; ++j)
        for (int i = c0 + lane; i < c1; i += 64) {
            const int64_t off = (int64_t)j * gd.pitch + i;
            U3<T> c = {P[0][off], P[1][off], P[2][off]};
            T sp = signal_speed(c, g);
            bad |= !(sp <= finite_max<T>());
            smax = fmax(smax, (double)sp);
            if (i == 0 || i == gd.nx - 1 || j == 0 || j == gd.ny - 1)
                write_ghosts(P, gd.pitch, gd.nx, gd.ny, a.bc_x, a.bc_y, i, j, c);
        }
    batch_reduce(a, tt.grid, 0, tile, smax, bad);
}

// The masked fallback of the surrogate's rollout in one launch: one
// workgroup per grid, all of that grid's steps.  A grid whose active entry is
// 0 leaves at once, so a jump the gate accepts everywhere costs one launch.
// A rejected grid takes the prologue (ghosts and max signal speed of buffer
// cur) and then nsteps steps of the fused tile body, the workgroup's waves
// walking its tiles; each step's max speed is reduced in LDS, and its writes
// reach the next step's loads through an agent-scope release before the
// barrier and an acquire after it (the acquire drops the CU's vector cache,
// which may hold lines of the buffer from two steps earlier).  Every cell is
// computed as in k_batch_step and every dt from the same max, so the grid
// ends bitwise where a prologue and nsteps launches of k_batch_step leave
// it, with the same time and step count.
constexpr int kFbWaves = 8;

// GATED: the surrogate gate's verdict is taken here instead of from a mask:
// from the jump's statistics (the same rule and expression as the
// gate-and-restore pass), recorded by thread 0; a rejected grid first copies
// U^n from buffer cur ^ 1 over the prediction in buffer cur (the whole halo'd
// rectangle) and makes the copy visible to the workgroup as above.
template <typename T, int VEC, int PD, bool TR, bool GATED>
__global__ __launch_bounds__(64 * kFbWaves) void k_batch_fallback(SwBatchLaunch a, SwFallbackGate gate, int nsteps) {
    const int gi = blockIdx.x;
    const SwBatchGrid &gd = a.grids[gi];
    if constexpr (GATED) {
        const SwGateStats &sg = gate.stats[gi];
        const double drift = fabs(sg.mass_new - sg.mass_old) / fabs(sg.mass_old);
        const int reject = !(drift <= gate.mass_tol) || !((double)sg.hmin > gate.hmin) || sg.nonfinite != 0u;
        __syncthreads();                        // every thread has read the statistics before thread 0 writes
        if (threadIdx.x == 0) {
            gate.stats[gi].fallback = reject;
            if (gate.fallbacks) gate.fallbacks[gi] += reject;
        }
        if (!reject) return;                    // uniform: the whole workgroup leaves
        const int64_t n = (int64_t)(gd.ny + 2) * (gd.nx + 2);
        for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
            const int yy = (int)(p / (gd.nx + 2)), xx = (int)(p - (int64_t)yy * (gd.nx + 2));
            const int64_t off = (int64_t)(yy - 1) * gd.pitch + (xx - 1);
#pragma unroll
            for (int k = 0; k < 3; ++k) ((T *)gd.plane[a.cur][k])[off] = ((const T *)gd.plane[a.cur ^ 1][k])[off];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    } else {
        if (!a.active[gi]) return;              // uniform: the whole workgroup leaves
    }
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    __shared__ double s_max[kFbWaves];
    __shared__ unsigned s_bad[kFbWaves];
    __shared__ double s_dt;
    const T g = (T)a.g;
    const int nx = gd.nx, ny = gd.ny;
    int cur = a.cur;

    // the grid's max speed over the workgroup; thread 0 turns it into the
    // next dt and raises the flag; every thread sees s_dt after the barrier
    auto finish = [&](double smax, bool bad) {
        smax = wave_max(smax);
        const unsigned long long anybad = __ballot(bad);
        if (lane == 0) {
            s_max[wave] = smax;
            s_bad[wave] = anybad != 0ull;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            double m = 0.0;
            unsigned b = 0u;
            for (int w = 0; w < kFbWaves; ++w) {
                m = fmax(m, s_max[w]);
                b |= s_bad[w];
            }
            if (b) atomicOr(&a.sc[gi].unstable, 1u);
            s_dt = a.dt_fixed > 0 ? a.dt_fixed : a.cfl * fmin(a.dx, a.dy) / m;
        }
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    };

    {   // prologue: ghosts of U^cur and its max speed
        T *P[3] = {(T *)gd.plane[cur][0], (T *)gd.plane[cur][1], (T *)gd.plane[cur][2]};
        double smax = 0.0;
        bool bad = false;
        const int64_t n = (int64_t)nx * ny;
        for (int64_t c = threadIdx.x; c < n; c += blockDim.x) {
            const int j = (int)(c / nx), i = (int)(c - (int64_t)j * nx);
            const int64_t off = (int64_t)j * gd.pitch + i;
            U3<T> u = {P[0][off], P[1][off], P[2][off]};
            T sp = signal_speed(u, g);
            bad |= !(sp <= finite_max<T>());
            smax = fmax(smax, (double)sp);
            if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1)
                write_ghosts(P, gd.pitch, nx, ny, a.bc_x, a.bc_y, i, j, u);
        }
        finish(smax, bad);
    }
    constexpr int W = 64 * VEC;
    const int nstrips = (nx + W - 1) / W, nrb = (ny + a.rows - 1) / a.rows;
    for (int k = 0; k < nsteps; ++k) {
        const double dt = s_dt;
        TileArgs t;
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
            t.in[kk] = gd.plane[cur][kk];
            t.out[kk] = const_cast<void *>(gd.plane[cur ^ 1][kk]);
        }
        t.pitch = gd.pitch;
        t.nx = nx;
        t.ny = ny;
        t.bc_x = a.bc_x;
        t.bc_y = a.bc_y;
        t.rows = a.rows;
        T smax = T(0);
        bool bad = false;
        for (int tile = wave; tile < nstrips * nrb; tile += kFbWaves) {
            t.s = tile % nstrips;
            t.rb = tile / nstrips;
            double dt_used = 0.0;
            if constexpr (TR)
                fused_tile_tr<T, VEC, PD>(t, [&] { return dt; }, a.g, a.dx, a.dy, smax, bad, dt_used);
            else
                fused_tile<T, VEC, PD>(t, [&] { return dt; }, a.g, a.dx, a.dy, smax, bad, dt_used);
        }
        if (threadIdx.x == 0) {
            a.sc[gi].t += dt;
            a.sc[gi].last_dt = dt;
            a.sc[gi].steps += 1;
        }
        finish((double)smax, bad);
        cur ^= 1;
    }
}

__global__ void k_batch_reset(SwBatchScalars *sc, int n, int clear_time) {
    const int gi = blockIdx.x;
    if (gi >= n) return;
    for (int k = threadIdx.x; k < 3 * kBatchStripes; k += blockDim.x)
        sc[gi].smax[k / kBatchStripes][k % kBatchStripes] = 0ull;
    if (clear_time && threadIdx.x == 0) {
        sc[gi].t = 0.0;
        sc[gi].last_dt = 0.0;
        sc[gi].steps = 0;
        sc[gi].unstable = 0u;
    }
}

// Dense [n][3][ny][nx] <-> every grid's interior in buffer `cur`.
template <typename T, bool EXPORT>
__global__ __launch_bounds__(256) void k_batch_copy(const SwBatchGrid *grids, int cur, int n, int nx, int ny, T *dense) {
    const int64_t per = (int64_t)3 * ny * nx;
    const int64_t total = per * n;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int g = (int)(i / per);
        int64_t r = i - (int64_t)g * per;
        const int k = (int)(r / ((int64_t)ny * nx));
        r -= (int64_t)k * ny * nx;
        const int y = (int)(r / nx), x = (int)(r - (int64_t)y * nx);
        T *p = (T *)grids[g].plane[cur][k] + (int64_t)y * grids[g].pitch + x;
        if (EXPORT) dense[i] = *p;
        else *p = dense[i];
    }
}

unsigned batch_blocks(int ntiles) {
    int64_t blocks = ((int64_t)ntiles + 3) / 4;
    return (unsigned)((blocks + 7) / 8 * 8);
}

template <typename T, int VEC, int MINW, int PD, bool TR>
hipError_t launch_batch_t(const SwBatchLaunch &a, int persistent, hipStream_t s) {
    if (!persistent) {
        k_batch_step<T, VEC, MINW, PD, TR><<<batch_blocks(a.ntiles), 256, 0, s>>>(a);
        return hipGetLastError();
    }
    static const int resident = [] {   // workgroups of this instance that fit on one CU at once
        int r = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_batch_step_pers<T, VEC, MINW, PD, TR>, 256, 0) ==
                               hipSuccess &&
                       r > 0
                   ? r
                   : 1;
    }();
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    int64_t blocks = (int64_t)cus * resident;
    blocks = std::min<int64_t>(blocks, ((int64_t)a.ntiles + 3) / 4);
    blocks = (blocks + 7) / 8 * 8;
    const int64_t waves = blocks * 4;
    const int per_wave = (int)((a.ntiles + waves - 1) / waves);
    k_batch_step_pers<T, VEC, MINW, PD, TR><<<(unsigned)blocks, 256, 0, s>>>(a, per_wave);
    return hipGetLastError();
}

}  // namespace

hipError_t sw_batch_launch_copy(const SwBatchGrid *grids, int cur, int n, int nx, int ny, int dtype, void *dense,
                                int to_dense, hipStream_t s) {
    int64_t blocks = ((int64_t)3 * n * nx * ny + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (dtype) {
        if (to_dense) k_batch_copy<double, true><<<(unsigned)blocks, 256, 0, s>>>(grids, cur, n, nx, ny, (double *)dense);
        else k_batch_copy<double, false><<<(unsigned)blocks, 256, 0, s>>>(grids, cur, n, nx, ny, (double *)dense);
    } else {
        if (to_dense) k_batch_copy<float, true><<<(unsigned)blocks, 256, 0, s>>>(grids, cur, n, nx, ny, (float *)dense);
        else k_batch_copy<float, false><<<(unsigned)blocks, 256, 0, s>>>(grids, cur, n, nx, ny, (float *)dense);
    }
    return hipGetLastError();
}

hipError_t sw_batch_launch_reset(SwBatchScalars *sc, int n, int clear_time, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_batch_reset<<<n, 64, 0, s>>>(sc, n, clear_time);
    return hipGetLastError();
}

hipError_t sw_batch_launch_prologue(const SwBatchLaunch &a, int vec, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
    if (a.dtype) k_batch_prologue<double><<<batch_blocks(a.ntiles), 256, 0, s>>>(a, 64 * vec);
    else k_batch_prologue<float><<<batch_blocks(a.ntiles), 256, 0, s>>>(a, 64 * vec);
    return hipGetLastError();
}

hipError_t sw_batch_launch_fallback(const SwBatchLaunch &a, int ngrids, int nsteps, hipStream_t s) {
    if (ngrids <= 0 || nsteps <= 0) return hipSuccess;
    if (a.dtype != 0 || !a.active || a.rows < 1) return hipErrorInvalidValue;
    const SwFallbackGate none{};
    if (a.scheme == 0) k_batch_fallback<float, 2, 1, false, false><<<ngrids, 64 * kFbWaves, 0, s>>>(a, none, nsteps);
    else k_batch_fallback<float, 2, 1, true, false><<<ngrids, 64 * kFbWaves, 0, s>>>(a, none, nsteps);
    return hipGetLastError();
}

hipError_t sw_batch_launch_gated_fallback(const SwBatchLaunch &a, const SwFallbackGate &gate, int ngrids, int nsteps,
                                          hipStream_t s) {
    if (ngrids <= 0) return hipSuccess;
    if (a.dtype != 0 || !gate.stats || a.rows < 1 || nsteps <= 0) return hipErrorInvalidValue;
    if (a.scheme == 0) k_batch_fallback<float, 2, 1, false, true><<<ngrids, 64 * kFbWaves, 0, s>>>(a, gate, nsteps);
    else k_batch_fallback<float, 2, 1, true, true><<<ngrids, 64 * kFbWaves, 0, s>>>(a, gate, nsteps);
    return hipGetLastError();
}

hipError_t sw_batch_launch_step(const SwBatchLaunch &a, int vec, int minw, int pd, int persistent, hipStream_t s) {
    if (a.ntiles <= 0) return hipSuccess;
#define SW_BATCH_CASE(T, V, M, P) \
    if ((a.dtype == 1) == (sizeof(T) == 8) && vec == V && minw == M && pd == P) \
        return launch_batch_t<T, V, M, P, false>(a, persistent, s);
#define SW_BATCH_TR_CASE(T, V, M, P) \
    if ((a.dtype == 1) == (sizeof(T) == 8) && vec == V && minw == M && pd == P) \
        return launch_batch_t<T, V, M, P, true>(a, persistent, s);
    if (a.scheme == 0) {
        SW_FUSED_SHAPES(SW_BATCH_CASE)
    } else if (a.scheme == 1) {
        SW_FUSED_TR_SHAPES(SW_BATCH_TR_CASE)
    }
#undef SW_BATCH_CASE
#undef SW_BATCH_TR_CASE
    return hipErrorInvalidValue;
}
