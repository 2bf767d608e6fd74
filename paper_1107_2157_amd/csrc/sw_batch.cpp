// libsw batched mode, host side: many independent grids of uneven sizes in
// one caller-allocated arena, one tile table over all of them, one kernel
// launch per time step for the whole batch, and the nsteps loop captured
// once into a hipGraph (replayed with a single hipGraphLaunch per call).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <new>
#include <numeric>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sw.h"
#include "sw_batch_internal.h"

// Shared with sw_api.cpp.
sw_status sw_fail(sw_status s, const char *fmt, ...);
sw_status sw_validate_opts(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts, sw_opts *resolved,
                           sw_layout *layout);

#define BHIP(call)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return sw_fail(SW_EHIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

struct sw_batch {
    int n = 0;
    std::vector<sw_grid> grids;
    sw_opts opts{};
    double g = 0, dx = 0, dy = 0;
    std::vector<sw_layout> lay;
    std::vector<size_t> off;          // byte offset of grid i's first plane inside a buffer region
    size_t region = 0;                // bytes of one buffer region (every grid, three planes)
    char *arena = nullptr;
    int device = 0;
    int cur = 0;
    sw_tuning tuning{};
    SwBatchGrid *d_grids = nullptr;
    SwBatchScalars *d_sc = nullptr;
    SwBatchTile *d_tiles = nullptr;
    size_t tiles_cap = 0;
    int ntiles = 0;
    int split = 0;                    // tiles [0, split) step on the call's stream, [split, ntiles) on `side`
    int table_rows = -1, table_vec = -1, table_order = -1;
    bool use_graph = true;
    uint64_t gen = 0;                 // renewed whenever launch arguments change (bind, tile table)
    hipStream_t cap = nullptr;
    hipStream_t side = nullptr;       // the second chain's stream (default priority)
    hipEvent_t fork = nullptr, join = nullptr;
    struct Graph {
        int nsteps, cur;
        sw_tuning t;
        hipGraphExec_t exec;                  // the whole call, or (split table) its reset and prologue
        hipGraphExec_t chain[2] = {nullptr, nullptr};   // split table: each chain's steps
    };
    std::vector<Graph> graphs;
};

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kSplitCells = (int64_t)1 << 22;   // batches split into two launch chains from this size

// Process-wide source of batch generations: a graph captured by another
// object over a batch's launches is valid while the batch's generation is
// unchanged (a batch created later at the same address gets a new one).
std::atomic<uint64_t> g_next_gen{1};

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

struct Resolved {
    int vec, rows, minw, pd, order;
};

sw_status resolve(const sw_batch *b, const sw_tuning &t, Resolved *r) {
    if (t.variant != 0 && t.variant != 2) return sw_fail(SW_EINVAL, "batch tuning: only the fused variant batches");
    r->vec = t.vec ? t.vec : 2;
    r->rows = t.rows ? t.rows : 16;
    r->minw = t.occupancy;
    r->pd = t.prefetch ? t.prefetch : 2;
    r->order = t.order;
    if (t.rows < 0) return sw_fail(SW_EINVAL, "batch tuning: rows = %d", t.rows);
    if (r->order < 0 || r->order > 2)
        return sw_fail(SW_EINVAL, "batch tuning: order %d (0 LPT, 1 round-robin, 2 LPT walked by persistent waves)",
                       r->order);
    if (!sw_fused_supported((int)b->opts.dtype, (int)b->opts.scheme, r->vec, r->minw, r->pd))
        return sw_fail(SW_EINVAL, "batch tuning: vec %d / occupancy %d / prefetch %d not available", r->vec, r->minw,
                       r->pd);
    for (int i = 0; i < b->n; ++i)   // the fused kernel reaches a tile's rows through 32-bit buffer offsets
        if (!sw_fused_tile_fits(r->rows, b->lay[i].pitch, b->lay[i].elem_bytes))
            return sw_fail(SW_EINVAL, "batch tuning: %d rows per tile of grid %d exceed the fused kernel's 2 GiB tile span",
                           r->rows, i);
    return SW_OK;
}

void drop_graphs(sw_batch *b) {
    for (auto &g : b->graphs) {
        (void)hipGraphExecDestroy(g.exec);
        for (auto c : g.chain)
            if (c) (void)hipGraphExecDestroy(c);
    }
    b->graphs.clear();
}

// Tile table: order 0 and 2 = LPT (grids by cell count, largest first, each
// grid's tiles row-block-major; order 2 launches persistent waves over it);
// order 1 = round-robin over the grids.
sw_status build_tiles(sw_batch *b, const Resolved &r) {
    if (b->table_rows == r.rows && b->table_vec == r.vec && b->table_order == r.order && b->d_tiles) return SW_OK;
    const int W = 64 * r.vec;
    std::vector<int> idx(b->n);
    std::iota(idx.begin(), idx.end(), 0);
    std::stable_sort(idx.begin(), idx.end(), [&](int x, int y) {
        return (int64_t)b->grids[x].nx * b->grids[x].ny > (int64_t)b->grids[y].nx * b->grids[y].ny;
    });
    std::vector<std::vector<SwBatchTile>> per(b->n);
    size_t total = 0;
    for (int gi : idx) {
        const int ns = (b->grids[gi].nx + W - 1) / W, nr = (b->grids[gi].ny + r.rows - 1) / r.rows;
        for (int rb = 0; rb < nr; ++rb)
            for (int s = 0; s < ns; ++s) per[gi].push_back(SwBatchTile{gi, s, rb, 0});
        total += per[gi].size();
    }
    if (total > 0x3fffffff) return sw_fail(SW_EINVAL, "batch: %zu tiles", total);
    // Two chains of grids, dealt alternately in order of size (so their
    // cells balance): each chain's tiles are contiguous in the table and
    // step as their own sequence of launches, on two streams, so that one
    // chain's launch start and drain overlap the other's work (the grids
    // are independent; every cell is computed the same either way).
    // Only batches of 4 M cells or more per step are split: below that a
    // step is short enough that its second launch costs more than the
    // overlap gains (measured: 2.1 M cells 5 % slower split, 4.2 M cells
    // 7-15 % faster).
    int64_t cells = 0;
    for (const auto &g : b->grids) cells += (int64_t)g.nx * g.ny;
    const bool two = b->n >= 2 && cells >= kSplitCells;
    std::vector<int> chain[2];
    for (size_t k = 0; k < idx.size(); ++k) chain[two ? k & 1 : 0].push_back(idx[k]);
    std::vector<SwBatchTile> tiles;
    tiles.reserve(total);
    int split = 0;
    for (int c = 0; c < 2; ++c) {
        if (r.order != 1) {
            for (int gi : chain[c]) tiles.insert(tiles.end(), per[gi].begin(), per[gi].end());
        } else {
            size_t want = tiles.size();
            for (int gi : chain[c]) want += per[gi].size();
            std::vector<size_t> pos(b->n, 0);
            while (tiles.size() < want)
                for (int gi : chain[c])
                    if (pos[gi] < per[gi].size()) tiles.push_back(per[gi][pos[gi]++]);
        }
        if (c == 0) split = (int)tiles.size();
    }
    if (total > b->tiles_cap) {
        if (b->d_tiles) BHIP(hipFree(b->d_tiles));
        b->d_tiles = nullptr;
        BHIP(hipMalloc((void **)&b->d_tiles, total * sizeof(SwBatchTile)));
        b->tiles_cap = total;
    }
    BHIP(hipMemcpy(b->d_tiles, tiles.data(), total * sizeof(SwBatchTile), hipMemcpyHostToDevice));
    b->ntiles = (int)total;
    b->split = split;
    b->gen = g_next_gen.fetch_add(1);
    b->table_rows = r.rows;
    b->table_vec = r.vec;
    b->table_order = r.order;
    drop_graphs(b);
    return SW_OK;
}

SwBatchLaunch launch_of(const sw_batch *b, const Resolved &r, int cur, int step) {
    SwBatchLaunch a{};
    a.tiles = b->d_tiles;
    a.grids = b->d_grids;
    a.sc = b->d_sc;
    a.ntiles = b->ntiles;
    a.cur = cur;
    a.step = step;
    a.rows = r.rows;
    a.g = b->g;
    a.dx = b->dx;
    a.dy = b->dy;
    a.cfl = b->opts.cfl;
    a.dt_fixed = b->opts.dt_fixed;
    a.bc_x = (int)b->opts.bc_x;
    a.bc_y = (int)b->opts.bc_y;
    a.dtype = (int)b->opts.dtype;
    a.scheme = (int)b->opts.scheme;
    a.ghosts = 1;
    return a;
}

// With reflective walls on both axes and every grid's width a multiple of
// the cells per lane, the paper's scheme reads no ghost cell (the walls'
// images are formed from the edge cells; a width that is not a multiple
// puts the right ghost inside a lane's vector, which is read), so only a
// call's last step writes them.
bool batch_ghost_free(const sw_batch *b, const Resolved &r) {
    bool ghost_free = b->opts.scheme == SW_SCHEME_PAPER && b->opts.bc_x == SW_BC_REFLECT && b->opts.bc_y == SW_BC_REFLECT;
    for (int i = 0; i < b->n && ghost_free; ++i) ghost_free = b->grids[i].nx % r.vec == 0;
    return ghost_free;
}

// The table is split into two launch chains (build_tiles).
bool split_table(const sw_batch *b) { return b->side && b->split > 0 && b->split < b->ntiles; }

// reset + prologue of a call on stream s, from buffer cur
sw_status enqueue_head(const sw_batch *b, const Resolved &r, int cur, hipStream_t s, const int32_t *active) {
    BHIP(sw_batch_launch_reset(b->d_sc, b->n, 0, s));
    SwBatchLaunch p = launch_of(b, r, cur, 0);
    p.active = active;
    BHIP(sw_batch_launch_prologue(p, r.vec, s));
    return SW_OK;
}

// nsteps step launches of table entries [t0, t0 + nt) on stream s
sw_status enqueue_chain(const sw_batch *b, const Resolved &r, int nsteps, int cur, int t0, int nt, hipStream_t s,
                        const int32_t *active) {
    const bool ghost_free = batch_ghost_free(b, r);
    for (int k = 0; k < nsteps; ++k) {
        SwBatchLaunch a = launch_of(b, r, cur, k);
        a.active = active;
        a.tiles = b->d_tiles + t0;
        a.ntiles = nt;
        a.ghosts = ghost_free && k + 1 < nsteps ? 0 : 1;
        BHIP(sw_batch_launch_step(a, r.vec, r.minw, r.pd, r.order == 2, s));
        cur ^= 1;
    }
    return SW_OK;
}

// reset + prologue + nsteps step launches on stream s, starting from buffer
// cur; active (device, optional) restricts the work to some grids.  A split
// table's second chain runs on the batch's side stream, forked from s after
// the prologue and joined back into s at the end; the two chains' launches
// are issued alternately so that both start at once.
sw_status enqueue(const sw_batch *b, const Resolved &r, int nsteps, int cur, hipStream_t s,
                  const int32_t *active = nullptr) {
    sw_status st = enqueue_head(b, r, cur, s, active);
    if (st != SW_OK) return st;
    if (!split_table(b)) return enqueue_chain(b, r, nsteps, cur, 0, b->ntiles, s, active);
    BHIP(hipEventRecord(b->fork, s));
    BHIP(hipStreamWaitEvent(b->side, b->fork, 0));
    for (int k = 0; k < nsteps; ++k) {
        const bool last = k + 1 == nsteps;
        // one step of each chain; ghost writes only in the call's last step
        for (int c = 0; c < 2; ++c) {
            SwBatchLaunch a = launch_of(b, r, cur, k);
            a.active = active;
            a.tiles = b->d_tiles + (c ? b->split : 0);
            a.ntiles = c ? b->ntiles - b->split : b->split;
            a.ghosts = batch_ghost_free(b, r) && !last ? 0 : 1;
            BHIP(sw_batch_launch_step(a, r.vec, r.minw, r.pd, r.order == 2, c ? b->side : s));
        }
        cur ^= 1;
    }
    BHIP(hipEventRecord(b->join, b->side));
    BHIP(hipStreamWaitEvent(s, b->join, 0));
    return SW_OK;
}

bool same_tuning(const sw_tuning &x, const sw_tuning &y) { return std::memcmp(&x, &y, sizeof x) == 0; }

sw_status check_bound(const sw_batch *b) {
    if (!b) return sw_fail(SW_EINVAL, "batch: NULL");
    if (!b->arena) return sw_fail(SW_EINVAL, "batch: no arena bound (sw_batch_bind)");
    int dev = -1;
    BHIP(hipGetDevice(&dev));
    if (dev != b->device) BHIP(hipSetDevice(b->device));
    return SW_OK;
}

}  // namespace

int sw_batch_internal_info(const sw_batch *b, SwBatchInfo *info) {
    if (!b || !info) return sw_fail(SW_EINVAL, "batch: NULL");
    if (!b->arena) return sw_fail(SW_EINVAL, "batch: no arena bound");
    info->d_grids = b->d_grids;
    info->d_sc = b->d_sc;
    info->n = b->n;
    info->cur = b->cur;
    info->dtype = (int)b->opts.dtype;
    info->bc_x = (int)b->opts.bc_x;
    info->bc_y = (int)b->opts.bc_y;
    info->same_nx = b->grids[0].nx;
    info->same_ny = b->grids[0].ny;
    for (auto &g : b->grids)
        if (g.nx != info->same_nx || g.ny != info->same_ny) info->same_nx = info->same_ny = -1;
    info->gen = b->gen;
    return SW_OK;
}

int sw_batch_internal_prepare(sw_batch *b) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    Resolved r;
    if ((st = resolve(b, b->tuning, &r)) != SW_OK) return st;
    return build_tiles(b, r);
}

int sw_batch_internal_fallback(sw_batch *b, int nsteps, const int32_t *active, hipStream_t s) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    if (nsteps < 0 || (nsteps & 1)) return sw_fail(SW_EINVAL, "batch: masked steps must be even (%d)", nsteps);
    if (!active || b->opts.dtype != SW_F32) return sw_fail(SW_EINVAL, "batch: the fallback runs FP32 batches");
    Resolved r;
    if ((st = resolve(b, b->tuning, &r)) != SW_OK) return st;
    SwBatchLaunch a = launch_of(b, r, b->cur, 0);
    a.active = active;
    BHIP(sw_batch_launch_fallback(a, b->n, nsteps, s));
    return SW_OK;
}

int sw_batch_internal_gated_fallback(sw_batch *b, int nsteps, const SwFallbackGate &gate, hipStream_t s) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    if (nsteps < 2 || (nsteps & 1)) return sw_fail(SW_EINVAL, "batch: masked steps must be even and > 0 (%d)", nsteps);
    if (!gate.stats || b->opts.dtype != SW_F32) return sw_fail(SW_EINVAL, "batch: the fallback runs FP32 batches");
    Resolved r;
    if ((st = resolve(b, b->tuning, &r)) != SW_OK) return st;
    SwBatchLaunch a = launch_of(b, r, b->cur, 0);
    BHIP(sw_batch_launch_gated_fallback(a, gate, b->n, nsteps, s));
    return SW_OK;
}

int sw_batch_internal_set_cur(sw_batch *b, int cur) {
    if (!b || (cur != 0 && cur != 1)) return sw_fail(SW_EINVAL, "batch: set_cur %d", cur);
    b->cur = cur;
    return SW_OK;
}

bool sw_batch_internal_compatible(const sw_batch *a, const sw_batch *b) {
    if (!a || !b || a->n != b->n || a->region != b->region || a->g != b->g || a->dx != b->dx) return false;
    if (std::memcmp(&a->opts, &b->opts, sizeof a->opts) != 0) return false;
    for (int i = 0; i < a->n; ++i)
        if (a->grids[i].nx != b->grids[i].nx || a->grids[i].ny != b->grids[i].ny) return false;
    return true;
}

int sw_batch_internal_clone(const sw_batch *src, sw_batch **out, void **arena) {
    if (!src || !out || !arena) return sw_fail(SW_EINVAL, "batch clone: NULL argument");
    *out = nullptr;
    *arena = nullptr;
    sw_batch *c = nullptr;
    const sw_halo halo{1, 1, 1, 1};
    sw_status st = sw_batch_create(src->n, src->grids.data(), halo, src->g, src->dx, &src->opts, &c);
    if (st != SW_OK) return st;
    c->tuning = src->tuning;
    hipError_t e = hipMalloc(arena, 2 * c->region);
    if (e != hipSuccess) {
        sw_batch_destroy(c);
        return sw_fail(e == hipErrorOutOfMemory ? SW_ENOMEM : SW_EHIP, "batch clone: %s", hipGetErrorString(e));
    }
    if ((st = sw_batch_bind(c, *arena)) != SW_OK) {
        sw_batch_destroy(c);
        (void)hipFree(*arena);
        *arena = nullptr;
        return st;
    }
    *out = c;
    return SW_OK;
}

int sw_batch_internal_copy_state(sw_batch *dst, const sw_batch *src, hipStream_t s) {
    sw_status st = check_bound(dst);
    if (st != SW_OK) return st;
    if ((st = check_bound(src)) != SW_OK) return st;
    if (!sw_batch_internal_compatible(dst, src)) return sw_fail(SW_EINVAL, "batch copy: batches differ");
    BHIP(hipMemcpyAsync(dst->arena + (size_t)src->cur * src->region, src->arena + (size_t)src->cur * src->region,
                        src->region, hipMemcpyDeviceToDevice, s));
    dst->cur = src->cur;
    BHIP(sw_batch_launch_reset(dst->d_sc, dst->n, 1, s));
    return SW_OK;
}

extern "C" {

sw_status sw_batch_create(int32_t n, const sw_grid *grids, sw_halo halo, double g, double dx, const sw_opts *opts,
                          sw_batch **out) {
    if (!out) return sw_fail(SW_EINVAL, "batch_create: NULL output");
    *out = nullptr;
    if (n < 1 || !grids) return sw_fail(SW_EINVAL, "batch_create: n = %d grids", n);
    sw_opts o{};
    std::vector<sw_layout> lay(n);
    for (int i = 0; i < n; ++i) {
        sw_status st = sw_validate_opts(grids[i], halo, g, dx, opts, &o, &lay[i]);
        if (st != SW_OK) return st;
    }
    auto *b = new (std::nothrow) sw_batch();
    if (!b) return sw_fail(SW_ENOMEM, "batch_create: host allocation");
    b->n = n;
    b->grids.assign(grids, grids + n);
    b->opts = o;
    b->g = g;
    b->dx = dx;
    b->dy = o.dy;
    b->lay = lay;
    b->off.resize(n);
    size_t at = 0;
    for (int i = 0; i < n; ++i) {
        b->off[i] = at;
        at += align_up((size_t)lay[i].buffer_elems * (size_t)lay[i].elem_bytes);   // three interleaved planes
    }
    b->region = at;
    hipError_t e = hipGetDevice(&b->device);
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_sc, (size_t)n * sizeof(SwBatchScalars));
    if (e == hipSuccess) e = hipMemset(b->d_sc, 0, (size_t)n * sizeof(SwBatchScalars));
    if (e == hipSuccess) e = hipMalloc((void **)&b->d_grids, (size_t)n * sizeof(SwBatchGrid));
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&b->side, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->join, hipEventDisableTiming);
    if (e != hipSuccess) {
        sw_batch_destroy(b);
        return sw_fail(e == hipErrorOutOfMemory ? SW_ENOMEM : SW_EHIP, "batch_create: %s", hipGetErrorString(e));
    }
    *out = b;
    return SW_OK;
}

sw_status sw_batch_destroy(sw_batch *b) {
    if (!b) return SW_OK;
    drop_graphs(b);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->side) (void)hipStreamDestroy(b->side);
    if (b->fork) (void)hipEventDestroy(b->fork);
    if (b->join) (void)hipEventDestroy(b->join);
    if (b->d_sc) (void)hipFree(b->d_sc);
    if (b->d_grids) (void)hipFree(b->d_grids);
    if (b->d_tiles) (void)hipFree(b->d_tiles);
    delete b;
    return SW_OK;
}

sw_status sw_batch_arena_bytes(const sw_batch *b, size_t *bytes) {
    if (!b || !bytes) return sw_fail(SW_EINVAL, "batch_arena_bytes: NULL argument");
    *bytes = 2 * b->region;
    return SW_OK;
}

sw_status sw_batch_bind(sw_batch *b, void *arena) {
    if (!b || !arena) return sw_fail(SW_EINVAL, "batch_bind: NULL argument");
    if ((uintptr_t)arena % kAlign) return sw_fail(SW_EINVAL, "batch_bind: arena not 256-byte aligned");
    int dev = -1;
    BHIP(hipGetDevice(&dev));
    if (dev != b->device) BHIP(hipSetDevice(b->device));
    b->arena = (char *)arena;
    b->gen = g_next_gen.fetch_add(1);
    std::vector<SwBatchGrid> d(b->n);
    for (int i = 0; i < b->n; ++i) {
        const size_t pb = (size_t)b->lay[i].plane_offset * (size_t)b->lay[i].elem_bytes;
        for (int buf = 0; buf < 2; ++buf)
            for (int k = 0; k < 3; ++k)
                d[i].plane[buf][k] = b->arena + buf * b->region + b->off[i] + k * pb +
                                     (size_t)b->lay[i].origin * (size_t)b->lay[i].elem_bytes;
        d[i].pitch = b->lay[i].pitch;
        d[i].nx = b->grids[i].nx;
        d[i].ny = b->grids[i].ny;
    }
    BHIP(hipMemcpy(b->d_grids, d.data(), d.size() * sizeof(SwBatchGrid), hipMemcpyHostToDevice));
    b->cur = 0;
    drop_graphs(b);
    Resolved r;
    sw_status st = resolve(b, b->tuning, &r);
    if (st != SW_OK) return st;
    return build_tiles(b, r);
}

sw_status sw_batch_view(const sw_batch *b, int32_t i, sw_state *view, sw_layout *layout) {
    if (!b || !view) return sw_fail(SW_EINVAL, "batch_view: NULL argument");
    if (i < 0 || i >= b->n) return sw_fail(SW_EINVAL, "batch_view: grid %d of %d", i, b->n);
    if (!b->arena) return sw_fail(SW_EINVAL, "batch_view: no arena bound");
    const size_t pb = (size_t)b->lay[i].plane_offset * (size_t)b->lay[i].elem_bytes;
    for (int buf = 0; buf < 2; ++buf)
        for (int k = 0; k < 3; ++k) view->plane[buf][k] = b->arena + buf * b->region + b->off[i] + k * pb;
    view->cur = b->cur;
    view->reserved = 0;
    if (layout) *layout = b->lay[i];
    return SW_OK;
}

sw_status sw_batch_set_tuning(sw_batch *b, const sw_tuning *t) {
    if (!b || !t) return sw_fail(SW_EINVAL, "batch_set_tuning: NULL argument");
    Resolved r, prev;
    sw_status st = resolve(b, *t, &r);
    if (st != SW_OK) return st;
    const bool had = resolve(b, b->tuning, &prev) == SW_OK;
    b->tuning = *t;
    // any change of the launch shape renews the generation, so rollouts
    // captured by a surrogate with the old shape are captured anew (the tile
    // table below renews it too when rows, vec or order change)
    if (!had || std::memcmp(&prev, &r, sizeof r) != 0) b->gen = g_next_gen.fetch_add(1);
    if (b->arena) {
        int dev = -1;
        BHIP(hipGetDevice(&dev));
        if (dev != b->device) BHIP(hipSetDevice(b->device));
        return build_tiles(b, r);
    }
    return SW_OK;
}

sw_status sw_batch_get_tuning(const sw_batch *b, sw_tuning *out) {
    if (!b || !out) return sw_fail(SW_EINVAL, "batch_get_tuning: NULL argument");
    Resolved r;
    sw_status st = resolve(b, b->tuning, &r);
    if (st != SW_OK) return st;
    *out = sw_tuning{2, r.rows, r.vec, r.minw, r.pd, r.order};
    return SW_OK;
}

sw_status sw_batch_set_graph(sw_batch *b, int32_t enable) {
    if (!b) return sw_fail(SW_EINVAL, "batch_set_graph: NULL");
    b->use_graph = enable != 0;
    return SW_OK;
}

sw_status sw_batch_fill_halo(sw_batch *b, void *stream) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    Resolved r;
    if ((st = resolve(b, b->tuning, &r)) != SW_OK) return st;
    if ((st = build_tiles(b, r)) != SW_OK) return st;
    // the prologue materialises the ghosts (its speed reduction is refreshed by the next step call)
    BHIP(sw_batch_launch_prologue(launch_of(b, r, b->cur, 0), r.vec, (hipStream_t)stream));
    return SW_OK;
}

sw_status sw_batch_step(sw_batch *b, int32_t nsteps, void *stream) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    if (nsteps < 0) return sw_fail(SW_EINVAL, "batch_step: nsteps = %d", nsteps);
    if (nsteps == 0) return SW_OK;
    Resolved r;
    if ((st = resolve(b, b->tuning, &r)) != SW_OK) return st;
    if ((st = build_tiles(b, r)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    if (!b->use_graph) {
        if ((st = enqueue(b, r, nsteps, b->cur, s)) != SW_OK) return st;
    } else {
        const bool two = split_table(b);
        const sw_batch::Graph *found = nullptr;
        for (auto &gr : b->graphs)
            if (gr.nsteps == nsteps && gr.cur == b->cur && same_tuning(gr.t, b->tuning)) found = &gr;
        if (!found) {
            if (b->graphs.size() >= 8) drop_graphs(b);
            // capture one part of the call on the capture stream
            auto capture = [&](auto &&fn, hipGraphExec_t *exec) -> sw_status {
                BHIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
                sw_status cst = fn(b->cap);
                hipGraph_t graph = nullptr;
                hipError_t e = hipStreamEndCapture(b->cap, &graph);
                if (cst != SW_OK) {
                    if (graph) (void)hipGraphDestroy(graph);
                    return cst;
                }
                if (e != hipSuccess) return sw_fail(SW_EHIP, "batch_step: capture: %s", hipGetErrorString(e));
                e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
                (void)hipGraphDestroy(graph);
                if (e != hipSuccess) return sw_fail(SW_EHIP, "batch_step: instantiate: %s", hipGetErrorString(e));
                return SW_OK;
            };
            sw_batch::Graph gr{nsteps, b->cur, b->tuning, nullptr};
            const int cur = b->cur;
            if (!two) {
                st = capture([&](hipStream_t cs) { return enqueue(b, r, nsteps, cur, cs); }, &gr.exec);
            } else {
                // the split table's chains as graphs of their own, launched on
                // two streams (branches of one graph were measured to overlap
                // less): the head (reset, prologue), then each chain's steps
                st = capture([&](hipStream_t cs) { return enqueue_head(b, r, cur, cs, nullptr); }, &gr.exec);
                if (st == SW_OK)
                    st = capture([&](hipStream_t cs) { return enqueue_chain(b, r, nsteps, cur, 0, b->split, cs, nullptr); },
                                 &gr.chain[0]);
                if (st == SW_OK)
                    st = capture([&](hipStream_t cs) {
                        return enqueue_chain(b, r, nsteps, cur, b->split, b->ntiles - b->split, cs, nullptr);
                    }, &gr.chain[1]);
            }
            if (st != SW_OK) {
                if (gr.exec) (void)hipGraphExecDestroy(gr.exec);
                for (auto c : gr.chain)
                    if (c) (void)hipGraphExecDestroy(c);
                return st;
            }
            b->graphs.push_back(gr);
            found = &b->graphs.back();
        }
        BHIP(hipGraphLaunch(found->exec, s));
        if (found->chain[0]) {
            BHIP(hipEventRecord(b->fork, s));
            BHIP(hipStreamWaitEvent(b->side, b->fork, 0));
            BHIP(hipGraphLaunch(found->chain[0], s));
            BHIP(hipGraphLaunch(found->chain[1], b->side));
            BHIP(hipEventRecord(b->join, b->side));
            BHIP(hipStreamWaitEvent(s, b->join, 0));
        }
    }
    b->cur ^= (nsteps & 1);
    return SW_OK;
}

sw_status sw_batch_sync_status(sw_batch *b, void *stream, double *t, int64_t *steps, int32_t *unstable) {
    if (!b) return sw_fail(SW_EINVAL, "batch_sync_status: NULL");
    int dev = -1;
    BHIP(hipGetDevice(&dev));
    if (dev != b->device) BHIP(hipSetDevice(b->device));
    BHIP(hipStreamSynchronize((hipStream_t)stream));
    std::vector<SwBatchScalars> h(b->n);
    BHIP(hipMemcpy(h.data(), b->d_sc, h.size() * sizeof(SwBatchScalars), hipMemcpyDeviceToHost));
    bool any = false;
    for (int i = 0; i < b->n; ++i) {
        if (t) t[i] = h[i].t;
        if (steps) steps[i] = h[i].steps;
        if (unstable) unstable[i] = (int32_t)h[i].unstable;
        any |= h[i].unstable != 0;
    }
    if (any) return sw_fail(SW_EUNSTABLE, "batch: a grid produced h <= 0 or a non-finite value");
    return SW_OK;
}

static sw_status batch_copy(sw_batch *b, void *dense, int to_dense, void *stream) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    if (!dense) return sw_fail(SW_EINVAL, "batch export/import: NULL buffer");
    for (auto &g : b->grids)
        if (g.nx != b->grids[0].nx || g.ny != b->grids[0].ny)
            return sw_fail(SW_EINVAL, "batch export/import: grids differ in size");
    BHIP(sw_batch_launch_copy(b->d_grids, b->cur, b->n, b->grids[0].nx, b->grids[0].ny, (int)b->opts.dtype, dense,
                              to_dense, (hipStream_t)stream));
    return SW_OK;
}

sw_status sw_batch_export(sw_batch *b, void *dense, void *stream) { return batch_copy(b, dense, 1, stream); }
sw_status sw_batch_import(sw_batch *b, const void *dense, void *stream) {
    return batch_copy(b, const_cast<void *>(dense), 0, stream);
}

sw_status sw_batch_reset_time(sw_batch *b, void *stream) {
    if (!b) return sw_fail(SW_EINVAL, "batch_reset_time: NULL");
    BHIP(sw_batch_launch_reset(b->d_sc, b->n, 1, (hipStream_t)stream));
    return SW_OK;
}

sw_status sw_batch_autotune(sw_batch *b, int32_t steps_per_trial, const char *cache_path, void *stream,
                            sw_tuning *best_out) {
    sw_status st = check_bound(b);
    if (st != SW_OK) return st;
    if (steps_per_trial < 1) return sw_fail(SW_EINVAL, "batch_autotune: steps_per_trial = %d", steps_per_trial);
    hipStream_t s = (hipStream_t)stream;
    // cache key: arch, CUs, dtype, scheme, number of grids and total cells
    std::string key;
    {
        hipDeviceProp_t prop;
        std::string arch = "unknown";
        int cus = 0;
        if (hipGetDeviceProperties(&prop, b->device) == hipSuccess) {
            arch = prop.gcnArchName;
            arch = arch.substr(0, arch.find(':'));
            cus = prop.multiProcessorCount;
        }
        int64_t cells = 0;
        for (auto &g : b->grids) cells += (int64_t)g.nx * g.ny;
        std::ostringstream k;
        k << arch << ":" << cus << ":" << (b->opts.dtype == SW_F64 ? "f64" : "f32") << ":" << (int)b->opts.scheme
          << ":batch" << b->n << ":" << cells;
        key = k.str();
    }
    if (cache_path && *cache_path) {
        std::ifstream f(cache_path);
        std::string line;
        sw_tuning c{}, hit{};
        bool found = false;
        while (std::getline(f, line)) {
            std::istringstream is(line);
            std::string k;
            double us;
            if (is >> k >> c.variant >> c.rows >> c.vec >> c.occupancy >> c.prefetch >> c.order >> us && k == key) {
                hit = c;
                found = true;
            }
        }
        if (found && sw_batch_set_tuning(b, &hit) == SW_OK) {
            if (best_out) sw_batch_get_tuning(b, best_out);
            return SW_OK;
        }
    }
    std::vector<sw_tuning> cands;
    const int vecs_f32[] = {1, 2, 4}, vecs_f64[] = {1, 2};
    const int nv = b->opts.dtype == SW_F64 ? 2 : 3;
    const int *vecs = b->opts.dtype == SW_F64 ? vecs_f64 : vecs_f32;
    for (int vi = 0; vi < nv; ++vi)
        for (int occ : {0, 3, 4})
            for (int pd = 1; pd <= 3; ++pd)
                if (sw_fused_supported((int)b->opts.dtype, (int)b->opts.scheme, vecs[vi], occ, pd))
                    for (int rows : {2, 4, 8, 16, 32})
                        for (int order = 0; order <= 2; ++order) cands.push_back(sw_tuning{2, rows, vecs[vi], occ, pd, order});
    const bool graph0 = b->use_graph;
    const sw_tuning prev = b->tuning;
    const int cur0 = b->cur;
    void *backup = nullptr, *sbackup = nullptr;
    const size_t sbytes = (size_t)b->n * sizeof(SwBatchScalars);
    if (hipMalloc(&backup, b->region) != hipSuccess) return sw_fail(SW_ENOMEM, "batch_autotune: backup");
    if (hipMalloc(&sbackup, sbytes) != hipSuccess) {
        (void)hipFree(backup);
        return sw_fail(SW_ENOMEM, "batch_autotune: backup");
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he == hipSuccess) he = hipMemcpyAsync(backup, b->arena + cur0 * b->region, b->region, hipMemcpyDeviceToDevice, s);
    if (he == hipSuccess) he = hipMemcpyAsync(sbackup, b->d_sc, sbytes, hipMemcpyDeviceToDevice, s);
    auto restore = [&]() -> hipError_t {
        b->cur = cur0;
        hipError_t e = hipMemcpyAsync(b->arena + cur0 * b->region, backup, b->region, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(b->d_sc, sbackup, sbytes, hipMemcpyDeviceToDevice, s);
        return e;
    };
    auto timed = [&](int k, float *ms) -> hipError_t {
        hipError_t e = hipEventRecord(e0, s);
        if (e != hipSuccess) return e;
        if (sw_batch_step(b, k, stream) != SW_OK) return hipErrorUnknown;
        if ((e = hipEventRecord(e1, s)) != hipSuccess) return e;
        if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
        return hipEventElapsedTime(ms, e0, e1);
    };
    // Trials replay graphs, as sw_batch_step runs (eager launches would time
    // the host's launch rate on small batches); each shape's graphs are
    // captured in an untimed warm-up first, and every run starts from the
    // saved state (so from the same buffer, whose graphs were captured).
    b->use_graph = true;
    auto warm = [&](int k1, int k2) -> hipError_t {
        drop_graphs(b);
        hipError_t e = restore();
        if (e != hipSuccess) return e;
        if (sw_batch_step(b, k1, stream) != SW_OK) return hipErrorUnknown;
        if (k2 > 0 && sw_batch_step(b, k2, stream) != SW_OK) return hipErrorUnknown;
        return restore();
    };
    // Steps per trial: enough for the timed difference to span about 2 ms
    // (small batches take a few microseconds per step), measured with the
    // tuning in place; each trial takes the best of two runs of each length.
    int steps = steps_per_trial;
    if (he == hipSuccess && (he = warm(steps, 0)) == hipSuccess) {
        float m = 0.f;
        if ((he = timed(steps, &m)) == hipSuccess && m > 0.f && m < 2.f)
            steps = (int)std::min<double>(2000.0, std::ceil(steps * 2.0 / m));
    }
    sw_tuning best{};
    double best_us = 1e300;
    for (size_t i = 0; i < cands.size() && he == hipSuccess; ++i) {
        if (sw_batch_set_tuning(b, &cands[i]) != SW_OK) continue;
        if ((he = warm(1, 1 + steps)) != hipSuccess) break;
        float m1 = 1e30f, mk = 1e30f;
        for (int rep = 0; rep < 2 && he == hipSuccess; ++rep) {
            float a = 0.f, c = 0.f;
            if (rep > 0 && (he = restore()) != hipSuccess) break;
            if ((he = timed(1, &a)) != hipSuccess) break;
            if ((he = timed(1 + steps, &c)) != hipSuccess) break;
            m1 = std::min(m1, a);
            mk = std::min(mk, c);
        }
        if (he != hipSuccess) break;
        const double us = 1000.0 * (mk - m1) / steps;
        if (us < best_us) {
            best_us = us;
            best = cands[i];
        }
    }
    if (he == hipSuccess) he = restore();
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);           // no trial graph is still running
    drop_graphs(b);                          // the trial shapes' graphs
    (void)hipFree(backup);
    (void)hipFree(sbackup);
    b->use_graph = graph0;
    if (he != hipSuccess || best_us >= 1e300) {
        sw_batch_set_tuning(b, &prev);
        return he != hipSuccess ? sw_fail(SW_EHIP, "batch_autotune: %s", hipGetErrorString(he))
                                : sw_fail(SW_ENOTSUP, "batch_autotune: no candidate ran");
    }
    sw_batch_set_tuning(b, &best);
    if (cache_path && *cache_path) {
        std::ofstream f(cache_path, std::ios::app);
        f << key << " " << best.variant << " " << best.rows << " " << best.vec << " " << best.occupancy << " "
          << best.prefetch << " " << best.order << " " << best_us << "\n";
    }
    if (best_out) sw_batch_get_tuning(b, best_out);
    return SW_OK;
}

}  // extern "C"
