// libsw C-ABI host side: argument validation, layout, context lifetime and
// the launch sequence of a time-step call.  All arguments are validated
// before any HIP call, so invalid input never reaches a kernel.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/sw.h"
#include "sw_internal.h"

struct sw_ctx {
    sw_grid grid;
    sw_opts opts;
    double g, dx, dy;
    sw_layout layout;
    int device;
    sw_tuning tuning;   // as set by the caller (zero = default)
    SwScalars *sc;      // device
    // sw_step as one graph launch: captured once per (nsteps, cur, planes,
    // launch shape) on a private stream, replayed on the caller's
    bool use_graph = true;
    hipStream_t cap = nullptr;
    struct Graph {
        int nsteps, cur;
        const void *planes[2][3];
        SwTuning tun;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
    // workspace of the comparison variants (face planes or AoS buffers),
    // allocated by the first sw_step that needs it, freed by sw_destroy
    void *ws = nullptr;
    size_t ws_bytes = 0;
    double *diag = nullptr;   // partials and result of sw_diagnostics (allocated by sw_create)
};

namespace {

thread_local std::string g_detail;

sw_status vfail(sw_status s, const char *fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof buf, fmt, ap);
    g_detail = buf;
    return s;
}

sw_status fail(sw_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(s, fmt, ap);
    va_end(ap);
    return s;
}

#define SW_HIP(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess) return fail(SW_EHIP, "%s: %s", #call, hipGetErrorString(e_)); \
    } while (0)

constexpr int64_t kAlignBytes = 256;

sw_status layout_for(sw_grid grid, sw_dtype dtype, sw_layout *out) {
    if (!out) return fail(SW_EINVAL, "layout: NULL output");
    if (dtype != SW_F32 && dtype != SW_F64) return fail(SW_EINVAL, "layout: unknown dtype %d", (int)dtype);
    if (grid.nx < 1 || grid.ny < 1) return fail(SW_EINVAL, "layout: grid %d x %d is empty", grid.nx, grid.ny);
    // The fused kernel addresses one tile through 32-bit buffer offsets; with
    // nx <= 2^21 its default tiles (at most 8 rows + 2 halo rows of three
    // interleaved planes) stay far below 2 GiB in FP64, and set_tuning refuses
    // taller tiles that would not.
    if (grid.nx > (1 << 21)) return fail(SW_EINVAL, "layout: nx = %d above 2^21", grid.nx);
    if (grid.ny > (1 << 30)) return fail(SW_EINVAL, "layout: ny = %d above 2^30", grid.ny);
    const int64_t eb = dtype == SW_F64 ? 8 : 4;
    const int64_t a = kAlignBytes / eb;                       // elements per 256 bytes
    const int64_t lead = a;                                   // interior starts 256 B into each row
    int64_t row = (lead + (int64_t)grid.nx + 1 + a - 1) / a * a;
    // Avoid row lengths that are a large power of two (rows would start on the
    // same HBM channel): add one 256-byte block if row*eb is a multiple of 64 KiB.
    if ((row * eb) % (64 * 1024) == 0) row += a;
    // Rows of h, hu and hv interleave inside one buffer: a step then streams
    // one contiguous region per buffer rather than three distant ones (the
    // same bytes, measured 2-6 % faster on MI355X than separate planes).
    const int64_t pitch = 3 * row;
    out->pitch = pitch;
    out->origin = pitch + lead;
    out->plane_elems = ((int64_t)grid.ny + 1) * pitch + row;
    out->plane_offset = row;
    out->buffer_elems = ((int64_t)grid.ny + 2) * pitch;
    out->elem_bytes = (int32_t)eb;
    out->reserved = 0;
    return SW_OK;
}

sw_status check_state(const sw_ctx *ctx, const sw_state *st, bool both_buffers) {
    if (!st) return fail(SW_EINVAL, "state: NULL");
    if (st->cur != 0 && st->cur != 1) return fail(SW_EINVAL, "state: cur = %d (must be 0 or 1)", st->cur);
    for (int b = 0; b < 2; ++b) {
        if (!both_buffers && b != st->cur) continue;
        for (int k = 0; k < 3; ++k) {
            const void *p = st->plane[b][k];
            if (!p) return fail(SW_EINVAL, "state: plane[%d][%d] is NULL", b, k);
            if ((uintptr_t)p % kAlignBytes) return fail(SW_EINVAL, "state: plane[%d][%d] not 256-byte aligned", b, k);
        }
    }
    if (both_buffers)
        for (int k = 0; k < 3; ++k)
            for (int m = 0; m < 3; ++m)
                if (st->plane[0][k] == st->plane[1][m])
                    return fail(SW_EINVAL, "state: buffers 0 and 1 share plane memory (double buffering needs distinct planes)");
    return SW_OK;
}

SwLaunch launch_of(const sw_ctx *ctx, const sw_state *st, int from) {
    SwLaunch a{};
    const int64_t eb = ctx->layout.elem_bytes;
    for (int k = 0; k < 3; ++k) {
        a.in[k] = (const char *)st->plane[from][k] + ctx->layout.origin * eb;
        a.out[k] = (char *)st->plane[from ^ 1][k] + ctx->layout.origin * eb;
    }
    a.pitch = ctx->layout.pitch;
    a.nx = ctx->grid.nx;
    a.ny = ctx->grid.ny;
    a.g = ctx->g;
    a.dx = ctx->dx;
    a.dy = ctx->dy;
    a.cfl = ctx->opts.cfl;
    a.dt_fixed = ctx->opts.dt_fixed;
    a.bc_x = (int32_t)ctx->opts.bc_x;
    a.bc_y = (int32_t)ctx->opts.bc_y;
    a.scheme = (int32_t)ctx->opts.scheme;
    a.dtype = (int32_t)ctx->opts.dtype;
    a.sc = ctx->sc;
    a.step = 0;
    a.ghosts = 1;
    return a;
}

sw_status use_device(const sw_ctx *ctx) {
    int cur = -1;
    SW_HIP(hipGetDevice(&cur));
    if (cur != ctx->device) SW_HIP(hipSetDevice(ctx->device));
    return SW_OK;
}

// Cells of one AoS copy of a buffer: ny + 2 rows of plane_offset cells (the
// AoS rows need no interleaving, so their pitch is one plane's row).
size_t aos_elems(const sw_ctx *ctx) { return (size_t)ctx->layout.plane_offset * ((size_t)ctx->grid.ny + 2); }

// Workspace bytes of a step variant: six face planes (unfused) or two AoS
// buffers of 4-vectors (AoS); none for the others.
// Face planes interleave by rows as the state's do (x faces in one block of
// ny + 1 rows of pitch elements, y faces in a second); each AoS copy holds
// ny + 2 rows of plane_offset 4-vectors.
size_t workspace_bytes(const sw_ctx *ctx, int variant) {
    const size_t eb = (size_t)ctx->layout.elem_bytes;
    if (variant == 4) return 2 * (size_t)ctx->layout.pitch * ((size_t)ctx->grid.ny + 1) * eb;
    if (variant == 5) return 2 * aos_elems(ctx) * 4 * eb;
    return 0;
}

// reset + prologue + nsteps step launches on stream s (no host sync)
sw_status enqueue_steps(sw_ctx *ctx, const sw_state *state, int nsteps, const SwTuning &tun, hipStream_t s) {
    SW_HIP(sw_launch_reset(ctx->sc, 0, s));
    SW_HIP(sw_launch_prologue(launch_of(ctx, state, state->cur), s));
    int cur = state->cur, n = 0;
    const size_t eb = (size_t)ctx->layout.elem_bytes;
    if (tun.variant == 4) {
        const size_t block = (size_t)ctx->layout.pitch * ((size_t)ctx->grid.ny + 1) * eb;
        const size_t row = (size_t)ctx->layout.plane_offset * eb;
        SwFaces f;
        for (int k = 0; k < 3; ++k) {
            f.x[k] = (char *)ctx->ws + k * row;
            f.y[k] = (char *)ctx->ws + block + k * row;
        }
        f.pitch = ctx->layout.pitch;
        for (; n < nsteps; ++n) {
            SwLaunch b = launch_of(ctx, state, cur);
            b.step = n;
            SW_HIP(sw_launch_unfused(b, f, s));
            cur ^= 1;
        }
        return SW_OK;
    }
    if (tun.variant == 6) {   // generated kernel; boundary values applied outside it, as in the paper
        for (; n < nsteps; ++n) {
            SwLaunch b = launch_of(ctx, state, cur);
            b.step = n;
            SW_HIP(sw_launch_rgn(b, tun.vec, tun.rows, tun.pd, s));
            SW_HIP(sw_launch_fill_halo(launch_of(ctx, state, cur ^ 1), s));
            cur ^= 1;
        }
        return SW_OK;
    }
    if (tun.variant == 5) {
        const size_t vb = 4 * eb, buf = aos_elems(ctx) * vb;
        char *aos[2] = {(char *)ctx->ws, (char *)ctx->ws + buf};
        const int64_t row = ctx->layout.plane_offset, rows = (int64_t)ctx->grid.ny + 2;
        const int64_t aos_origin = row + (ctx->layout.origin - ctx->layout.pitch);   // cell (0, 0) in an AoS copy
        SW_HIP(sw_launch_aos_convert((int)ctx->opts.dtype, state->plane[cur], ctx->layout.pitch, aos[0], row, rows,
                                     true, s));
        for (; n < nsteps; ++n) {
            SwLaunch b = launch_of(ctx, state, cur);
            b.step = n;
            b.pitch = row;   // the step reads and writes only the AoS copies
            SW_HIP(sw_launch_aos_step(b, aos[n & 1] + aos_origin * vb, aos[(n + 1) & 1] + aos_origin * vb, tun.rows, s));
        }
        SW_HIP(sw_launch_aos_convert((int)ctx->opts.dtype, state->plane[cur ^ (nsteps & 1)], ctx->layout.pitch,
                                     aos[nsteps & 1], row, rows, false, s));
        return SW_OK;
    }
    if (tun.variant == 3) {   // K steps per launch (K odd: one buffer flip per launch, as K single steps)
        for (; n + tun.rows <= nsteps; n += tun.rows) {
            SwLaunch b = launch_of(ctx, state, cur);
            b.step = n;
            SW_HIP(sw_launch_tb(b, tun.rows, tun.vec, s));
            cur ^= 1;
        }
    }
    SwTuning single = tun;    // the remaining steps: the fused kernel in its default shape
    if (tun.variant == 3) {
        single.variant = 2;
        single.vec = sw_fused_default_vec((int)ctx->opts.dtype, ctx->grid.nx);
        single.rows = sw_fused_default_rows(ctx->grid.nx, ctx->grid.ny, single.vec);
        single.minw = 0;
        single.pd = 2;
        single.order = 0;
    }
    // With reflective walls on both axes and the width a multiple of the
    // cells per lane, the paper's scheme reads no ghost cell (the walls'
    // images are formed from the edge cells; a width that is not a multiple
    // puts the right ghost inside a lane's vector, which is read), so only
    // the call's last step writes them.
    const bool ghost_free = ctx->opts.scheme == SW_SCHEME_PAPER && ctx->opts.bc_x == SW_BC_REFLECT &&
                            ctx->opts.bc_y == SW_BC_REFLECT && single.vec > 0 && ctx->grid.nx % single.vec == 0;
    for (; n < nsteps; ++n) {
        SwLaunch b = launch_of(ctx, state, cur);
        b.step = n;
        b.ghosts = ghost_free && n + 1 < nsteps ? 0 : 1;
        SW_HIP(sw_launch_step(b, single, s));
        cur ^= 1;
    }
    return SW_OK;
}

void drop_graphs(sw_ctx *ctx) {
    for (auto &g : ctx->graphs) (void)hipGraphExecDestroy(g.exec);
    ctx->graphs.clear();
}

}  // namespace

sw_status sw_ctx_describe(const sw_ctx *ctx, sw_grid *grid, sw_opts *opts, sw_layout *layout, void **scalars,
                          size_t *scalars_bytes) {
    if (!ctx) return fail(SW_EINVAL, "NULL context");
    *grid = ctx->grid;
    *opts = ctx->opts;
    *layout = ctx->layout;
    *scalars = ctx->sc;
    *scalars_bytes = sizeof(SwScalars);
    return use_device(ctx);
}

// Shared with the batched mode: record an error detail and return the status.
sw_status sw_fail(sw_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vfail(s, fmt, ap);
    va_end(ap);
    return s;
}

// Validate one grid's creation arguments (no HIP call); resolve the options
// (defaults, dy) and compute the layout.
sw_status sw_validate_opts(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts, sw_opts *resolved,
                           sw_layout *layout) {
    sw_opts o;
    if (opts) {
        o = *opts;
    } else {
        o.dtype = SW_F32;
        o.bc_x = o.bc_y = SW_BC_REFLECT;
        o.scheme = SW_SCHEME_PAPER;
        o.dy = 0.0;
        o.cfl = 0.5;
        o.dt_fixed = 0.0;
    }
    sw_status st = layout_for(grid, o.dtype, layout);
    if (st != SW_OK) return st;
    if (!(g > 0) || !(dx > 0)) return fail(SW_EINVAL, "create: g = %g and dx = %g must be > 0", g, dx);
    o.dy = o.dy > 0 ? o.dy : dx;
    if ((o.bc_x != SW_BC_REFLECT && o.bc_x != SW_BC_PERIODIC) || (o.bc_y != SW_BC_REFLECT && o.bc_y != SW_BC_PERIODIC))
        return fail(SW_EINVAL, "create: unknown boundary condition");
    if (o.scheme != SW_SCHEME_PAPER && o.scheme != SW_SCHEME_TRANSVERSE)
        return fail(SW_EINVAL, "create: unknown scheme %d", (int)o.scheme);
    if ((o.cfl > 0) == (o.dt_fixed > 0))
        return fail(SW_EINVAL, "create: exactly one of cfl (%g) and dt_fixed (%g) must be > 0", o.cfl, o.dt_fixed);
    if (!(o.cfl >= 0) || !(o.dt_fixed >= 0)) return fail(SW_EINVAL, "create: cfl / dt_fixed not a number");
    if (halo.left < 0 || halo.right < 0 || halo.down < 0 || halo.up < 0)
        return fail(SW_EINVAL, "create: negative halo width");
    if (halo.left != 1 || halo.right != 1 || halo.down != 1 || halo.up != 1)
        return fail(SW_ENOTSUP, "create: halo [%d,%d,%d,%d]; the scheme uses [1,1,1,1]", halo.left, halo.right,
                    halo.down, halo.up);
    *resolved = o;
    return SW_OK;
}

extern "C" {

const char *sw_strerror(sw_status s) {
    switch (s) {
        case SW_OK: return "ok";
        case SW_EINVAL: return "invalid argument";
        case SW_ENOTSUP: return "not supported";
        case SW_ENOMEM: return "out of memory";
        case SW_EHIP: return "HIP runtime error";
        case SW_EUNSTABLE: return "unstable: h <= 0 or non-finite value";
    }
    return "unknown status";
}

const char *sw_last_error_detail(void) { return g_detail.c_str(); }

sw_status sw_layout_query(sw_grid grid, sw_dtype dtype, sw_layout *out) { return layout_for(grid, dtype, out); }

sw_status sw_create(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts, sw_ctx **out) {
    if (!out) return fail(SW_EINVAL, "create: NULL output");
    *out = nullptr;
    sw_opts o;
    sw_layout lay;
    sw_status st = sw_validate_opts(grid, halo, g, dx, opts, &o, &lay);
    if (st != SW_OK) return st;
    const double dy = o.dy;
    sw_ctx *c = new (std::nothrow) sw_ctx{};
    if (!c) return fail(SW_ENOMEM, "create: host allocation");
    c->grid = grid;
    c->opts = o;
    c->opts.dy = dy;
    c->g = g;
    c->dx = dx;
    c->dy = dy;
    c->layout = lay;
    c->tuning = sw_tuning{0, 0, 0, 0, 0, 0};
    hipError_t e = hipGetDevice(&c->device);
    if (e == hipSuccess) e = hipMalloc((void **)&c->sc, sizeof(SwScalars));
    if (e == hipSuccess) e = hipMemset(c->sc, 0, sizeof(SwScalars));
    if (e == hipSuccess) e = hipMalloc((void **)&c->diag, sw_diag_scratch_bytes());
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->cap, hipStreamNonBlocking);
    if (e != hipSuccess) {
        if (c->sc) (void)hipFree(c->sc);
        if (c->diag) (void)hipFree(c->diag);
        if (c->cap) (void)hipStreamDestroy(c->cap);
        delete c;
        return fail(e == hipErrorOutOfMemory ? SW_ENOMEM : SW_EHIP, "create: %s", hipGetErrorString(e));
    }
    *out = c;
    return SW_OK;
}

sw_status sw_destroy(sw_ctx *ctx) {
    if (!ctx) return SW_OK;
    (void)use_device(ctx);
    drop_graphs(ctx);
    if (ctx->ws) (void)hipFree(ctx->ws);
    if (ctx->diag) (void)hipFree(ctx->diag);
    if (ctx->cap) (void)hipStreamDestroy(ctx->cap);
    if (ctx->sc) (void)hipFree(ctx->sc);
    delete ctx;
    return SW_OK;
}

sw_status sw_get_layout(const sw_ctx *ctx, sw_layout *out) {
    if (!ctx || !out) return fail(SW_EINVAL, "get_layout: NULL argument");
    *out = ctx->layout;
    return SW_OK;
}

namespace {
constexpr int kRgnDefaultPrefetch = 1;   // generated row march: input rows loaded ahead by default

// Resolve defaults; returns SW_OK or an error for unsupported settings.
sw_status resolve_tuning(const sw_ctx *ctx, const sw_tuning &in, SwTuning *out) {
    int variant = in.variant;
    if (variant < 0 || variant > 6) return fail(SW_EINVAL, "tuning: unknown variant %d", variant);
    if (variant == 0) variant = 2;
    if (variant >= 3 && ctx->opts.scheme != SW_SCHEME_PAPER)
        return fail(SW_ENOTSUP, "tuning: the blocked, unfused, AoS and generated kernels implement the paper scheme only");
    if (variant == 4) {
        *out = SwTuning{4, 0, 0, 0, 0, 0};
        return SW_OK;
    }
    if (variant == 6) {
        const int design = in.vec ? in.vec : 2;
        const int rows = in.rows ? in.rows : (design == 2 ? 16 : 8);
        if (!sw_rgn_rows_supported(design, rows))
            return fail(SW_EINVAL, "tuning: generated kernel has no design %d with %d rows (design 1: 4, 8 or 16; "
                        "design 2: 4, 8, 16 or 32)", design, rows);
        if (design == 1 && (ctx->grid.ny + rows - 1) / rows > 65535)
            return fail(SW_ENOTSUP, "tuning: %d rows exceed the generated kernel's 65535 tile rows of %d",
                        ctx->grid.ny, rows);
        // row march: input rows loaded ahead of the row being updated (1 = none beyond the ring)
        const int pf = design == 2 ? (in.prefetch ? in.prefetch : kRgnDefaultPrefetch) : in.prefetch;
        if (design == 2 ? (pf < 1 || pf > 3) : pf != 0)
            return fail(SW_EINVAL, "tuning: generated design %d takes prefetch %s", design,
                        design == 2 ? "1, 2 or 3" : "0");
        *out = SwTuning{6, rows, design, 0, pf, 0};
        return SW_OK;
    }
    if (variant == 5) {
        if (in.rows < 0) return fail(SW_EINVAL, "tuning: rows = %d", in.rows);
        *out = SwTuning{5, in.rows ? in.rows : 8, 1, 0, 0, 0};
        return SW_OK;
    }
    if (variant == 3) {
        if (!(ctx->opts.dt_fixed > 0))
            return fail(SW_ENOTSUP, "tuning: temporal blocking needs a fixed dt (a CFL dt depends on every cell)");
        const int k = in.rows ? in.rows : 5;
        if (!sw_tb_supported((int)ctx->opts.dtype, k))
            return fail(SW_EINVAL, "tuning: %d steps per blocked launch not available for this dtype", k);
        if ((ctx->grid.ny + sw_tb_tile_rows((int)ctx->opts.dtype, k) - 1) / sw_tb_tile_rows((int)ctx->opts.dtype, k) >
            65535)
            return fail(SW_ENOTSUP, "tuning: %d rows exceed the blocked kernel's 65535 tile rows of %d", ctx->grid.ny,
                        sw_tb_tile_rows((int)ctx->opts.dtype, k));
        const int waves = in.vec ? in.vec : (ctx->opts.dtype == SW_F64 ? 8 : 16);
        if (waves != 4 && waves != 8 && waves != 12 && waves != 16)
            return fail(SW_EINVAL, "tuning: %d waves per blocked tile (4, 8, 12 or 16)", waves);
        *out = SwTuning{3, k, waves, 0, 0, 0};
        return SW_OK;
    }
    out->variant = variant;
    out->vec = in.vec ? in.vec : sw_fused_default_vec((int)ctx->opts.dtype, ctx->grid.nx);
    out->rows = in.rows ? in.rows : sw_fused_default_rows(ctx->grid.nx, ctx->grid.ny, out->vec);
    out->minw = in.occupancy;
    out->pd = in.prefetch ? in.prefetch : 2;
    out->order = in.order;
    if (in.order < 0 || in.order > 2) return fail(SW_EINVAL, "tuning: order = %d", in.order);
    if (in.rows < 0) return fail(SW_EINVAL, "tuning: rows = %d", in.rows);
    if (variant == 2 && !sw_fused_supported((int)ctx->opts.dtype, (int)ctx->opts.scheme, out->vec, out->minw, out->pd))
        return fail(SW_EINVAL, "tuning: vec %d / occupancy %d / prefetch %d not available for this dtype", out->vec,
                    out->minw, out->pd);
    // the fused kernel reaches a tile's rows through 32-bit buffer offsets
    if (variant == 2 && !sw_fused_tile_fits(out->rows, ctx->layout.pitch, ctx->layout.elem_bytes))
        return fail(SW_EINVAL, "tuning: %d rows per tile of %lld-element rows exceed the fused kernel's 2 GiB tile span",
                    out->rows, (long long)ctx->layout.pitch);
    return SW_OK;
}
}  // namespace

sw_status sw_set_variant(sw_ctx *ctx, int32_t variant) {
    if (!ctx) return fail(SW_EINVAL, "set_variant: NULL context");
    if (variant < 0 || variant > 6) return fail(SW_EINVAL, "set_variant: unknown variant %d", variant);
    sw_tuning t = ctx->tuning;
    t.variant = variant;
    SwTuning r;
    sw_status st = resolve_tuning(ctx, t, &r);
    if (st != SW_OK && st != SW_ENOTSUP) return st;
    ctx->tuning = t;
    return SW_OK;
}

sw_status sw_set_tuning(sw_ctx *ctx, const sw_tuning *tuning) {
    if (!ctx || !tuning) return fail(SW_EINVAL, "set_tuning: NULL argument");
    SwTuning r;
    sw_status st = resolve_tuning(ctx, *tuning, &r);
    if (st != SW_OK) return st;
    ctx->tuning = *tuning;
    return SW_OK;
}

sw_status sw_get_tuning(const sw_ctx *ctx, sw_tuning *out) {
    if (!ctx || !out) return fail(SW_EINVAL, "get_tuning: NULL argument");
    SwTuning r;
    sw_status st = resolve_tuning(ctx, ctx->tuning, &r);
    if (st != SW_OK) return st;
    *out = sw_tuning{r.variant, r.rows, r.vec, r.minw, r.pd, r.order};
    return SW_OK;
}

sw_status sw_fill_halo(sw_ctx *ctx, const sw_state *state, void *stream) {
    if (!ctx) return fail(SW_EINVAL, "fill_halo: NULL context");
    sw_status st = check_state(ctx, state, false);
    if (st != SW_OK) return st;
    if ((st = use_device(ctx)) != SW_OK) return st;
    SwLaunch a = launch_of(ctx, state, state->cur);
    SW_HIP(sw_launch_fill_halo(a, (hipStream_t)stream));
    return SW_OK;
}

sw_status sw_step(sw_ctx *ctx, sw_state *state, int32_t nsteps, void *stream) {
    if (!ctx) return fail(SW_EINVAL, "step: NULL context");
    if (nsteps < 0) return fail(SW_EINVAL, "step: nsteps = %d < 0", nsteps);
    sw_status st = check_state(ctx, state, true);
    if (st != SW_OK) return st;
    if (nsteps == 0) return SW_OK;
    if ((st = use_device(ctx)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    SwTuning tun;
    if ((st = resolve_tuning(ctx, ctx->tuning, &tun)) != SW_OK) return st;
    const size_t need = workspace_bytes(ctx, tun.variant);
    if (need > ctx->ws_bytes) {            // before any capture: graphs hold the old address
        drop_graphs(ctx);
        SW_HIP(hipStreamSynchronize(s));
        if (ctx->ws) SW_HIP(hipFree(ctx->ws));
        ctx->ws = nullptr;
        ctx->ws_bytes = 0;
        hipError_t e = hipMalloc(&ctx->ws, need);
        if (e != hipSuccess) {
            ctx->ws = nullptr;
            return fail(e == hipErrorOutOfMemory ? SW_ENOMEM : SW_EHIP, "step: workspace of %zu bytes: %s", need,
                        hipGetErrorString(e));
        }
        ctx->ws_bytes = need;
    }
    if (!ctx->use_graph) {
        if ((st = enqueue_steps(ctx, state, nsteps, tun, s)) != SW_OK) return st;
    } else {
        hipGraphExec_t exec = nullptr;
        for (auto &gr : ctx->graphs)
            if (gr.nsteps == nsteps && gr.cur == state->cur && std::memcmp(gr.planes, state->plane, sizeof gr.planes) == 0 &&
                std::memcmp(&gr.tun, &tun, sizeof tun) == 0)
                exec = gr.exec;
        if (!exec) {
            if (ctx->graphs.size() >= 8) drop_graphs(ctx);
            SW_HIP(hipStreamBeginCapture(ctx->cap, hipStreamCaptureModeThreadLocal));
            st = enqueue_steps(ctx, state, nsteps, tun, ctx->cap);
            hipGraph_t graph = nullptr;
            hipError_t e = hipStreamEndCapture(ctx->cap, &graph);
            if (st != SW_OK) {
                if (graph) (void)hipGraphDestroy(graph);
                return st;
            }
            if (e != hipSuccess) return fail(SW_EHIP, "step: capture: %s", hipGetErrorString(e));
            e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (e != hipSuccess) return fail(SW_EHIP, "step: instantiate: %s", hipGetErrorString(e));
            sw_ctx::Graph gr{nsteps, state->cur, {}, tun, exec};
            std::memcpy(gr.planes, state->plane, sizeof gr.planes);
            ctx->graphs.push_back(gr);
        }
        SW_HIP(hipGraphLaunch(exec, s));
    }
    state->cur ^= (nsteps & 1);
    return SW_OK;
}

sw_status sw_set_graph(sw_ctx *ctx, int32_t enable) {
    if (!ctx) return fail(SW_EINVAL, "set_graph: NULL context");
    ctx->use_graph = enable != 0;
    return SW_OK;
}

sw_status sw_sync_status(sw_ctx *ctx, void *stream, double *t, double *last_dt, int64_t *steps) {
    if (!ctx) return fail(SW_EINVAL, "sync_status: NULL context");
    sw_status st = use_device(ctx);
    if (st != SW_OK) return st;
    SW_HIP(hipStreamSynchronize((hipStream_t)stream));
    SwScalars h;
    SW_HIP(hipMemcpy(&h, ctx->sc, sizeof h, hipMemcpyDeviceToHost));
    if (t) *t = h.t;
    if (last_dt) *last_dt = h.last_dt;
    if (steps) *steps = h.steps;
    if (h.unstable) return fail(SW_EUNSTABLE, "a step produced h <= 0 or a non-finite value");
    return SW_OK;
}

sw_status sw_diagnostics(sw_ctx *ctx, const sw_state *state, void *stream, double out[6]) {
    if (!ctx || !out) return fail(SW_EINVAL, "diagnostics: NULL argument");
    sw_status st = check_state(ctx, state, false);
    if (st != SW_OK) return st;
    if ((st = use_device(ctx)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    SW_HIP(sw_launch_diagnostics(launch_of(ctx, state, state->cur), ctx->diag, s));
    const size_t nres = sw_diag_scratch_bytes() / sizeof(double);
    SW_HIP(hipMemcpyAsync(out, ctx->diag + nres - 6, 6 * sizeof(double), hipMemcpyDeviceToHost, s));
    SW_HIP(hipStreamSynchronize(s));
    return SW_OK;
}

sw_status sw_reset_time(sw_ctx *ctx, void *stream) {
    if (!ctx) return fail(SW_EINVAL, "reset_time: NULL context");
    sw_status st = use_device(ctx);
    if (st != SW_OK) return st;
    SW_HIP(sw_launch_reset(ctx->sc, 1, (hipStream_t)stream));
    return SW_OK;
}

}  // extern "C"

bool sw_ctx_use_graph(const sw_ctx *ctx) { return ctx && ctx->use_graph; }

void sw_ctx_drop_graphs(sw_ctx *ctx) {
    if (ctx) drop_graphs(ctx);
}
