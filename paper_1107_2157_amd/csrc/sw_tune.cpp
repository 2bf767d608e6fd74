// Autotuner of the step kernel's launch shape.
//
// Candidates (fused kernel): cells per lane x register budget x prefetch
// depth x rows per tile x tile order.  Each candidate is timed with HIP
// events on the caller's stream over a few steps of the caller's own state,
// as replays of sw_step's graphs; the state (buf[cur] with its halo)
// and the context's time scalars are saved first and restored before every
// trial and at the end, so tuning leaves the simulation where it was.  Every
// fused shape produces bitwise identical cells, so the choice affects speed
// only.  With a fixed dt the temporally blocked kernel (K steps per launch,
// 8, 12 or 16 waves per tile) joins the candidates; it too reproduces the
// fused kernel's bits.  Results are cached in a text file, one line per key
//   <arch>:<CUs>:<dtype>:<scheme>:<nx>x<ny>[:fixeddt] variant rows vec occupancy prefetch order us_per_step
// (the suffix marks contexts with a fixed dt, whose choice may be a blocked
// launch that a CFL-dt context cannot use).
#include <hip/hip_runtime.h>

#include <algorithm>

#include <cstdio>
#include <cstring>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/sw.h"
#include "sw_internal.h"

namespace {

std::string tune_key(sw_dtype dtype, sw_scheme scheme, int nx, int ny, bool fixed_dt, int device) {
    hipDeviceProp_t prop;
    std::string arch = "unknown";
    int cus = 0;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) {
        arch = prop.gcnArchName;
        auto colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
        cus = prop.multiProcessorCount;
    }
    std::ostringstream k;
    k << arch << ":" << cus << ":" << (dtype == SW_F64 ? "f64" : "f32") << ":" << (int)scheme << ":" << nx << "x"
      << ny;
    if (fixed_dt) k << ":fixeddt";
    return k.str();
}

bool cache_lookup(const char *path, const std::string &key, sw_tuning *t) {
    if (!path || !*path) return false;
    std::ifstream f(path);
    std::string line;
    bool found = false;
    while (std::getline(f, line)) {
        std::istringstream is(line);
        std::string k;
        sw_tuning c{};
        double us;
        if (is >> k >> c.variant >> c.rows >> c.vec >> c.occupancy >> c.prefetch >> c.order >> us && k == key) {
            *t = c;       // the last entry for a key wins
            found = true;
        }
    }
    return found;
}

void cache_store(const char *path, const std::string &key, const sw_tuning &t, double us) {
    if (!path || !*path) return;
    std::ofstream f(path, std::ios::app);
    f << key << " " << t.variant << " " << t.rows << " " << t.vec << " " << t.occupancy << " " << t.prefetch << " "
      << t.order << " " << us << "\n";
}

}  // namespace

// Context accessor (sw_api.cpp).
sw_status sw_ctx_describe(const sw_ctx *ctx, sw_grid *grid, sw_opts *opts, sw_layout *layout, void **scalars,
                          size_t *scalars_bytes);

bool sw_ctx_use_graph(const sw_ctx *ctx);
void sw_ctx_drop_graphs(sw_ctx *ctx);   // the context's captured graphs (none may be in flight)

extern "C" sw_status sw_autotune(sw_ctx *ctx, sw_state *state, int32_t steps_per_trial, const char *cache_path,
                                 void *stream, sw_tuning *best_out) {
    sw_grid grid;
    sw_opts opts;
    sw_layout lay;
    void *scal = nullptr;
    size_t scal_bytes = 0;
    sw_status st = sw_ctx_describe(ctx, &grid, &opts, &lay, &scal, &scal_bytes);
    if (st != SW_OK) return st;
    if (!state || steps_per_trial < 1) return SW_EINVAL;
    hipStream_t s = (hipStream_t)stream;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return SW_EHIP;
    const std::string key = tune_key(opts.dtype, opts.scheme, grid.nx, grid.ny, opts.dt_fixed > 0, device);

    sw_tuning best{};
    if (cache_lookup(cache_path, key, &best) && sw_set_tuning(ctx, &best) == SW_OK) {
        if (best_out) sw_get_tuning(ctx, best_out);
        return SW_OK;
    }

    std::vector<sw_tuning> cands;
    {
        const int vecs_f32[] = {1, 2, 4}, vecs_f64[] = {1, 2};
        const int *vecs = opts.dtype == SW_F64 ? vecs_f64 : vecs_f32;
        const int nvec = opts.dtype == SW_F64 ? 2 : 3;
        const int rows_list[] = {2, 4, 8, 16, 32, 64, 128};
        const int occs[] = {0, 3, 4};
        for (int vi = 0; vi < nvec; ++vi)
            for (int occ : occs)
                for (int pd = 1; pd <= 3; ++pd)
                    if (sw_fused_supported((int)opts.dtype, (int)opts.scheme, vecs[vi], occ, pd))
                        for (int rows : rows_list)
                            for (int order = 0; order <= 1; ++order)
                                cands.push_back(sw_tuning{2, rows, vecs[vi], occ, pd, order});
        if (opts.dt_fixed > 0 && opts.scheme == SW_SCHEME_PAPER)   // temporal blocking: K steps per launch
            for (int k : {3, 5, 7})
                for (int waves : {8, 12, 16})
                    if (sw_tb_supported((int)opts.dtype, k)) cands.push_back(sw_tuning{3, k, waves, 0, 0, 0});
    }

    // save buf[cur] (every row of each plane, halo included) and the time scalars
    const size_t eb = (size_t)lay.elem_bytes, row_bytes = (size_t)lay.plane_offset * eb;
    const size_t pitch_bytes = (size_t)lay.pitch * eb, nrows = (size_t)grid.ny + 2;
    const size_t plane_bytes = row_bytes * nrows;
    void *backup = nullptr, *scal_backup = nullptr;
    if (hipMalloc(&backup, 3 * plane_bytes) != hipSuccess) return SW_ENOMEM;
    if (hipMalloc(&scal_backup, scal_bytes) != hipSuccess) {
        (void)hipFree(backup);
        return SW_ENOMEM;
    }
    const int cur0 = state->cur;
    auto save = [&]() -> hipError_t {
        for (int k = 0; k < 3; ++k) {
            hipError_t e = hipMemcpy2DAsync((char *)backup + k * plane_bytes, row_bytes, state->plane[cur0][k],
                                            pitch_bytes, row_bytes, nrows, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        return hipMemcpyAsync(scal_backup, scal, scal_bytes, hipMemcpyDeviceToDevice, s);
    };
    auto restore = [&]() -> hipError_t {
        state->cur = cur0;
        for (int k = 0; k < 3; ++k) {
            hipError_t e = hipMemcpy2DAsync(state->plane[cur0][k], pitch_bytes, (char *)backup + k * plane_bytes,
                                            row_bytes, row_bytes, nrows, hipMemcpyDeviceToDevice, s);
            if (e != hipSuccess) return e;
        }
        return hipMemcpyAsync(scal, scal_backup, scal_bytes, hipMemcpyDeviceToDevice, s);
    };

    sw_tuning prev{};
    sw_get_tuning(ctx, &prev);
    // trials replay graphs, as sw_step runs: eager launches would time the
    // host's launch rate on small grids; each shape's two call lengths are
    // captured in an untimed warm-up first
    const bool graph = sw_ctx_use_graph(ctx);
    sw_set_graph(ctx, 1);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    double best_us = 1e300;
    hipError_t he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    if (he == hipSuccess) he = save();
    for (size_t i = 0; i < cands.size() && he == hipSuccess; ++i) {
        if (sw_set_tuning(ctx, &cands[i]) != SW_OK) continue;
        // room for this shape's two graphs (the cache evicts all when full);
        // the previous trial ended with an event synchronisation
        sw_ctx_drop_graphs(ctx);
        // blocked candidates: a whole number of K-step launches in the difference
        const int kt = cands[i].variant == 3 ? cands[i].rows * steps_per_trial : steps_per_trial;
        if ((he = restore()) != hipSuccess) break;
        if (sw_step(ctx, state, 1, stream) != SW_OK) continue;        // capture + warm (code load, caches)
        if (sw_step(ctx, state, 1 + kt, stream) != SW_OK) continue;
        if ((he = restore()) != hipSuccess) break;
        // per-step time = (T(1 + k) - T(1)) / k: the per-call prologue cancels;
        // the best of two runs of each length (a single run's launch jitter is
        // a percent of a short run)
        float ms1 = 1e30f, msk = 1e30f;
        bool ran = true;
        for (int rep = 0; rep < 2 && ran && he == hipSuccess; ++rep) {
            float a1 = 0.f, ak = 0.f;
            if (rep > 0 && (he = restore()) != hipSuccess) break;
            if ((he = hipEventRecord(e0, s)) != hipSuccess) break;
            if (sw_step(ctx, state, 1, stream) != SW_OK) { ran = false; break; }
            if ((he = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
            if ((he = hipEventElapsedTime(&a1, e0, e1)) != hipSuccess) break;
            if ((he = hipEventRecord(e0, s)) != hipSuccess) break;
            if (sw_step(ctx, state, 1 + kt, stream) != SW_OK) { ran = false; break; }
            if ((he = hipEventRecord(e1, s)) != hipSuccess) break;
            if ((he = hipEventSynchronize(e1)) != hipSuccess) break;
            if ((he = hipEventElapsedTime(&ak, e0, e1)) != hipSuccess) break;
            ms1 = std::min(ms1, a1);
            msk = std::min(msk, ak);
        }
        if (he != hipSuccess) break;
        if (!ran) continue;
        double us = 1000.0 * (msk - ms1) / kt;
        if (us < best_us) {
            best_us = us;
            best = cands[i];
        }
    }
    if (he == hipSuccess) he = restore();
    if (he == hipSuccess) he = hipStreamSynchronize(s);
    sw_ctx_drop_graphs(ctx);                 // the trial shapes' graphs
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(backup);
    (void)hipFree(scal_backup);
    sw_set_graph(ctx, graph ? 1 : 0);
    if (he != hipSuccess) {
        sw_set_tuning(ctx, &prev);
        return SW_EHIP;
    }
    if (best_us >= 1e300) {
        sw_set_tuning(ctx, &prev);
        return SW_ENOTSUP;
    }
    sw_set_tuning(ctx, &best);
    cache_store(cache_path, key, best, best_us);
    if (best_out) sw_get_tuning(ctx, best_out);
    return SW_OK;
}
