// sw_step_noalloc: the time-step call without a context, for callers that
// cannot allocate device memory.  The device scalars a step sequence needs
// (the CFL ring, time, step count, sticky flag: one SwScalars) live in a
// file-scope device array instead of a context's allocation; everything else
// is the caller's (state buffers, optional status output).  Kernels and
// launch shape are those of sw_step with the default tuning, launched
// eagerly, so the results are bitwise those of sw_create + sw_step.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <mutex>

#include "../../include/sw.h"
#include "sw_internal.h"

sw_status sw_fail(sw_status s, const char *fmt, ...);
sw_status sw_validate_opts(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts, sw_opts *resolved,
                           sw_layout *layout);

// Bytes of the per-device scratch: one SwScalars (the same for every grid size).
constexpr size_t kScratchBytes = 2048;
static_assert(sizeof(SwScalars) <= kScratchBytes, "the no-alloc scratch must hold the step scalars");

// Each device holds its own copy until the process ends.  Host code never
// passes this name to a kernel or a copy: it uses the address
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_ptr[kMaxDevices];   // device address of `scratch` per device (null until resolved)

// Address of the current device's scratch, resolved once per device with that
// device current.
sw_status scratch_ptr(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return sw_fail(SW_EHIP, "step_noalloc: hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return sw_fail(SW_ENOTSUP, "step_noalloc: device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_ptr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sw_fail(SW_EHIP, "step_noalloc: hipGetSymbolAddress: %s", hipGetErrorString(e));
        g_ptr[dev] = p;
    }
    *out = g_ptr[dev];
    return SW_OK;
}

// status[0..3] = time, last dt, steps, sticky flag of this call.
__global__ void k_noalloc_status(const SwScalars *sc, double *status) {
    if (threadIdx.x == 0) {
        status[0] = sc->t;
        status[1] = sc->last_dt;
        status[2] = (double)sc->steps;
        status[3] = sc->unstable ? 1.0 : 0.0;
    }
}

}  // namespace

extern "C" sw_status sw_step_noalloc(sw_grid grid, sw_halo halo, double g, double dx, const sw_opts *opts,
                                     sw_state *state, int32_t nsteps, double *status, void *stream) {
    sw_opts o;
    sw_layout lay;
    sw_status st = sw_validate_opts(grid, halo, g, dx, opts, &o, &lay);
    if (st != SW_OK) return st;
    if (!state) return sw_fail(SW_EINVAL, "step_noalloc: NULL state");
    if (nsteps < 0) return sw_fail(SW_EINVAL, "step_noalloc: nsteps = %d < 0", nsteps);
    if (state->cur != 0 && state->cur != 1) return sw_fail(SW_EINVAL, "step_noalloc: cur = %d", state->cur);
    for (int b = 0; b < 2; ++b)
        for (int k = 0; k < 3; ++k) {
            const void *p = state->plane[b][k];
            if (!p || (uintptr_t)p % 256)
                return sw_fail(SW_EINVAL, "step_noalloc: plane[%d][%d] NULL or not 256-byte aligned", b, k);
            for (int m = 0; m < 3; ++m)
                if (b == 0 && p == state->plane[1][m])
                    return sw_fail(SW_EINVAL, "step_noalloc: buffers 0 and 1 share plane memory");
        }
    if ((uintptr_t)status % 8) return sw_fail(SW_EINVAL, "step_noalloc: status not 8-byte aligned");
    // the default launch shape of sw_step
    SwTuning tun{2, 0, 0, 0, 2, 0};
    tun.vec = sw_fused_default_vec((int)o.dtype, grid.nx);
    tun.rows = sw_fused_default_rows(grid.nx, grid.ny, tun.vec);
    if (!sw_fused_supported((int)o.dtype, (int)o.scheme, tun.vec, tun.minw, tun.pd) ||
        !sw_fused_tile_fits(tun.rows, lay.pitch, lay.elem_bytes))
        return sw_fail(SW_ENOTSUP, "step_noalloc: no default fused shape for this grid");
    void *sp = nullptr;
    if ((st = scratch_ptr(&sp)) != SW_OK) return st;
    SwScalars *sc = (SwScalars *)sp;
    hipStream_t s = (hipStream_t)stream;

    auto launch_of = [&](int from, int step) {
        SwLaunch a{};
        for (int k = 0; k < 3; ++k) {
            a.in[k] = (const char *)state->plane[from][k] + lay.origin * lay.elem_bytes;
            a.out[k] = (char *)state->plane[from ^ 1][k] + lay.origin * lay.elem_bytes;
        }
        a.pitch = lay.pitch;
        a.nx = grid.nx;
        a.ny = grid.ny;
        a.g = g;
        a.dx = dx;
        a.dy = o.dy;
        a.cfl = o.cfl;
        a.dt_fixed = o.dt_fixed;
        a.bc_x = (int32_t)o.bc_x;
        a.bc_y = (int32_t)o.bc_y;
        a.scheme = (int32_t)o.scheme;
        a.dtype = (int32_t)o.dtype;
        a.sc = sc;
        a.step = step;
        a.ghosts = 1;
        return a;
    };
#define NA_HIP(call)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (call);                                                                   \
        if (e_ != hipSuccess) return sw_fail(SW_EHIP, "step_noalloc: %s: %s", #call, hipGetErrorString(e_)); \
    } while (0)
    // the previous call's ring, time and flag are cleared by a kernel (no memset node)
    NA_HIP(sw_launch_reset(sc, 1, s));
    int cur = state->cur;
    if (nsteps > 0) {
        NA_HIP(sw_launch_prologue(launch_of(cur, 0), s));
        for (int n = 0; n < nsteps; ++n) {
            NA_HIP(sw_launch_step(launch_of(cur, n), tun, s));
            cur ^= 1;
        }
    }
    if (status) {
        k_noalloc_status<<<1, 64, 0, s>>>(sc, status);
        NA_HIP(hipGetLastError());
    }
#undef NA_HIP
    state->cur = cur;
    return SW_OK;
}
