// libsw HIP kernels (gfx950): context reset, CFL prologue with halo fill,
// stand-alone halo fill, and the per-cell baseline step.
#include "sw_common.h"

using namespace sw;

namespace {

__global__ void k_reset(SwScalars *sc, int clear_time) {
    if (threadIdx.x < 3 * kStripes) sc->smax[threadIdx.x / kStripes][threadIdx.x % kStripes] = 0ull;
    if (threadIdx.x == 0) {
        if (clear_time) {
            sc->t = 0.0;
            sc->last_dt = 0.0;
            sc->steps = 0;
            sc->unstable = 0u;
        }
    }
}

// Fill the halo of the buffer from its interior and max-reduce the interior
// signal speed into ring slot 0 (the dt of the first step of a call).
template <typename T>
__global__ __launch_bounds__(256) void k_prologue(SwLaunch a) {
    T *P[3] = {(T *)a.in[0], (T *)a.in[1], (T *)a.in[2]};
    const int nx = a.nx, ny = a.ny;
    const int64_t n = (int64_t)nx * ny;
    const T g = (T)a.g;
    double smax = 0.0;
    bool bad = false;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n;
         idx += (int64_t)gridDim.x * blockDim.x) {
        int j = (int)(idx / nx), i = (int)(idx - (int64_t)j * nx);
        int64_t off = (int64_t)j * a.pitch + i;
        U3<T> c = {P[0][off], P[1][off], P[2][off]};
        T s = signal_speed(c, g);
        bad |= !(s <= finite_max<T>());
        smax = fmax(smax, (double)s);
        if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1)
            write_ghosts(P, a.pitch, nx, ny, a.bc_x, a.bc_y, i, j, c);
    }
    reduce_speed(a.sc, 0, (int)(blockIdx.x * 4 + (threadIdx.x >> 6)), smax, bad);
}

// Halo only: one thread per perimeter cell (corner cells appear twice and
// write identical values).
template <typename T>
__global__ __launch_bounds__(256) void k_fill_halo(SwLaunch a) {
    T *P[3] = {(T *)a.in[0], (T *)a.in[1], (T *)a.in[2]};
    const int nx = a.nx, ny = a.ny;
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    int i, j;
    if (t < nx) { i = t; j = 0; }
    else if (t < 2 * nx) { i = t - nx; j = ny - 1; }
    else if (t < 2 * nx + ny) { i = 0; j = t - 2 * nx; }
    else if (t < 2 * nx + 2 * ny) { i = nx - 1; j = t - 2 * nx - ny; }
    else return;
    int64_t off = (int64_t)j * a.pitch + i;
    U3<T> c = {P[0][off], P[1][off], P[2][off]};
    write_ghosts(P, a.pitch, nx, ny, a.bc_x, a.bc_y, i, j, c);
}

// Baseline step: one thread per interior cell, neighbours read straight from
// global memory, each face computed by both cells that share it.  64 x 4
// threads per block, each thread doing CELL_ROWS cells 4 rows apart.
constexpr int CELL_ROWS = 4;
template <typename T, int TRANS>
__global__ __launch_bounds__(256) void k_step_cell(SwLaunch a) {
    const int i = blockIdx.x * 64 + (threadIdx.x & 63);
    const double dt = step_dt(a);
    const T k = (T)(0.5 * a.g), g = (T)a.g;
    const T lx = (T)(0.5 * dt / a.dx), ly = (T)(0.5 * dt / a.dy);
    const T mx = (T)(dt / a.dx), my = (T)(dt / a.dy);
    const T lx4 = (T)(0.125 * dt / a.dx), ly4 = (T)(0.125 * dt / a.dy);
    const T *I[3] = {(const T *)a.in[0], (const T *)a.in[1], (const T *)a.in[2]};
    T *O[3] = {(T *)a.out[0], (T *)a.out[1], (T *)a.out[2]};
    const int64_t pitch = a.pitch;
    double smax = 0.0;
    bool bad = false;
    for (int rr = 0; rr < CELL_ROWS; ++rr) {
        const int j = (blockIdx.y * CELL_ROWS + rr) * 4 + (threadIdx.x >> 6);
        if (!(i < a.nx && j < a.ny)) continue;
        auto ld = [&](int di, int dj) {
            int64_t off = (int64_t)(j + dj) * pitch + (i + di);
            return U3<T>{I[0][off], I[1][off], I[2][off]};
        };
        U3<T> c = ld(0, 0), w = ld(-1, 0), e = ld(1, 0), s = ld(0, -1), n = ld(0, 1);
        U3<T> Fc = flux_f(c, k), Fw = flux_f(w, k), Fe = flux_f(e, k);
        U3<T> Gc = flux_g(c, k), Gs = flux_g(s, k), Gn = flux_g(n, k);
        U3<T> xl = half_step(w, c, Fw, Fc, lx), xr = half_step(c, e, Fc, Fe, lx);
        U3<T> yd = half_step(s, c, Gs, Gc, ly), yu = half_step(c, n, Gc, Gn, ly);
        if (TRANS) {
            U3<T> sw_ = ld(-1, -1), se = ld(1, -1), nw = ld(-1, 1), ne = ld(1, 1);
            U3<T> Gsw = flux_g(sw_, k), Gse = flux_g(se, k), Gnw = flux_g(nw, k), Gne = flux_g(ne, k);
            U3<T> Gw = flux_g(w, k), Ge = flux_g(e, k);
            U3<T> Fsw = flux_f(sw_, k), Fse = flux_f(se, k), Fnw = flux_f(nw, k), Fne = flux_f(ne, k);
            U3<T> Fs = flux_f(s, k), Fn = flux_f(n, k);
            xl = add_transverse(xl, Gsw, Gs, Gnw, Gn, ly4);
            xr = add_transverse(xr, Gs, Gse, Gn, Gne, ly4);
            yd = add_transverse(yd, Fsw, Fw, Fse, Fe, lx4);
            yu = add_transverse(yu, Fw, Fnw, Fe, Fne, lx4);
        }
        U3<T> FL = flux_f(xl, k), FR = flux_f(xr, k), GD = flux_g(yd, k), GU = flux_g(yu, k);
        U3<T> r = {fma(-my, GU.h - GD.h, fma(-mx, FR.h - FL.h, c.h)),
                   fma(-my, GU.p - GD.p, fma(-mx, FR.p - FL.p, c.p)),
                   fma(-my, GU.q - GD.q, fma(-mx, FR.q - FL.q, c.q))};
        int64_t off = (int64_t)j * pitch + i;
        O[0][off] = r.h; O[1][off] = r.p; O[2][off] = r.q;
        write_ghosts(O, pitch, a.nx, a.ny, a.bc_x, a.bc_y, i, j, r);
        T sp = signal_speed(r, g);
        bad |= !(sp <= finite_max<T>());
        smax = fmax(smax, (double)sp);
    }
    step_epilogue(a, smax, bad, dt, blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x < 64,
                  (int)((blockIdx.y * gridDim.x + blockIdx.x) * 4 + (threadIdx.x >> 6)));
}

template <typename T> hipError_t launch_step_cell(const SwLaunch &a, hipStream_t s) {
    dim3 grid((a.nx + 63) / 64, (a.ny + 4 * CELL_ROWS - 1) / (4 * CELL_ROWS));
    if (a.scheme) k_step_cell<T, 1><<<grid, 256, 0, s>>>(a);
    else k_step_cell<T, 0><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

// Diagnostics of the interior: per block, in a fixed order, the sums of h,
// hu, hv (FP64), the max signal speed, the min h and the count of cells
// with a non-finite value; a second single-block pass combines the
// partials in a fixed order, so the result does not depend on timing.
constexpr int kDiagBlocks = 1024;
constexpr int kDiagThreads = 256;

__device__ __forceinline__ void diag_combine(double *a, const double *b) {
    a[0] += b[0];
    a[1] += b[1];
    a[2] += b[2];
    a[3] = fmax(a[3], b[3]);
    a[4] = fmin(a[4], b[4]);
    a[5] += b[5];
}

// Block reduction of each thread's 6 values in a fixed tree order; thread 0
// ends with the result.
__device__ __forceinline__ void diag_block_reduce(double v[6]) {
    __shared__ double sh[kDiagThreads][6];
    for (int k = 0; k < 6; ++k) sh[threadIdx.x][k] = v[k];
    __syncthreads();
    for (int w = kDiagThreads / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) diag_combine(sh[threadIdx.x], sh[threadIdx.x + w]);
        __syncthreads();
    }
    for (int k = 0; k < 6; ++k) v[k] = sh[0][k];
}

template <typename T>
__global__ __launch_bounds__(kDiagThreads) void k_diag_partial(SwLaunch a, double *part) {
    const T *P[3] = {(const T *)a.in[0], (const T *)a.in[1], (const T *)a.in[2]};
    const int nx = a.nx, ny = a.ny;
    const T g = (T)a.g;
    double v[6] = {0.0, 0.0, 0.0, 0.0, INFINITY, 0.0};
    // block b takes rows b, b + kDiagBlocks, ...; thread t columns t, t + 256, ...
    for (int j = blockIdx.x; j < ny; j += kDiagBlocks) {
        const int64_t row = (int64_t)j * a.pitch;
        for (int i = threadIdx.x; i < nx; i += kDiagThreads) {
            const U3<T> c = {P[0][row + i], P[1][row + i], P[2][row + i]};
            const bool finite = isfinite((double)c.h) && isfinite((double)c.p) && isfinite((double)c.q);
            v[0] += (double)c.h;
            v[1] += (double)c.p;
            v[2] += (double)c.q;
            if (finite && c.h > T(0)) v[3] = fmax(v[3], (double)signal_speed(c, g));
            v[4] = fmin(v[4], (double)c.h);
            v[5] += finite ? 0.0 : 1.0;
        }
    }
    diag_block_reduce(v);
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) part[blockIdx.x * 6 + k] = v[k];
}

__global__ __launch_bounds__(kDiagThreads) void k_diag_final(double *part, double *out) {
    double v[6] = {0.0, 0.0, 0.0, 0.0, INFINITY, 0.0};
    for (int b = threadIdx.x; b < kDiagBlocks; b += kDiagThreads) diag_combine(v, part + b * 6);
    diag_block_reduce(v);
    if (threadIdx.x == 0)
        for (int k = 0; k < 6; ++k) out[k] = v[k];
}

}  // namespace

hipError_t sw_launch_reset(SwScalars *sc, int clear_time, hipStream_t s) {
    k_reset<<<1, 256, 0, s>>>(sc, clear_time);
    return hipGetLastError();
}

hipError_t sw_launch_prologue(const SwLaunch &a, hipStream_t s) {
    int64_t n = (int64_t)a.nx * a.ny;
    int64_t blocks = (n + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    if (a.dtype) k_prologue<double><<<(unsigned)blocks, 256, 0, s>>>(a);
    else k_prologue<float><<<(unsigned)blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t sw_launch_fill_halo(const SwLaunch &a, hipStream_t s) {
    int64_t n = 2 * ((int64_t)a.nx + a.ny);
    unsigned blocks = (unsigned)((n + 255) / 256);
    if (a.dtype) k_fill_halo<double><<<blocks, 256, 0, s>>>(a);
    else k_fill_halo<float><<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

size_t sw_diag_scratch_bytes() { return (size_t)(kDiagBlocks + 1) * 6 * sizeof(double); }

hipError_t sw_launch_diagnostics(const SwLaunch &a, double *scratch, hipStream_t s) {
    if (a.dtype) k_diag_partial<double><<<kDiagBlocks, kDiagThreads, 0, s>>>(a, scratch);
    else k_diag_partial<float><<<kDiagBlocks, kDiagThreads, 0, s>>>(a, scratch);
    k_diag_final<<<1, kDiagThreads, 0, s>>>(scratch, scratch + kDiagBlocks * 6);
    return hipGetLastError();
}

hipError_t sw_launch_step(const SwLaunch &a, const SwTuning &t, hipStream_t s) {
    if (t.variant == 2) return sw_launch_fused_cfg(a, t.rows, t.vec, t.minw, t.pd, t.order, s);
    return a.dtype ? launch_step_cell<double>(a, s) : launch_step_cell<float>(a, s);
}
