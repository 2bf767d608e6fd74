// Device helpers shared by the libsw HIP kernels: the SWE fluxes, the
// Lax-Wendroff half-step on one face, the boundary ghost writes, the signal
// speed and wave-level reductions.
#pragma once
#include <hip/hip_runtime.h>
#include <cfloat>
#include <cstdint>
#include "sw_internal.h"

namespace sw {

template <typename T> struct U3 { T h, p, q; };   // (h, hu, hv)

template <typename T> __device__ __forceinline__ T finite_max();
template <> __device__ __forceinline__ float finite_max<float>() { return FLT_MAX; }
template <> __device__ __forceinline__ double finite_max<double>() { return DBL_MAX; }

// x flux F(U) = (hu, hu^2/h + g h^2 / 2, hu hv / h); k = g / 2.
// Every multiply-add is an explicit fma (the library is built without
// automatic contraction), so mirror-image cells round identically.
template <typename T> __device__ __forceinline__ U3<T> flux_f(U3<T> c, T k) {
    T u = c.p / c.h;
    return {c.p, fma(k * c.h, c.h, c.p * u), c.q * u};
}
// y flux G(U) = (hv, hu hv / h, hv^2/h + g h^2 / 2).
template <typename T> __device__ __forceinline__ U3<T> flux_g(U3<T> c, T k) {
    T v = c.q / c.h;
    return {c.q, c.p * v, fma(k * c.h, c.h, c.q * v)};
}
// Step 1 on one face between cells a (low side) and b (high side):
// (a + b)/2 - l (flux_b - flux_a), l = dt / (2 d).
template <typename T>
__device__ __forceinline__ U3<T> half_step(U3<T> a, U3<T> b, U3<T> fa, U3<T> fb, T l) {
    return {fma(-l, fb.h - fa.h, T(0.5) * (a.h + b.h)),
            fma(-l, fb.p - fa.p, T(0.5) * (a.p + b.p)),
            fma(-l, fb.q - fa.q, T(0.5) * (a.q + b.q))};
}
// Transverse correction added to a face: - l/4 [(t1 + t2) - (t0 + t3)],
// with (t0, t3) the low-side and (t1, t2) the high-side transverse fluxes.
template <typename T>
__device__ __forceinline__ U3<T> add_transverse(U3<T> f, U3<T> lo0, U3<T> lo1, U3<T> hi0, U3<T> hi1, T l4) {
    return {fma(-l4, (hi0.h + hi1.h) - (lo0.h + lo1.h), f.h),
            fma(-l4, (hi0.p + hi1.p) - (lo0.p + lo1.p), f.p),
            fma(-l4, (hi0.q + hi1.q) - (lo0.q + lo1.q), f.q)};
}

// Reciprocal and square root of the step kernels: the hardware's
// approximations in FP32 (v_rcp_f32, v_sqrt_f32, about 1 ulp), correctly
// rounded division and sqrt in FP64.
template <typename T> __device__ __forceinline__ T fast_rcp(T x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }
template <typename T> __device__ __forceinline__ T fast_sqrt(T x);
template <> __device__ __forceinline__ float fast_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fast_sqrt<double>(double x) { return sqrt(x); }

// Largest signal speed of a cell: max(|u|, |v|) + sqrt(g h).  Every kernel
// that feeds the CFL max uses this one formula, so a run split over several
// calls takes bitwise the same dt as one call.
template <typename T> __device__ __forceinline__ T signal_speed(U3<T> c, T g) {
    return fmax(fabs(c.p), fabs(c.q)) * fast_rcp(c.h) + fast_sqrt(g * c.h);
}

// Ghost cells fed by interior cell (i, j) holding c, under the boundary
// conditions: reflective walls mirror the cell with the wall-normal momentum
// negated, periodic walls copy it to the opposite side; corner ghosts get the
// composition (x rule then y rule).  Cell (i, j) itself is not written.
template <typename T>
__device__ __forceinline__ void write_ghosts(T *const o[3], int64_t pitch, int nx, int ny, int bcx, int bcy,
                                             int i, int j, U3<T> c) {
    int xt[2], yt[2];
    T xs[2], ys[2];
    int nxt = 0, nyt = 0;
    if (i == 0) { xt[nxt] = bcx ? nx : -1; xs[nxt++] = bcx ? T(1) : T(-1); }
    if (i == nx - 1) { xt[nxt] = bcx ? -1 : nx; xs[nxt++] = bcx ? T(1) : T(-1); }
    if (j == 0) { yt[nyt] = bcy ? ny : -1; ys[nyt++] = bcy ? T(1) : T(-1); }
    if (j == ny - 1) { yt[nyt] = bcy ? -1 : ny; ys[nyt++] = bcy ? T(1) : T(-1); }
    for (int a = 0; a < nxt; ++a) {
        int64_t off = (int64_t)j * pitch + xt[a];
        o[0][off] = c.h; o[1][off] = xs[a] * c.p; o[2][off] = c.q;
    }
    for (int b = 0; b < nyt; ++b) {
        int64_t off = (int64_t)yt[b] * pitch + i;
        o[0][off] = c.h; o[1][off] = c.p; o[2][off] = ys[b] * c.q;
        for (int a = 0; a < nxt; ++a) {
            int64_t oc = (int64_t)yt[b] * pitch + xt[a];
            o[0][oc] = c.h; o[1][oc] = xs[a] * c.p; o[2][oc] = ys[b] * c.q;
        }
    }
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}

// Max over the 64 stripes of ring slot `slot`.  Called by all 64 lanes of a
// wave in uniform control flow; every lane gets the result.
__device__ __forceinline__ double read_smax(const SwScalars *sc, int slot) {
    return wave_max(__longlong_as_double((long long)sc->smax[slot][threadIdx.x & 63]));
}

// dt of step a.step: fixed, or cfl * min(dx, dy) / (max speed of U^n).
// Wave-wide (all 64 lanes, uniform control flow).
__device__ __forceinline__ double step_dt(const SwLaunch &a) {
    if (a.dt_fixed > 0) return a.dt_fixed;
    return a.cfl * fmin(a.dx, a.dy) / read_smax(a.sc, a.step % 3);
}

// step_dt in two halves, so that a kernel can issue its first row loads while
// the ring slot is in flight: the lane's stripe of the slot (a load; 0 with a
// fixed dt), then the wave max and the division (wave-wide, uniform control
// flow).  step_dt_finish(a, step_dt_stripe(a)) is step_dt(a), bit for bit.
__device__ __forceinline__ double step_dt_stripe(const SwLaunch &a) {
    if (a.dt_fixed > 0) return 0.0;
    return __longlong_as_double((long long)a.sc->smax[a.step % 3][threadIdx.x & 63]);
}
__device__ __forceinline__ double step_dt_finish(const SwLaunch &a, double stripe) {
    if (a.dt_fixed > 0) return a.dt_fixed;
    return a.cfl * fmin(a.dx, a.dy) / wave_max(stripe);
}

// Wave-wide: max-reduce the lanes' signal speeds into stripe `stripe` of
// ring slot `slot` and raise the sticky flag if any lane saw a broken cell.
__device__ __forceinline__ void reduce_speed(SwScalars *sc, int slot, int stripe, double smax, bool bad) {
    smax = wave_max(smax);
    unsigned long long anybad = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&sc->smax[slot][stripe & (kStripes - 1)], (unsigned long long)__double_as_longlong(smax));
        if (anybad) atomicOr(&sc->unstable, 1u);
    }
}

// End of a step kernel (wave-wide): reduce this wave's speeds into the next
// ring slot; the grid's first wave clears the slot after next and advances
// the simulated time.
__device__ __forceinline__ void step_epilogue(const SwLaunch &a, double smax, bool bad, double dt, bool first_wave,
                                              int stripe) {
    reduce_speed(a.sc, (a.step + 1) % 3, stripe, smax, bad);
    if (first_wave) {
        atomicExch(&a.sc->smax[(a.step + 2) % 3][threadIdx.x & 63], 0ull);
        if ((threadIdx.x & 63) == 0) {
            a.sc->t += dt;
            a.sc->last_dt = dt;
            a.sc->steps += 1;
        }
    }
}

}  // namespace sw
