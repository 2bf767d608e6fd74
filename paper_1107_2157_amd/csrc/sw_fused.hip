// Fused row-marching step kernel for gfx950.
//
// One wavefront owns a tile of W = 64 * VEC columns x R rows of the interior.
// Lane l holds VEC consecutive cells of a row (one 16-byte load per plane).
// The wave marches up its rows with a register window:
//   - the new row j+1 arrives (its load was issued one iteration earlier);
//   - per-cell fluxes F, G and the half-step contributions
//       L = U/2 + lx F, R = U/2 - lx F   (x: face = L_left + R_right)
//       B = U/2 + ly G, T = U/2 - ly G   (y: face = B_below + T_above)
//     are formed once per cell (lx = dt/2dx, ly = dt/2dy);
//   - x faces of row j+1 use the neighbour lanes' L/R through cross-lane
//     moves (the strip's outer neighbours come from two edge loads) and give
//     the x part of the update S = U - dt/dx (F_{i+1/2} - F_{i-1/2});
//   - the y face j+1/2 = B_j + T_{j+1} gives G_{j+1/2}; row j is finished as
//     S_j - dt/dy (G_{j+1/2} - G_{j-1/2}) and stored, with its ghost copies if
//     it is an edge cell, and its signal speed enters the CFL max.
// Face states never leave registers; every input cell is loaded once per
// tile (plus one halo row above and below and two edge columns).
#include <type_traits>

#include "sw_common.h"

using namespace sw;

namespace {

template <typename T> __device__ __forceinline__ T fast_rcp(T x);
template <> __device__ __forceinline__ float fast_rcp<float>(float x) { return __builtin_amdgcn_rcpf(x); }
template <> __device__ __forceinline__ double fast_rcp<double>(double x) { return 1.0 / x; }

template <typename T> __device__ __forceinline__ T fast_sqrt(T x);
template <> __device__ __forceinline__ float fast_sqrt<float>(float x) { return __builtin_amdgcn_sqrtf(x); }
template <> __device__ __forceinline__ double fast_sqrt<double>(double x) { return sqrt(x); }

template <typename T, int VEC> __device__ __forceinline__ void vload(const T *p, T o[VEC]);
template <> __device__ __forceinline__ void vload<float, 4>(const float *p, float o[4]) {
    float4 v = *reinterpret_cast<const float4 *>(p);
    o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
}
template <> __device__ __forceinline__ void vload<float, 2>(const float *p, float o[2]) {
    float2 v = *reinterpret_cast<const float2 *>(p);
    o[0] = v.x; o[1] = v.y;
}
template <> __device__ __forceinline__ void vload<double, 2>(const double *p, double o[2]) {
    double2 v = *reinterpret_cast<const double2 *>(p);
    o[0] = v.x; o[1] = v.y;
}
template <> __device__ __forceinline__ void vload<double, 4>(const double *p, double o[4]) {
    double2 v = *reinterpret_cast<const double2 *>(p);
    double2 w = *reinterpret_cast<const double2 *>(p + 2);
    o[0] = v.x; o[1] = v.y; o[2] = w.x; o[3] = w.y;
}

template <> __device__ __forceinline__ void vload<double, 1>(const double *p, double o[1]) { o[0] = *p; }

template <typename T, int VEC> __device__ __forceinline__ void vstore(T *p, const T o[VEC]);
template <> __device__ __forceinline__ void vstore<double, 1>(double *p, const double o[1]) { *p = o[0]; }
template <> __device__ __forceinline__ void vstore<float, 4>(float *p, const float o[4]) {
    *reinterpret_cast<float4 *>(p) = make_float4(o[0], o[1], o[2], o[3]);
}
template <> __device__ __forceinline__ void vstore<float, 2>(float *p, const float o[2]) {
    *reinterpret_cast<float2 *>(p) = make_float2(o[0], o[1]);
}
template <> __device__ __forceinline__ void vstore<double, 2>(double *p, const double o[2]) {
    *reinterpret_cast<double2 *>(p) = make_double2(o[0], o[1]);
}
template <> __device__ __forceinline__ void vstore<double, 4>(double *p, const double o[4]) {
    *reinterpret_cast<double2 *>(p) = make_double2(o[0], o[1]);
    *reinterpret_cast<double2 *>(p + 2) = make_double2(o[2], o[3]);
}

// Cross-lane moves along the wave.  DPP wave_shr:1 / wave_shl:1 (GFX9
// whole-wave shifts) move a register one lane up / down; the lane with no
// source keeps `edge` (bound_ctrl off), which is exactly the strip's outer
// neighbour.
__device__ __forceinline__ int dpp_prev(int x, int edge) { return __builtin_amdgcn_update_dpp(edge, x, 0x138, 0xf, 0xf, false); }
__device__ __forceinline__ int dpp_next(int x, int edge) { return __builtin_amdgcn_update_dpp(edge, x, 0x130, 0xf, 0xf, false); }

// Lane l receives x from lane l - 1; lane 0 receives `edge`.
__device__ __forceinline__ float from_prev_lane(float x, float edge) {
    return __int_as_float(dpp_prev(__float_as_int(x), __float_as_int(edge)));
}
__device__ __forceinline__ double from_prev_lane(double x, double edge) {
    long long xi = __double_as_longlong(x), ei = __double_as_longlong(edge);
    int lo = dpp_prev((int)xi, (int)ei), hi = dpp_prev((int)(xi >> 32), (int)(ei >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}
// Lane l receives x from lane l + 1; lane 63 receives `edge`.
__device__ __forceinline__ float from_next_lane(float x, float edge) {
    return __int_as_float(dpp_next(__float_as_int(x), __float_as_int(edge)));
}
__device__ __forceinline__ double from_next_lane(double x, double edge) {
    long long xi = __double_as_longlong(x), ei = __double_as_longlong(edge);
    int lo = dpp_next((int)xi, (int)ei), hi = dpp_next((int)(xi >> 32), (int)(ei >> 32));
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Flux through an x face from its half-step state X: F(X).
template <typename T> __device__ __forceinline__ void xface_flux(T xh, T xp, T xq, T k, T f[3]) {
    T r = fast_rcp(xh);
    T u = xp * r;
    f[0] = xp;
    f[1] = fma(k * xh, xh, xp * u);
    f[2] = xq * u;
}
// Flux through a y face from its half-step state Y: G(Y).
template <typename T> __device__ __forceinline__ void yface_flux(T yh, T yp, T yq, T k, T f[3]) {
    T r = fast_rcp(yh);
    T v = yq * r;
    f[0] = yq;
    f[1] = yp * v;
    f[2] = fma(k * yh, yh, yq * v);
}

template <bool B> using bconst = std::integral_constant<bool, B>;

// MINW: register budget expressed as waves per SIMD (0 = compiler's choice).
template <typename T, int VEC, int MINW>
__global__ __launch_bounds__(256, (MINW > 0 ? MINW : 1)) void k_step_fused(SwLaunch a, int rows, int nstrips, int ntiles) {
    constexpr int W = 64 * VEC;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // XCD-aware tile order: blocks are dispatched round-robin over the 8
    // XCDs, so block b runs on XCD b % 8.  Give every XCD a contiguous run of
    // the row-major tile sequence, so the tiles that share halo rows and edge
    // columns meet in the same L2.
    const int per_xcd = gridDim.x >> 3;
    const int tile = (((int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3)) << 2) + wave;
    const double dt = step_dt(a);
    const T k = (T)(0.5 * a.g), g = (T)a.g;
    const T lx = (T)(0.5 * dt / a.dx), ly = (T)(0.5 * dt / a.dy);
    const T mx = (T)(dt / a.dx), my = (T)(dt / a.dy);
    const int nx = a.nx, ny = a.ny;
    const int64_t pitch = a.pitch;
    T smax = T(0);
    bool bad = false;

    if (tile < ntiles) {
        const int s = tile % nstrips, rb = tile / nstrips;
        const int c0 = s * W, j0 = rb * rows, j1 = min(j0 + rows, ny);
        const unsigned c = (unsigned)(c0 + VEC * lane);
        const bool in_row = (int)c <= nx;                    // the vector stays inside the row's allocation
        const bool full = (int)c + VEC <= nx;                // all VEC cells are interior
        const unsigned ec = lane == 0 ? (unsigned)c0 : (unsigned)(c0 + W + 1);   // edge column + 1
        const bool edge_ok = lane == 0 || (lane == 63 && c0 + W <= nx);
        const T elx = lane == 0 ? lx : -lx;                  // lane 0 needs L of its edge, lane 63 needs R
        const bool tile_at_wall = s == 0 || c0 + W >= nx || j0 == 0 || j1 >= ny;
        const T *I[3] = {(const T *)a.in[0], (const T *)a.in[1], (const T *)a.in[2]};
        T *O[3] = {(T *)a.out[0], (T *)a.out[1], (T *)a.out[2]};

        auto load_row = [&](int j, T h[VEC], T p[VEC], T q[VEC], T e[3]) {
            const int64_t ro = (int64_t)j * pitch;
            if (in_row) {
                vload<T, VEC>(I[0] + ro + c, h);
                vload<T, VEC>(I[1] + ro + c, p);
                vload<T, VEC>(I[2] + ro + c, q);
            } else {
#pragma unroll
                for (int m = 0; m < VEC; ++m) { h[m] = T(1); p[m] = T(0); q[m] = T(0); }
            }
            if (edge_ok) {
                e[0] = (I[0] + ro - 1)[ec]; e[1] = (I[1] + ro - 1)[ec]; e[2] = (I[2] + ro - 1)[ec];
            } else {
                e[0] = T(1); e[1] = T(0); e[2] = T(0);
            }
        };

        // Carried from one row to the next (lane's VEC cells):
        T S[3][VEC];    // x part of the update of the row below: U - mx (F_{i+1/2} - F_{i-1/2})
        T Bp[3][VEC];   // y-face contribution of the row below: U/2 + ly G
        T Gd[3][VEC];   // G flux through the face below the current row

        // One pass over a newly arrived row r (= j + 1): its y face with the
        // row below gives G_{r-1/2}, which finishes row r - 1 (if EMIT); then
        // r's own B and (if want_x) the x part S of its update.
        auto row_pass = [&](auto face_c, auto emit_c, const T h[VEC], const T p[VEC], const T q[VEC],
                            const T e[3], bool want_x, int jout) {
            constexpr bool FACE = decltype(face_c)::value, EMIT = decltype(emit_c)::value;
            T L[3][VEC], R[3][VEC], out[3][VEC];
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                T r = fast_rcp(h[m]);
                T u = p[m] * r, v = q[m] * r;
                T kh = k * h[m];
                T fp = fma(kh, h[m], p[m] * u);
                T fq = q[m] * u;            // = hu hv / h: x flux of hv and y flux of hu
                T gq = fma(kh, h[m], q[m] * v);
                T hh = T(0.5) * h[m], hp = T(0.5) * p[m], hq = T(0.5) * q[m];
                if (FACE) {
                    T f[3];
                    yface_flux<T>(Bp[0][m] + fma(-ly, q[m], hh), Bp[1][m] + fma(-ly, fq, hp),
                               Bp[2][m] + fma(-ly, gq, hq), k, f);
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        if (EMIT) out[kk][m] = fma(-my, f[kk] - Gd[kk][m], S[kk][m]);
                        Gd[kk][m] = f[kk];
                    }
                }
                Bp[0][m] = fma(ly, q[m], hh); Bp[1][m] = fma(ly, fq, hp); Bp[2][m] = fma(ly, gq, hq);
                L[0][m] = fma(lx, p[m], hh); R[0][m] = fma(-lx, p[m], hh);
                L[1][m] = fma(lx, fp, hp);   R[1][m] = fma(-lx, fp, hp);
                L[2][m] = fma(lx, fq, hq);   R[2][m] = fma(-lx, fq, hq);
            }
            if (EMIT) {
                const int64_t ro = (int64_t)jout * pitch;
                if (full) {
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) vstore<T, VEC>(O[kk] + ro + c, out[kk]);
#pragma unroll
                    for (int m = 0; m < VEC; ++m) {
                        T sp = fmax(fabs(out[1][m]), fabs(out[2][m])) * fast_rcp(out[0][m]) +
                               fast_sqrt(g * out[0][m]);
                        bad |= !(sp <= finite_max<T>());
                        smax = fmax(smax, sp);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < VEC; ++m) {
                        if ((int)c + m < nx) {
#pragma unroll
                            for (int kk = 0; kk < 3; ++kk) O[kk][ro + c + m] = out[kk][m];
                            T sp = fmax(fabs(out[1][m]), fabs(out[2][m])) * fast_rcp(out[0][m]) +
                                   fast_sqrt(g * out[0][m]);
                            bad |= !(sp <= finite_max<T>());
                            smax = fmax(smax, sp);
                        }
                    }
                }
                if (tile_at_wall) {
#pragma unroll
                    for (int m = 0; m < VEC; ++m) {
                        const int i = (int)c + m;
                        if (i < nx && (i == 0 || i == nx - 1 || jout == 0 || jout == ny - 1))
                            write_ghosts(O, pitch, nx, ny, a.bc_x, a.bc_y, i, jout,
                                         U3<T>{out[0][m], out[1][m], out[2][m]});
                    }
                }
            }
            if (!want_x) return;
            // the lane's edge cell: L (lane 0) or R (lane 63) of the column
            // just outside the strip
            T E[3];
            {
                T r = fast_rcp(e[0]);
                T u = e[1] * r;
                T fp = fma(k * e[0], e[0], e[1] * u);
                T fq = e[2] * u;
                E[0] = fma(elx, e[1], T(0.5) * e[0]);
                E[1] = fma(elx, fp, T(0.5) * e[1]);
                E[2] = fma(elx, fq, T(0.5) * e[2]);
            }
            T fl[3], fr[3];
            {
                T Lm[3];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) Lm[kk] = from_prev_lane(L[kk][VEC - 1], E[kk]);
                xface_flux<T>(Lm[0] + R[0][0], Lm[1] + R[1][0], Lm[2] + R[2][0], k, fl);
            }
            const T *U[3] = {h, p, q};
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                if (m + 1 < VEC) {
                    xface_flux<T>(L[0][m] + R[0][m + 1], L[1][m] + R[1][m + 1], L[2][m] + R[2][m + 1], k, fr);
                } else {
                    T Rp[3];
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) Rp[kk] = from_next_lane(R[kk][0], E[kk]);
                    xface_flux<T>(L[0][m] + Rp[0], L[1][m] + Rp[1], L[2][m] + Rp[2], k, fr);
                }
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    S[kk][m] = fma(-mx, fr[kk] - fl[kk], U[kk][m]);
                    fl[kk] = fr[kk];
                }
            }
        };

        // Prologue: row j0 - 1 gives B; row j0 gives G_{j0-1/2}, B and S.
        T ah[VEC], ap[VEC], aq[VEC], ae[3];
        T bh[VEC], bp[VEC], bq[VEC], be[3];
        load_row(j0 - 1, ah, ap, aq, ae);
        load_row(j0, bh, bp, bq, be);
        row_pass(bconst<false>{}, bconst<false>{}, ah, ap, aq, ae, false, 0);
        row_pass(bconst<true>{}, bconst<false>{}, bh, bp, bq, be, true, 0);
        load_row(j0 + 1, ah, ap, aq, ae);
        // March: two rows per trip so the prefetched row alternates between
        // the register sets a and b without copies.
        for (int j = j0; j < j1; j += 2) {
            if (j + 2 <= j1) load_row(j + 2, bh, bp, bq, be);
            row_pass(bconst<true>{}, bconst<true>{}, ah, ap, aq, ae, j + 1 < j1, j);
            if (j + 1 >= j1) break;
            if (j + 3 <= j1) load_row(j + 3, ah, ap, aq, ae);
            row_pass(bconst<true>{}, bconst<true>{}, bh, bp, bq, be, j + 2 < j1, j + 1);
        }
    }
    step_epilogue(a, (double)smax, bad, dt, blockIdx.x == 0 && wave == 0, (int)blockIdx.x * 4 + wave);
}

template <typename T, int VEC, int MINW>
hipError_t launch_fused_t(const SwLaunch &a, int rows, hipStream_t s) {
    constexpr int W = 64 * VEC;
    const int nstrips = (a.nx + W - 1) / W;
    const int nrb = (a.ny + rows - 1) / rows;
    const int64_t ntiles = (int64_t)nstrips * nrb;
    int64_t blocks = (ntiles + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    k_step_fused<T, VEC, MINW><<<(unsigned)blocks, 256, 0, s>>>(a, rows, nstrips, (int)ntiles);
    return hipGetLastError();
}

}  // namespace

// Rows per tile: enough tiles to give every CU several waves, tall enough
// that the two halo rows per tile stay a small fraction.
int sw_fused_default_rows(int nx, int ny, int vec) {
    const int64_t nstrips = (nx + 64 * vec - 1) / (64 * vec);
    int rows = 256;
    while (rows > 16 && nstrips * ((ny + rows - 1) / rows) < 8192) rows >>= 1;
    return rows;
}

int sw_fused_default_vec(int dtype) { return dtype ? 2 : 4; }

bool sw_fused_supported(int dtype, int vec, int minw) {
    if (minw != 0 && minw != 3 && minw != 4) return false;
    return dtype ? (vec == 1 || vec == 2) : (vec == 2 || vec == 4);
}

hipError_t sw_launch_fused_cfg(const SwLaunch &a, int rows, int vec, int minw, hipStream_t s) {
    if (a.scheme != 0 || rows < 1 || !sw_fused_supported(a.dtype, vec, minw)) return hipErrorInvalidValue;
#define SW_FUSED_CASE(T, V, M) \
    if (vec == V && minw == M) return launch_fused_t<T, V, M>(a, rows, s);
    if (a.dtype) {
        SW_FUSED_CASE(double, 2, 0) SW_FUSED_CASE(double, 2, 3) SW_FUSED_CASE(double, 2, 4)
        SW_FUSED_CASE(double, 1, 0) SW_FUSED_CASE(double, 1, 3) SW_FUSED_CASE(double, 1, 4)
    } else {
        SW_FUSED_CASE(float, 4, 0) SW_FUSED_CASE(float, 4, 3) SW_FUSED_CASE(float, 4, 4)
        SW_FUSED_CASE(float, 2, 0) SW_FUSED_CASE(float, 2, 3) SW_FUSED_CASE(float, 2, 4)
    }
#undef SW_FUSED_CASE
    return hipErrorInvalidValue;
}
