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

template <typename T, int VEC> __device__ __forceinline__ void vstore(T *p, const T o[VEC]);
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

// Lane l receives x from lane l - 1; lane 0 receives `edge`.
template <typename T> __device__ __forceinline__ T from_prev_lane(T x, T edge, int lane) {
    T y = __shfl_up(x, 1);
    return lane == 0 ? edge : y;
}
// Lane l receives x from lane l + 1; lane 63 receives `edge`.
template <typename T> __device__ __forceinline__ T from_next_lane(T x, T edge, int lane) {
    T y = __shfl_down(x, 1);
    return lane == 63 ? edge : y;
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

template <typename T, int VEC>
__global__ __launch_bounds__(256) void k_step_fused(SwLaunch a, int rows, int nstrips, int ntiles) {
    constexpr int W = 64 * VEC;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
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
    double smax = 0.0;
    bool bad = false;

    if (tile < ntiles) {
        const int s = tile % nstrips, rb = tile / nstrips;
        const int c0 = s * W, j0 = rb * rows, j1 = min(j0 + rows, ny);
        const int c = c0 + VEC * lane;
        const bool in_row = c <= nx;                      // the vector stays inside the row's allocation
        const int ec = lane == 0 ? c0 - 1 : c0 + W;       // this lane's edge column
        const bool edge_ok = lane == 0 || (lane == 63 && c0 + W <= nx);
        const T elx = lane == 0 ? lx : -lx;               // lane 0 needs L of its edge, lane 63 needs R
        const bool tile_at_wall = s == 0 || c0 + W >= nx || j0 == 0 || j1 >= ny;
        const T *I0 = (const T *)a.in[0], *I1 = (const T *)a.in[1], *I2 = (const T *)a.in[2];
        T *O[3] = {(T *)a.out[0], (T *)a.out[1], (T *)a.out[2]};

        // Raw row: the lane's VEC cells and its edge cell.
        T rh[VEC], rp[VEC], rq[VEC], eh, ep, eq;
        auto load_row = [&](int j, T *h, T *p, T *q, T &e0, T &e1, T &e2) {
            const int64_t ro = (int64_t)j * pitch;
            if (in_row) {
                vload<T, VEC>(I0 + ro + c, h);
                vload<T, VEC>(I1 + ro + c, p);
                vload<T, VEC>(I2 + ro + c, q);
            } else {
#pragma unroll
                for (int m = 0; m < VEC; ++m) { h[m] = T(1); p[m] = T(0); q[m] = T(0); }
            }
            if (edge_ok) {
                e0 = I0[ro + ec]; e1 = I1[ro + ec]; e2 = I2[ro + ec];
            } else {
                e0 = T(1); e1 = T(0); e2 = T(0);
            }
        };

        // From a raw row: the x part of the update (S), and the y-face
        // contributions B (as lower cell) and T (as upper cell).
        auto derive = [&](const T *h, const T *p, const T *q, T e0, T e1, T e2, bool want_x, T S[3][VEC],
                          T Bc[3][VEC], T Tc[3][VEC]) {
            T L[3][VEC], R[3][VEC];
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                T r = fast_rcp(h[m]);
                T u = p[m] * r, v = q[m] * r;
                T kh = k * h[m];
                T fp = fma(kh, h[m], p[m] * u);
                T fq = q[m] * u;            // = hu hv / h, also the G flux of hu
                T gq = fma(kh, h[m], q[m] * v);
                T hh = T(0.5) * h[m], hp = T(0.5) * p[m], hq = T(0.5) * q[m];
                L[0][m] = fma(lx, p[m], hh); R[0][m] = fma(-lx, p[m], hh);
                L[1][m] = fma(lx, fp, hp);   R[1][m] = fma(-lx, fp, hp);
                L[2][m] = fma(lx, fq, hq);   R[2][m] = fma(-lx, fq, hq);
                Bc[0][m] = fma(ly, q[m], hh); Tc[0][m] = fma(-ly, q[m], hh);
                Bc[1][m] = fma(ly, fq, hp);   Tc[1][m] = fma(-ly, fq, hp);
                Bc[2][m] = fma(ly, gq, hq);   Tc[2][m] = fma(-ly, gq, hq);
            }
            if (!want_x) return;
            // edge cell: L (lane 0) or R (lane 63) of the neighbouring column
            T E[3];
            {
                T r = fast_rcp(e0);
                T u = e1 * r;
                T fp = fma(k * e0, e0, e1 * u);
                T fq = e2 * u;
                E[0] = fma(elx, e1, T(0.5) * e0);
                E[1] = fma(elx, fp, T(0.5) * e1);
                E[2] = fma(elx, fq, T(0.5) * e2);
            }
            T Lm[3], Rp[3];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                Lm[kk] = from_prev_lane(L[kk][VEC - 1], E[kk], lane);
                Rp[kk] = from_next_lane(R[kk][0], E[kk], lane);
            }
            T fl[3], fr[3];
            xface_flux(Lm[0] + R[0][0], Lm[1] + R[1][0], Lm[2] + R[2][0], k, fl);
            const T *U[3] = {h, p, q};
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                if (m + 1 < VEC)
                    xface_flux(L[0][m] + R[0][m + 1], L[1][m] + R[1][m + 1], L[2][m] + R[2][m + 1], k, fr);
                else
                    xface_flux(L[0][m] + Rp[0], L[1][m] + Rp[1], L[2][m] + Rp[2], k, fr);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    S[kk][m] = fma(-mx, fr[kk] - fl[kk], U[kk][m]);
                    fl[kk] = fr[kk];
                }
            }
        };

        // Prologue: row j0 - 1 gives B; row j0 gives S, B, T and G_{j0-1/2}.
        T S[3][VEC], Bp[3][VEC], Gd[3][VEC];
        {
            T Sd[3][VEC], Td[3][VEC];
            load_row(j0 - 1, rh, rp, rq, eh, ep, eq);
            derive(rh, rp, rq, eh, ep, eq, false, Sd, Bp, Td);
            load_row(j0, rh, rp, rq, eh, ep, eq);
            T Bc[3][VEC];
            derive(rh, rp, rq, eh, ep, eq, true, S, Bc, Td);
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                T f[3];
                yface_flux(Bp[0][m] + Td[0][m], Bp[1][m] + Td[1][m], Bp[2][m] + Td[2][m], k, f);
                Gd[0][m] = f[0]; Gd[1][m] = f[1]; Gd[2][m] = f[2];
            }
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int m = 0; m < VEC; ++m) Bp[kk][m] = Bc[kk][m];
        }
        load_row(j0 + 1, rh, rp, rq, eh, ep, eq);

        for (int j = j0; j < j1; ++j) {
            // current raw row j+1 -> registers; prefetch row j+2
            T nh[VEC], np[VEC], nq[VEC], n0, n1, n2;
#pragma unroll
            for (int m = 0; m < VEC; ++m) { nh[m] = rh[m]; np[m] = rp[m]; nq[m] = rq[m]; }
            n0 = eh; n1 = ep; n2 = eq;
            if (j + 2 <= j1) load_row(j + 2, rh, rp, rq, eh, ep, eq);

            T Sn[3][VEC], Bn[3][VEC], Tn[3][VEC];
            derive(nh, np, nq, n0, n1, n2, j + 1 < j1, Sn, Bn, Tn);

            // y face j + 1/2 and the finished row j
            T out[3][VEC];
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                T f[3];
                yface_flux(Bp[0][m] + Tn[0][m], Bp[1][m] + Tn[1][m], Bp[2][m] + Tn[2][m], k, f);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    out[kk][m] = fma(-my, f[kk] - Gd[kk][m], S[kk][m]);
                    Gd[kk][m] = f[kk];
                }
            }
            // store row j
            const int64_t ro = (int64_t)j * pitch;
            if (c + VEC <= nx) {
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) vstore<T, VEC>(O[kk] + ro + c, out[kk]);
            } else {
#pragma unroll
                for (int m = 0; m < VEC; ++m)
                    if (c + m < nx) {
                        O[0][ro + c + m] = out[0][m];
                        O[1][ro + c + m] = out[1][m];
                        O[2][ro + c + m] = out[2][m];
                    }
            }
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                if (c + m < nx) {
                    T hn = out[0][m];
                    T sp = fmax(fabs(out[1][m]), fabs(out[2][m])) * fast_rcp(hn) + fast_sqrt(g * hn);
                    bad |= !(sp <= finite_max<T>());
                    smax = fmax(smax, (double)sp);
                    if (tile_at_wall && (c + m == 0 || c + m == nx - 1 || j == 0 || j == ny - 1))
                        write_ghosts(O, pitch, nx, ny, a.bc_x, a.bc_y, c + m, j, U3<T>{out[0][m], out[1][m], out[2][m]});
                }
            }
            // carry row j+1
#pragma unroll
            for (int kk = 0; kk < 3; ++kk)
#pragma unroll
                for (int m = 0; m < VEC; ++m) { S[kk][m] = Sn[kk][m]; Bp[kk][m] = Bn[kk][m]; }
        }
    }
    step_epilogue(a, smax, bad, dt, blockIdx.x == 0 && threadIdx.x == 0);
}

template <typename T, int VEC>
hipError_t launch_fused_t(const SwLaunch &a, int rows, hipStream_t s) {
    constexpr int W = 64 * VEC;
    const int nstrips = (a.nx + W - 1) / W;
    const int nrb = (a.ny + rows - 1) / rows;
    const int64_t ntiles = (int64_t)nstrips * nrb;
    int64_t blocks = (ntiles + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    k_step_fused<T, VEC><<<(unsigned)blocks, 256, 0, s>>>(a, rows, nstrips, (int)ntiles);
    return hipGetLastError();
}

// Rows per tile: enough tiles to give every CU several waves, tall enough
// that the two halo rows per tile stay a small fraction.
int pick_rows(const SwLaunch &a, int W) {
    const int64_t nstrips = (a.nx + W - 1) / W;
    int rows = 256;
    while (rows > 16 && nstrips * ((a.ny + rows - 1) / rows) < 8192) rows >>= 1;
    return rows;
}

}  // namespace

hipError_t sw_launch_fused_rows(const SwLaunch &a, int rows, hipStream_t s) {
    if (a.scheme != 0) return hipErrorNotSupported;
    if (rows < 1) return hipErrorInvalidValue;
    if (a.dtype) return launch_fused_t<double, 2>(a, rows, s);
    return launch_fused_t<float, 4>(a, rows, s);
}

hipError_t sw_launch_fused(const SwLaunch &a, hipStream_t s) {
    const int W = a.dtype ? 128 : 256;
    return sw_launch_fused_rows(a, pick_rows(a, W), s);
}
