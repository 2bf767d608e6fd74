// The fused per-tile body of the step kernel (shared by the single-grid and
// the batched kernels so that both compute every cell identically).
//
// One wavefront owns a tile of W = 64 * VEC columns x R rows of the interior.
// Lane l holds VEC consecutive cells of a row (one 8- or 16-byte access per
// plane).  The wave marches up its rows with a register window:
//   - the new row j+1 arrives (its load was issued PD rows earlier);
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
// tile (plus one halo row above and below and two edge columns).  Tiles of
// odd row blocks march downwards instead, with the roles of B and T swapped
// (fused_tile below says why).
#pragma once
#include <type_traits>

#include "sw_common.h"

namespace sw {
namespace tile {


// Buffer (V#) access: a scalar resource descriptor per plane and tile, a
// loop-invariant 32-bit byte offset per lane (VGPR) and the row's byte
// offset (SGPR).  Marching to the next row changes only the scalar offset.
// Out-of-range accesses are bounds-checked by the hardware (loads return 0,
// stores are dropped).
typedef __amdgpu_buffer_rsrc_t rsrc_t;
constexpr int kRsrcWord3 = 0x00020000;   // GFX9 descriptor dword 3 (32-bit data format)
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ rsrc_t make_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, kRsrcWord3);
}

// Cache policy bits of the step's row loads and stores (buffer instruction
// aux field: 1 = sc0, 2 = nt, 16 = sc1).  Stores are non-temporal: the new
// state is not read again before the whole grid has been written, and
// streaming it past the caches was measured 5-16 % faster on every workload
// (with sc1 as well, 0.4-1 % faster again at 4096^2 and 16384^2; sc0 alone
// or sc1 alone was slower).  Loads keep the default policy, so the halo rows
// that neighbouring tiles share stay in L2 (non-temporal loads were measured
// 15-20 % slower).
#ifndef SW_LOAD_POLICY
#define SW_LOAD_POLICY 0
#endif
#ifndef SW_STORE_POLICY
#define SW_STORE_POLICY 18
#endif

template <typename T, int VEC> __device__ __forceinline__ void bload(rsrc_t r, unsigned vo, unsigned so, T o[VEC]);
template <> __device__ __forceinline__ void bload<float, 1>(rsrc_t r, unsigned vo, unsigned so, float o[1]) {
    o[0] = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, SW_LOAD_POLICY));
}
template <> __device__ __forceinline__ void bload<float, 2>(rsrc_t r, unsigned vo, unsigned so, float o[2]) {
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, SW_LOAD_POLICY);
    o[0] = __uint_as_float(v.x); o[1] = __uint_as_float(v.y);
}
template <> __device__ __forceinline__ void bload<float, 4>(rsrc_t r, unsigned vo, unsigned so, float o[4]) {
    u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, SW_LOAD_POLICY);
    o[0] = __uint_as_float(v.x); o[1] = __uint_as_float(v.y); o[2] = __uint_as_float(v.z); o[3] = __uint_as_float(v.w);
}
template <> __device__ __forceinline__ void bload<double, 1>(rsrc_t r, unsigned vo, unsigned so, double o[1]) {
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, SW_LOAD_POLICY);
    o[0] = __hiloint2double((int)v.y, (int)v.x);
}
template <> __device__ __forceinline__ void bload<double, 2>(rsrc_t r, unsigned vo, unsigned so, double o[2]) {
    u32x4 v = __builtin_amdgcn_raw_buffer_load_b128(r, vo, so, SW_LOAD_POLICY);
    o[0] = __hiloint2double((int)v.y, (int)v.x); o[1] = __hiloint2double((int)v.w, (int)v.z);
}
__device__ __forceinline__ float bload1(rsrc_t r, unsigned vo, unsigned so, float) {
    return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(r, vo, so, SW_LOAD_POLICY));
}
__device__ __forceinline__ double bload1(rsrc_t r, unsigned vo, unsigned so, double) {
    u32x2 v = __builtin_amdgcn_raw_buffer_load_b64(r, vo, so, SW_LOAD_POLICY);
    return __hiloint2double((int)v.y, (int)v.x);
}

template <typename T, int VEC> __device__ __forceinline__ void bstore(rsrc_t r, unsigned vo, unsigned so, const T o[VEC]);
template <> __device__ __forceinline__ void bstore<float, 1>(rsrc_t r, unsigned vo, unsigned so, const float o[1]) {
    __builtin_amdgcn_raw_buffer_store_b32(__float_as_uint(o[0]), r, vo, so, SW_STORE_POLICY);
}
template <> __device__ __forceinline__ void bstore<float, 2>(rsrc_t r, unsigned vo, unsigned so, const float o[2]) {
    u32x2 v = {__float_as_uint(o[0]), __float_as_uint(o[1])};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, SW_STORE_POLICY);
}
template <> __device__ __forceinline__ void bstore<float, 4>(rsrc_t r, unsigned vo, unsigned so, const float o[4]) {
    u32x4 v = {__float_as_uint(o[0]), __float_as_uint(o[1]), __float_as_uint(o[2]), __float_as_uint(o[3])};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, vo, so, SW_STORE_POLICY);
}
template <> __device__ __forceinline__ void bstore<double, 1>(rsrc_t r, unsigned vo, unsigned so, const double o[1]) {
    u32x2 v = {(unsigned)__double2loint(o[0]), (unsigned)__double2hiint(o[0])};
    __builtin_amdgcn_raw_buffer_store_b64(v, r, vo, so, SW_STORE_POLICY);
}
template <> __device__ __forceinline__ void bstore<double, 2>(rsrc_t r, unsigned vo, unsigned so, const double o[2]) {
    u32x4 v = {(unsigned)__double2loint(o[0]), (unsigned)__double2hiint(o[0]), (unsigned)__double2loint(o[1]),
               (unsigned)__double2hiint(o[1])};
    __builtin_amdgcn_raw_buffer_store_b128(v, r, vo, so, SW_STORE_POLICY);
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

// One tile of one grid: rows [rb * rows, min(rb * rows + rows, ny)) of the
// strip of W = 64 * VEC columns starting at s * W.  Writes the new interior
// cells (and their ghost images at walls) to t.out and folds their signal
// speeds into smax / bad.  Wave-wide: all 64 lanes call it together.
struct TileArgs {
    const void *in[3];
    void *out[3];
    int64_t pitch;
    int nx, ny, bc_x, bc_y;
    int s, rb, rows;
    // 0: leave the ghost cells of t.out unwritten (a step whose successor in
    // the same launch sequence reads no ghost: reflective walls on both axes
    // and the paper's scheme); the last step of a call writes them
    int ghosts = 1;
};

template <typename T, int VEC, int PD, bool DOWN, typename DtFn>
__device__ __forceinline__ void fused_tile_dir(const TileArgs &t, DtFn &&dt_of, double g_, double dx, double dy,
                                               T &smax, bool &bad, double &dt_out) {
    constexpr int W = 64 * VEC;
    const int lane = threadIdx.x & 63;
    const T k = (T)(0.5 * g_), g = (T)g_;
    // set from dt once the tile's first rows are in flight (dt_of waits for
    // the CFL ring slot and divides: wave-wide, called in uniform control flow)
    T lx, ly, mx, my, elx;
    const int nx = t.nx, ny = t.ny, s = t.s, rb = t.rb, rows = t.rows;
    const int64_t pitch = t.pitch;
    {
        const int c0 = s * W, j0 = rb * rows, j1 = min(j0 + rows, ny);
        const unsigned c = (unsigned)(c0 + VEC * lane);
        // At a reflective right wall whose ghost column starts a lane's vector
        // (nx a multiple of VEC, the strip ragged) that vector holds only the
        // ghost and row padding: the lane loads the strip's first vector
        // instead, and the wall cell's right neighbour is formed from the
        // cell itself (its mirror image: L with the hu part negated, exactly
        // what the ghost gives).
        const bool ghost_lane = t.bc_x == 0 && (int)c == nx;
        const bool rwall = t.bc_x == 0 && (int)c + VEC == nx;   // the lane's last cell is nx - 1
        const bool in_row = (int)c <= nx && !ghost_lane;     // the vector stays inside the row's allocation
        const bool full = (int)c + VEC <= nx;                // all VEC cells are interior
        // Edge loads: lanes 0..31 read the column left of the strip, lanes
        // 32..63 the column right of it (two addresses per instruction);
        // lane 0 and lane 63 use them.  Past the right end of the grid the
        // right edge is never needed and reads the left one instead.  At a
        // wall the ghost column holds the image of an interior column (the
        // boundary rule, refreshed before every step): the load reads that
        // column instead, whose line the interior loads share (the ghost's
        // line holds nothing else a tile reads), and a reflective wall's hu is
        // negated where the value is used (esign).  Same values, fewer lines.
        const bool right_ok = c0 + W <= nx;
        const bool left_lane = lane < 32 || !right_ok;
        const bool wall = left_lane ? s == 0 : c0 + W == nx;
        unsigned ec = left_lane ? (unsigned)c0 : (unsigned)(c0 + W + 1);   // column + 1
        if (wall) ec = (left_lane == (t.bc_x == 0)) ? 1u : (unsigned)nx;   // column 0 or nx - 1
        const T esign = wall && t.bc_x == 0 ? T(-1) : T(1);
        // Lanes past the end of the row read the strip's first vector; their
        // cells are never stored and never enter the CFL max.  All loads are
        // unconditional (rows past the tile are clamped to its last row) so
        // that the compiler can count the loads in flight exactly and keep
        // the prefetched rows outstanding while it computes.
        const unsigned cl = in_row ? c : (unsigned)c0;
        const bool tile_at_wall = t.ghosts && (s == 0 || c0 + W >= nx || j0 == 0 || j1 >= ny);
        T *O[3] = {(T *)t.out[0], (T *)t.out[1], (T *)t.out[2]};
        // Descriptors of this tile: they start at cell (-1, j0 - 1) and span
        // rows j0 - 1 .. j1; a row's byte offset is (j - j0 + 1) * pitch * size.
        const int64_t tile_base = (int64_t)(j0 - 1) * pitch - 1;
        const int64_t span = (int64_t)(j1 - j0 + 2) * pitch * (int64_t)sizeof(T);
        const unsigned nrec = span > 0x7fffffff ? 0x7fffffffu : (unsigned)span;
        const rsrc_t rin0 = make_rsrc((const T *)t.in[0] + tile_base, nrec);
        const rsrc_t rin1 = make_rsrc((const T *)t.in[1] + tile_base, nrec);
        const rsrc_t rin2 = make_rsrc((const T *)t.in[2] + tile_base, nrec);
        const rsrc_t rout[3] = {make_rsrc(O[0] + tile_base, nrec), make_rsrc(O[1] + tile_base, nrec),
                                make_rsrc(O[2] + tile_base, nrec)};
        const unsigned row_bytes = (unsigned)(pitch * (int64_t)sizeof(T));
        const unsigned lb = (cl + 1) * (unsigned)sizeof(T);   // lane's vector
        const unsigned eb = ec * (unsigned)sizeof(T);         // lane's edge cell (ec is column + 1)
        const unsigned sb = (c + 1) * (unsigned)sizeof(T);    // lane's store vector

        // A reflective wall's ghost row (row -1 or ny) is the mirror of the
        // edge row with hv negated: the row is loaded instead and its hv
        // negated where the march takes it in (ymirror), so the step reads no
        // ghost row either.
        const bool ymirror = t.bc_y == 0;
        auto load_row = [&](int j, T h[VEC], T p[VEC], T q[VEC], T e[3]) {
            if (ymirror) j = j < 0 ? 0 : (j >= ny ? ny - 1 : j);
            const unsigned so = (unsigned)(j - j0 + 1) * row_bytes;
            bload<T, VEC>(rin0, lb, so, h);
            bload<T, VEC>(rin1, lb, so, p);
            bload<T, VEC>(rin2, lb, so, q);
            e[0] = bload1(rin0, eb, so, T(0));
            e[1] = bload1(rin1, eb, so, T(0));
            e[2] = bload1(rin2, eb, so, T(0));
        };

        // Carried from one row to the next (lane's VEC cells), for a march
        // upwards (downwards):
        T S[3][VEC];    // x part of the update of the row below (above): U - mx (F_{i+1/2} - F_{i-1/2})
        T Bp[3][VEC];   // y-face contribution of the row below, U/2 + ly G (of the row above, U/2 - ly G)
        T Gd[3][VEC];   // G flux through the face below (above) the current row

        // One pass over a newly arrived row r (= j + 1 upwards, j - 1
        // downwards): its y face with the carried row gives G_{r-1/2}
        // (G_{r+1/2}), which finishes row j (if EMIT); then r's own B (T) and
        // (if want_x) the x part S of its update.  The face state is B of the
        // lower row plus T of the upper one and the update subtracts
        // G_{j+1/2} - G_{j-1/2}, in that operand order either way, so both
        // directions round every cell identically.
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
                    if (DOWN)
                        yface_flux<T>(fma(ly, q[m], hh) + Bp[0][m], fma(ly, fq, hp) + Bp[1][m],
                                      fma(ly, gq, hq) + Bp[2][m], k, f);
                    else
                        yface_flux<T>(Bp[0][m] + fma(-ly, q[m], hh), Bp[1][m] + fma(-ly, fq, hp),
                                      Bp[2][m] + fma(-ly, gq, hq), k, f);
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) {
                        if (EMIT) out[kk][m] = DOWN ? fma(-my, Gd[kk][m] - f[kk], S[kk][m])
                                                    : fma(-my, f[kk] - Gd[kk][m], S[kk][m]);
                        Gd[kk][m] = f[kk];
                    }
                }
                if (DOWN) {
                    Bp[0][m] = fma(-ly, q[m], hh); Bp[1][m] = fma(-ly, fq, hp); Bp[2][m] = fma(-ly, gq, hq);
                } else {
                    Bp[0][m] = fma(ly, q[m], hh); Bp[1][m] = fma(ly, fq, hp); Bp[2][m] = fma(ly, gq, hq);
                }
                L[0][m] = fma(lx, p[m], hh); R[0][m] = fma(-lx, p[m], hh);
                L[1][m] = fma(lx, fp, hp);   R[1][m] = fma(-lx, fp, hp);
                L[2][m] = fma(lx, fq, hq);   R[2][m] = fma(-lx, fq, hq);
            }
            if (EMIT) {
                const int64_t ro = (int64_t)jout * pitch;
                if (full) {
                    const unsigned so = (unsigned)(jout - j0 + 1) * row_bytes;
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) bstore<T, VEC>(rout[kk], sb, so, out[kk]);
#pragma unroll
                    for (int m = 0; m < VEC; ++m) {
                        T sp = signal_speed(U3<T>{out[0][m], out[1][m], out[2][m]}, g);
                        bad |= !(sp <= finite_max<T>());
                        smax = fmax(smax, sp);
                    }
                } else {
#pragma unroll
                    for (int m = 0; m < VEC; ++m) {
                        if ((int)c + m < nx) {
#pragma unroll
                            for (int kk = 0; kk < 3; ++kk) O[kk][ro + c + m] = out[kk][m];
                            T sp = signal_speed(U3<T>{out[0][m], out[1][m], out[2][m]}, g);
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
                            write_ghosts(O, pitch, nx, ny, t.bc_x, t.bc_y, i, jout,
                                         U3<T>{out[0][m], out[1][m], out[2][m]});
                    }
                }
            }
            if (!want_x) return;
            // the lane's edge cell: L (lane 0) or R (lane 63) of the column
            // just outside the strip
            T E[3];
            {
                const T e1 = e[1] * esign;
                T r = fast_rcp(e[0]);
                T u = e1 * r;
                T fp = fma(k * e[0], e[0], e1 * u);
                T fq = e[2] * u;
                E[0] = fma(elx, e1, T(0.5) * e[0]);
                E[1] = fma(elx, fp, T(0.5) * e1);
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
                    if (rwall) {
                        Rp[0] = L[0][m];
                        Rp[1] = -L[1][m];
                        Rp[2] = L[2][m];
                    }
                    xface_flux<T>(L[0][m] + Rp[0], L[1][m] + Rp[1], L[2][m] + Rp[2], k, fr);
                }
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    S[kk][m] = fma(-mx, fr[kk] - fl[kk], U[kk][m]);
                    fl[kk] = fr[kk];
                }
            }
        };

        // The march visits rows rowat(0), rowat(1), ..., rowat(nr + 1): the
        // halo row, the nr = j1 - j0 interior rows, the other halo row
        // (upwards j0 - 1 .. j1, downwards j1 .. j0 - 1).  Prologue: the first
        // halo row gives B (T); the first interior row gives its face flux,
        // B (T) and S.  Raw rows rowat(2 ..) pass through a ring of PD + 1
        // register sets: rowat(k) sits in set (k - 2) % (PD + 1), loaded PD
        // rows before it is used.
        const int nr = j1 - j0;
        auto rowat = [&](int kk) { return DOWN ? j1 - kk : j0 - 1 + kk; };
        T rh[PD + 1][VEC], rp[PD + 1][VEC], rq[PD + 1][VEC], re[PD + 1][3];
        load_row(rowat(0), rh[0], rp[0], rq[0], re[0]);
        load_row(rowat(1), rh[1 % (PD + 1)], rp[1 % (PD + 1)], rq[1 % (PD + 1)], re[1 % (PD + 1)]);
        // keep the scheduler from hoisting the dt arithmetic (and its wait for
        // the ring slot) above these loads: both latencies then overlap
        __builtin_amdgcn_sched_barrier(0);
        {
            const double dt = dt_of();
            dt_out = dt;
            lx = (T)(0.5 * dt / dx);
            ly = (T)(0.5 * dt / dy);
            mx = (T)(dt / dx);
            my = (T)(dt / dy);
            elx = lane == 0 ? lx : -lx;                      // lane 0 needs L of its edge, lane 63 needs R
        }
        const int jfirst = rowat(0), jlast = rowat(nr + 1);   // the march's halo rows
        if (ymirror && (jfirst < 0 || jfirst >= ny)) {
#pragma unroll
            for (int m = 0; m < VEC; ++m) rq[0][m] = -rq[0][m];
        }
        row_pass(bconst<false>{}, bconst<false>{}, rh[0], rp[0], rq[0], re[0], false, 0);
        row_pass(bconst<true>{}, bconst<false>{}, rh[1 % (PD + 1)], rp[1 % (PD + 1)], rq[1 % (PD + 1)],
                 re[1 % (PD + 1)], true, 0);
        const bool mirror_last = ymirror && (jlast < 0 || jlast >= ny);
#pragma unroll
        for (int u = 0; u < PD; ++u) load_row(rowat(min(2 + u, nr + 1)), rh[u], rp[u], rq[u], re[u]);
        for (int ib = 0; ib < nr; ib += PD + 1) {
#pragma unroll
            for (int u = 0; u <= PD; ++u) {
                const int i = ib + u;          // output row rowat(i + 1); the arriving row rowat(i + 2) is in set u
                if (i >= nr) break;
                const int slot = (u + PD) % (PD + 1);
                load_row(rowat(min(i + 2 + PD, nr + 1)), rh[slot], rp[slot], rq[slot], re[slot]);
                if (mirror_last && i + 1 == nr) {     // the arriving row is the last halo row
#pragma unroll
                    for (int m = 0; m < VEC; ++m) rq[u][m] = -rq[u][m];
                }
                row_pass(bconst<true>{}, bconst<true>{}, rh[u], rp[u], rq[u], re[u], i + 1 < nr, rowat(i + 1));
            }
        }
    }
}


// The tile body: odd row blocks march downwards, even ones upwards.  The
// rows two vertically adjacent tiles share (one's last interior row and the
// other's halo row, both ways) are then read by both near the start, or both
// near the end, of their marches, so the second read finds them in L2; in a
// march all one way one tile reads them first and its neighbour a whole
// march later, after the XCD's other in-flight tiles have evicted them
// (counters: 1.13x the input bytes at 4096^2 FP32 with 4-row tiles, 1.24x
// in FP64 with 8-row tiles).  Results are bitwise the same either way.
template <typename T, int VEC, int PD, typename DtFn>
__device__ __forceinline__ void fused_tile(const TileArgs &t, DtFn &&dt_of, double g_, double dx, double dy, T &smax,
                                           bool &bad, double &dt_out) {
    if (t.rb & 1)
        fused_tile_dir<T, VEC, PD, true>(t, dt_of, g_, dx, dy, smax, bad, dt_out);
    else
        fused_tile_dir<T, VEC, PD, false>(t, dt_of, g_, dx, dy, smax, bad, dt_out);
}

}  // namespace tile
}  // namespace sw
