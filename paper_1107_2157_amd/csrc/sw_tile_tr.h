// The fused per-tile body with the transverse term in the half-step (the
// standard 2-D Lax-Wendroff correction, not in the paper's equations):
//   x face (i+1/2, j):  + (dt/2dy)/4 [(G_{i,j-1} + G_{i+1,j-1}) - (G_{i,j+1} + G_{i+1,j+1})]
//   y face (i, j+1/2):  + (dt/2dx)/4 [(F_{i-1,j} + F_{i-1,j+1}) - (F_{i+1,j} + F_{i+1,j+1})]
// Shared by the single-grid and the batched kernels, like fused_tile.
//
// Same organisation as fused_tile (sw_tile.h): one wave marches up a strip
// of W = 64 * VEC columns with a register window, x neighbours across lanes
// by DPP, no LDS.  The x faces of a row need the G fluxes of the rows below
// and above it, so the x part of row r's update is formed when row r + 1
// arrives (one row later than in the paper scheme), from row r's state and
// fluxes and from the G fluxes of rows r - 1 and r + 1, carried in
// registers.  Both transverse terms split over the two cells of a face:
//   x face = L'_i + R'_{i+1},  L' = U/2 + lx F + ly/4 D,  R' = U/2 - lx F + ly/4 D,
//            D = G_{row below} - G_{row above} (same column);
//   y face = B'_j + T'_{j+1},  B' = U/2 + ly G + lx/4 C,  T' = U/2 - ly G + lx/4 C,
//            C = F_{i-1} - F_{i+1} (same row),
// so the x term costs no extra lane moves and the y term six per row.  At a
// reflective wall the mirrored ghost makes the normal momentum of the wall
// face exactly zero (fma(-a, b, -c) = -fma(a, b, c)), so no mass crosses it.
// Corner ghosts are read at tile corners on the domain's corners.
#pragma once
#include "sw_tile.h"

namespace sw {
namespace tile {

template <typename T, int VEC, int PD, typename DtFn>
__device__ __forceinline__ void fused_tile_tr(const TileArgs &t, DtFn &&dt_of, double g_, double dx, double dy,
                                              T &smax, bool &bad, double &dt_out) {
    constexpr int W = 64 * VEC;
    const int lane = threadIdx.x & 63;
    const T k = (T)(0.5 * g_), g = (T)g_;
    T lx, ly, mx, my, lx4, ly4, elx;
    const int nx = t.nx, ny = t.ny, s = t.s, rb = t.rb, rows = t.rows;
    const int64_t pitch = t.pitch;
    const int c0 = s * W, j0 = rb * rows, j1 = min(j0 + rows, ny);
    const unsigned c = (unsigned)(c0 + VEC * lane);
    const bool in_row = (int)c <= nx;
    const bool full = (int)c + VEC <= nx;
    const bool right_ok = c0 + W <= nx;
    const unsigned ec = (lane < 32 || !right_ok) ? (unsigned)c0 : (unsigned)(c0 + W + 1);   // column + 1
    const unsigned cl = in_row ? c : (unsigned)c0;
    const bool tile_at_wall = s == 0 || c0 + W >= nx || j0 == 0 || j1 >= ny;
    T *O[3] = {(T *)t.out[0], (T *)t.out[1], (T *)t.out[2]};
    const int64_t tile_base = (int64_t)(j0 - 1) * pitch - 1;
    const int64_t span = (int64_t)(j1 - j0 + 2) * pitch * (int64_t)sizeof(T);
    const unsigned nrec = span > 0x7fffffff ? 0x7fffffffu : (unsigned)span;
    const rsrc_t rin0 = make_rsrc((const T *)t.in[0] + tile_base, nrec);
    const rsrc_t rin1 = make_rsrc((const T *)t.in[1] + tile_base, nrec);
    const rsrc_t rin2 = make_rsrc((const T *)t.in[2] + tile_base, nrec);
    const rsrc_t rout[3] = {make_rsrc(O[0] + tile_base, nrec), make_rsrc(O[1] + tile_base, nrec),
                            make_rsrc(O[2] + tile_base, nrec)};
    const unsigned row_bytes = (unsigned)(pitch * (int64_t)sizeof(T));
    const unsigned lb = (cl + 1) * (unsigned)sizeof(T);
    const unsigned eb = ec * (unsigned)sizeof(T);
    const unsigned sb = (c + 1) * (unsigned)sizeof(T);

    auto load_row = [&](int j, T h[VEC], T p[VEC], T q[VEC], T e[3]) {
        const unsigned so = (unsigned)(j - j0 + 1) * row_bytes;
        bload<T, VEC>(rin0, lb, so, h);
        bload<T, VEC>(rin1, lb, so, p);
        bload<T, VEC>(rin2, lb, so, q);
        e[0] = bload1(rin0, eb, so, T(0));
        e[1] = bload1(rin1, eb, so, T(0));
        e[2] = bload1(rin2, eb, so, T(0));
    };

    // Carried from one row to the next.  Row r (the row whose x faces are
    // formed when row r + 1 arrives): its state and the flux parts
    // fp = hu^2/h + g h^2/2, fq = hu hv / h, gq = hv^2/h + g h^2/2
    // (F = (hu, fp, fq), G = (hv, fq, gq)); the G fluxes of row r - 1; the
    // y-face contribution B' of row r; the G flux through the face below r.
    T Uh[VEC], Up[VEC], Uq[VEC], Rfp[VEC], Rfq[VEC], Rgq[VEC];
    T Gm[3][VEC];
    T Bp[3][VEC];
    T Gd[3][VEC];
    // The lane's edge cell (lane 0: left of the strip, lane 63: right) in row
    // r (state and flux parts) and its G in row r - 1.
    T eU[3], efp = T(0), efq = T(0), egq = T(0);
    T eGm[3];

    // One newly arrived row n.  STAGE 0: the tile's lower halo row (only
    // carried).  STAGE 1: the first row of the tile (the face below it).
    // STAGE 2: the face n - 1/2, the x faces of row n - 1 and its update.
    auto pass = [&](auto stage_c, const T h[VEC], const T p[VEC], const T q[VEC], const T e[3], int jout) {
        constexpr int STAGE = decltype(stage_c)::value;
        T nfp[VEC], nfq[VEC], ngq[VEC];
#pragma unroll
        for (int m = 0; m < VEC; ++m) {
            T r = fast_rcp(h[m]);
            T u = p[m] * r, v = q[m] * r;
            T kh = k * h[m];
            nfp[m] = fma(kh, h[m], p[m] * u);
            nfq[m] = q[m] * u;
            ngq[m] = fma(kh, h[m], q[m] * v);
        }
        T nefp, nefq, negq;
        {
            T r = fast_rcp(e[0]);
            T u = e[1] * r, v = e[2] * r;
            T kh = k * e[0];
            nefp = fma(kh, e[0], e[1] * u);
            nefq = e[2] * u;
            negq = fma(kh, e[0], e[2] * v);
        }
        // C = F_{i-1} - F_{i+1} of the new row; the strip's outer neighbours
        // are the edge cells (lane 0: left edge, lane 63: right edge)
        T C[3][VEC];
        {
            const T *Fc[3] = {p, nfp, nfq};
            const T Fe[3] = {e[1], nefp, nefq};
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                const T lo0 = from_prev_lane(Fc[kk][VEC - 1], Fe[kk]);
                const T hiL = from_next_lane(Fc[kk][0], Fe[kk]);
#pragma unroll
                for (int m = 0; m < VEC; ++m) {
                    const T lo = m == 0 ? lo0 : Fc[kk][m - 1];
                    const T hi = m == VEC - 1 ? hiL : Fc[kk][m + 1];
                    C[kk][m] = lo - hi;
                }
            }
        }
        T Gy[3][VEC];   // G flux through the face n - 1/2 (STAGE >= 1)
        if (STAGE >= 1) {
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                const T hh = T(0.5) * h[m], hp = T(0.5) * p[m], hq = T(0.5) * q[m];
                T f[3];
                yface_flux<T>(Bp[0][m] + fma(lx4, C[0][m], fma(-ly, q[m], hh)),
                              Bp[1][m] + fma(lx4, C[1][m], fma(-ly, nfq[m], hp)),
                              Bp[2][m] + fma(lx4, C[2][m], fma(-ly, ngq[m], hq)), k, f);
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    if (STAGE == 1) Gd[kk][m] = f[kk];
                    else Gy[kk][m] = f[kk];
                }
            }
        }
        if (STAGE == 2) {
            // x faces of row r = n - 1 from L', R' of its cells
            T L[3][VEC], R[3][VEC];
#pragma unroll
            for (int m = 0; m < VEC; ++m) {
                const T d0 = Gm[0][m] - q[m], d1 = Gm[1][m] - nfq[m], d2 = Gm[2][m] - ngq[m];
                const T hh = T(0.5) * Uh[m], hp = T(0.5) * Up[m], hq = T(0.5) * Uq[m];
                L[0][m] = fma(ly4, d0, fma(lx, Up[m], hh));  R[0][m] = fma(ly4, d0, fma(-lx, Up[m], hh));
                L[1][m] = fma(ly4, d1, fma(lx, Rfp[m], hp)); R[1][m] = fma(ly4, d1, fma(-lx, Rfp[m], hp));
                L[2][m] = fma(ly4, d2, fma(lx, Rfq[m], hq)); R[2][m] = fma(ly4, d2, fma(-lx, Rfq[m], hq));
            }
            T E[3];   // L' (lane 0) or R' (lane 63) of the edge cell of row r
            E[0] = fma(ly4, eGm[0] - e[2], fma(elx, eU[1], T(0.5) * eU[0]));
            E[1] = fma(ly4, eGm[1] - nefq, fma(elx, efp, T(0.5) * eU[1]));
            E[2] = fma(ly4, eGm[2] - negq, fma(elx, efq, T(0.5) * eU[2]));
            T S[3][VEC];
            T fl[3], fr[3];
            {
                T Lm[3];
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) Lm[kk] = from_prev_lane(L[kk][VEC - 1], E[kk]);
                xface_flux<T>(Lm[0] + R[0][0], Lm[1] + R[1][0], Lm[2] + R[2][0], k, fl);
            }
            const T *U[3] = {Uh, Up, Uq};
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
            T out[3][VEC];
#pragma unroll
            for (int m = 0; m < VEC; ++m)
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) {
                    out[kk][m] = fma(-my, Gy[kk][m] - Gd[kk][m], S[kk][m]);
                    Gd[kk][m] = Gy[kk][m];
                }
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
                        write_ghosts(O, pitch, nx, ny, t.bc_x, t.bc_y, i, jout, U3<T>{out[0][m], out[1][m], out[2][m]});
                }
            }
        }
        // the new row becomes row r: its G moves down, its B' is formed
#pragma unroll
        for (int m = 0; m < VEC; ++m) {
            Gm[0][m] = Uq[m]; Gm[1][m] = Rfq[m]; Gm[2][m] = Rgq[m];
            Uh[m] = h[m]; Up[m] = p[m]; Uq[m] = q[m];
            Rfp[m] = nfp[m]; Rfq[m] = nfq[m]; Rgq[m] = ngq[m];
            const T hh = T(0.5) * h[m], hp = T(0.5) * p[m], hq = T(0.5) * q[m];
            Bp[0][m] = fma(lx4, C[0][m], fma(ly, q[m], hh));
            Bp[1][m] = fma(lx4, C[1][m], fma(ly, nfq[m], hp));
            Bp[2][m] = fma(lx4, C[2][m], fma(ly, ngq[m], hq));
        }
        eGm[0] = eU[2]; eGm[1] = efq; eGm[2] = egq;
        eU[0] = e[0]; eU[1] = e[1]; eU[2] = e[2];
        efp = nefp; efq = nefq; egq = negq;
    };

    // Rows j0 - 1 .. j1 pass through a ring of PD + 1 register sets as in
    // fused_tile: row r sits in set (r - j0 - 1) % (PD + 1), loaded PD rows
    // before it is used.
    T rh[PD + 1][VEC], rp[PD + 1][VEC], rq[PD + 1][VEC], re[PD + 1][3];
    load_row(j0 - 1, rh[0], rp[0], rq[0], re[0]);
    load_row(j0, rh[1 % (PD + 1)], rp[1 % (PD + 1)], rq[1 % (PD + 1)], re[1 % (PD + 1)]);
    __builtin_amdgcn_sched_barrier(0);
    {
        const double dt = dt_of();
        dt_out = dt;
        lx = (T)(0.5 * dt / dx);
        ly = (T)(0.5 * dt / dy);
        mx = (T)(dt / dx);
        my = (T)(dt / dy);
        lx4 = (T)(0.125 * dt / dx);
        ly4 = (T)(0.125 * dt / dy);
        elx = lane == 0 ? lx : -lx;
    }
#pragma unroll
    for (int m = 0; m < VEC; ++m) Uq[m] = Rfq[m] = Rgq[m] = T(0);
    eU[2] = T(0);
    pass(std::integral_constant<int, 0>{}, rh[0], rp[0], rq[0], re[0], 0);
    pass(std::integral_constant<int, 1>{}, rh[1 % (PD + 1)], rp[1 % (PD + 1)], rq[1 % (PD + 1)], re[1 % (PD + 1)], 0);
#pragma unroll
    for (int u = 0; u < PD; ++u) load_row(min(j0 + 1 + u, j1), rh[u], rp[u], rq[u], re[u]);
    for (int jb = j0; jb < j1; jb += PD + 1) {
#pragma unroll
        for (int u = 0; u <= PD; ++u) {
            const int j = jb + u;          // output row; its upper neighbour j + 1 is in set u
            if (j >= j1) break;
            const int slot = (u + PD) % (PD + 1);
            load_row(min(j + 1 + PD, j1), rh[slot], rp[slot], rq[slot], re[slot]);
            pass(std::integral_constant<int, 2>{}, rh[u], rp[u], rq[u], re[u], j);
        }
    }
}

}  // namespace tile
}  // namespace sw
