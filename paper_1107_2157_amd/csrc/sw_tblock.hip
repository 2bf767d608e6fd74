// Temporal blocking of the fixed-dt step: K time steps per launch.
//
// With a fixed dt (the paper's mode) a cell after K steps depends only on the
// state within K cells of it, so a block can stage a tile plus a K-cell halo
// in LDS, advance it K steps there and write only the tile's own cells: the
// state crosses HBM once per K steps instead of once per step.  Each step
// shrinks the region that can still be advanced by one cell on every side;
// on periodic axes the halo is loaded wrapped and simply advanced with the
// rest, on reflective axes the ghost layer is re-derived from the new state
// after every step (mirror image, wall-normal momentum negated), exactly as
// the boundary rule does between single steps.  Within a step each wave
// marches a chunk of rows the way the fused single-step kernel marches a
// strip (same fluxes, same rounding, reciprocal included), so K blocked steps
// give bitwise the state of K fused steps.
//
// Tile: RX = 64 staged columns (one lane per column, one wave width), so
// TX = 64 - 2K output columns; RY staged rows (98 in FP32, 50 in FP64), so
// TY = RY - 2K output rows; one buffer of 3 * 64 * RY values, updated in
// place.  K is odd, so a K-step launch flips the global buffers once, as K
// single steps would.
#include "sw_tile.h"

using namespace sw;
using namespace sw::tile;

namespace {

// Staged rows per tile (the tile's own rows TY = RY - 2K): three planes of
// 64 x RY values in LDS, two tiles per CU (75 KB in FP32, 77 KB in FP64).
// With 16 (FP32) or 12 / 8 (FP64) waves, RY - 2 - 2s rows split into equal
// chunks at every step s, so no wave waits for a longer one at the barrier.
// x neighbours for the row march: lane l receives x from lane l + 1 (next)
// or l - 1 (prev); the wave's edge lane, which is never a live cell of a
// blocked step, receives 0.  In FP32 that form lets the compiler fold the
// lane move into the add or subtract that consumes it (a DPP operand).
__device__ __forceinline__ float tb_next(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ float tb_prev(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ double tb_next(double x) { return from_next_lane(x, x); }
__device__ __forceinline__ double tb_prev(double x) { return from_prev_lane(x, x); }

template <typename T> constexpr int tb_staged_rows() { return sizeof(T) == 4 ? 98 : 50; }
constexpr int kTbCols = 64;

// Lanes of one staged column, for the whole launch.
struct TbCols {
    bool store;    // a cell of the domain that this step advances
    bool ghost_lo; // the reflective ghost left of x = 0, refreshed this step
    bool ghost_hi; // the reflective ghost right of x = nx - 1
};

// One wave advances staged rows r0 .. r1 - 1 of one step in place (lane =
// staged column), marching upward: each row's state is read once, the G
// flux of the face below a row is carried to the next row and the F flux of
// the face right of a lane reaches the lane to its right by DPP.  The
// arithmetic is the fused single-step kernel's, operation for operation.
// Rows r0 - 1 and r1 belong to the neighbouring waves' chunks; they were
// read into E0 / E1 before the step's first barrier.  A new row is stored
// where its column and row lie in the domain; at reflective walls the wave
// also stores the mirror image into the ghost cell beside it (wall-normal
// momentum negated), as the boundary rule does between single steps.
// Wave-uniform: all 64 lanes call it together; `xwall` is uniform.
template <typename T, int RX>
__device__ __forceinline__ void tb_march(T *const B[3], const T E0[3], const T E1[3], int r0, int r1, TbCols c,
                                         bool xwall, int y0, int ny, bool pery, T k, T lx, T ly, T mx, T my) {
    const int lane = threadIdx.x & 63;
    T S[3], Bp[3], Gd[3];
    auto load = [&](int r, T u[3]) {
        const int o = r * RX + lane;
        u[0] = B[0][o];
        u[1] = B[1][o];
        u[2] = B[2][o];
    };
    auto row = [&](auto face_c, auto emit_c, const T U[3], bool want_x, int rout) {
        constexpr bool FACE = decltype(face_c)::value, EMIT = decltype(emit_c)::value;
        const T h = U[0], p = U[1], q = U[2];
        const T rc = fast_rcp(h);
        const T u = p * rc, v = q * rc;
        const T kh = k * h;
        const T fp = fma(kh, h, p * u), fq = q * u, gq = fma(kh, h, q * v);
        const T hh = T(0.5) * h, hp = T(0.5) * p, hq = T(0.5) * q;
        if (FACE) {
            T f[3];
            yface_flux<T>(Bp[0] + fma(-ly, q, hh), Bp[1] + fma(-ly, fq, hp), Bp[2] + fma(-ly, gq, hq), k, f);
            if (EMIT) {
                const int y = y0 + rout;
                if (pery || (y >= 0 && y < ny)) {
                    T out[3];
#pragma unroll
                    for (int kk = 0; kk < 3; ++kk) out[kk] = fma(-my, f[kk] - Gd[kk], S[kk]);
                    const int o = rout * RX + lane;
                    if (c.store) {
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk) B[kk][o] = out[kk];
                    }
                    if (xwall) {
                        // both shifts by every lane (DPP reads the neighbour's register), then select
                        T mn[3], mp[3];
#pragma unroll
                        for (int kk = 0; kk < 3; ++kk) {
                            mn[kk] = from_next_lane(out[kk], out[kk]);
                            mp[kk] = from_prev_lane(out[kk], out[kk]);
                        }
                        if (c.ghost_lo) {
                            B[0][o] = mn[0];
                            B[1][o] = -mn[1];
                            B[2][o] = mn[2];
                        }
                        if (c.ghost_hi) {
                            B[0][o] = mp[0];
                            B[1][o] = -mp[1];
                            B[2][o] = mp[2];
                        }
                    }
                    if (!pery && c.store) {
                        if (y == 0) {
                            B[0][o - RX] = out[0];
                            B[1][o - RX] = out[1];
                            B[2][o - RX] = -out[2];
                        }
                        if (y == ny - 1) {
                            B[0][o + RX] = out[0];
                            B[1][o + RX] = out[1];
                            B[2][o + RX] = -out[2];
                        }
                    }
                }
            }
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) Gd[kk] = f[kk];
        }
        Bp[0] = fma(ly, q, hh);
        Bp[1] = fma(ly, fq, hp);
        Bp[2] = fma(ly, gq, hq);
        if (!want_x) return;
        T L[3], R[3], Rn[3], fr[3];
        L[0] = fma(lx, p, hh);
        L[1] = fma(lx, fp, hp);
        L[2] = fma(lx, fq, hq);
        R[0] = fma(-lx, p, hh);
        R[1] = fma(-lx, fp, hp);
        R[2] = fma(-lx, fq, hq);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) Rn[kk] = tb_next(R[kk]);
        xface_flux<T>(L[0] + Rn[0], L[1] + Rn[1], L[2] + Rn[2], k, fr);
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) S[kk] = fma(-mx, fr[kk] - tb_prev(fr[kk]), U[kk]);
    };
    T U[3], N[3];
    load(r0, U);
    row(bconst<false>{}, bconst<false>{}, E0, false, 0);
    if (r0 + 1 < r1) load(r0 + 1, N);
    else N[0] = E1[0], N[1] = E1[1], N[2] = E1[2];
    row(bconst<true>{}, bconst<false>{}, U, true, 0);
    for (int r = r0 + 1; r < r1; ++r) {
        U[0] = N[0], U[1] = N[1], U[2] = N[2];            // row r
        if (r + 1 < r1) load(r + 1, N);
        else N[0] = E1[0], N[1] = E1[1], N[2] = E1[2];
        row(bconst<true>{}, bconst<true>{}, U, true, r - 1);
    }
    row(bconst<true>{}, bconst<true>{}, N, false, r1 - 1);   // row r1 closes the chunk
}

template <typename T, int K, int NW>
__global__ __launch_bounds__(64 * NW) void k_step_tb(SwLaunch a) {
    constexpr int RX = kTbCols, TX = RX - 2 * K;
    constexpr int RY = tb_staged_rows<T>(), TY = RY - 2 * K, RN = RX * RY;
    __shared__ T buf[3][RN];
    T *const Bf[3] = {buf[0], buf[1], buf[2]};
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // uniform: row loops run on scalars
    const int nx = a.nx, ny = a.ny;
    const bool perx = a.bc_x == 1, pery = a.bc_y == 1;
    const int gx0 = blockIdx.x * TX - K, gy0 = blockIdx.y * TY - K;   // global cell of staged (0, 0)
    const int64_t pitch = a.pitch;
    const T *I[3] = {(const T *)a.in[0], (const T *)a.in[1], (const T *)a.in[2]};
    T *O[3] = {(T *)a.out[0], (T *)a.out[1], (T *)a.out[2]};
    const double dt = a.dt_fixed;
    const T k = (T)(0.5 * a.g), g = (T)a.g;
    const T lx = (T)(0.5 * dt / a.dx), ly = (T)(0.5 * dt / a.dy);
    const T mx = (T)(dt / a.dx), my = (T)(dt / a.dy);

    // staged column / row -> global index: wrapped on periodic axes, clamped to
    // the ghost layer [-1, n] on reflective ones (cells beyond it feed no cell
    // of the domain)
    const int x = gx0 + lane;
    int gx = x;
    if (perx) {
        gx %= nx;
        if (gx < 0) gx += nx;
    } else {
        gx = min(max(gx, -1), nx);
    }
    const bool col_in = perx || (x >= 0 && x < nx);
    const bool col_lo_wall = !perx && x == -1, col_hi_wall = !perx && x == nx;
    const bool xwall = !perx && (gx0 < 0 || gx0 + RX > nx);            // uniform
    for (int r = wave; r < RY; r += NW) {
        int gy = gy0 + r;
        if (pery) {
            gy %= ny;
            if (gy < 0) gy += ny;
        } else {
            gy = min(max(gy, -1), ny);
        }
        const int64_t off = (int64_t)gy * pitch + gx;
        const int o = r * RX + lane;
#pragma unroll
        for (int f = 0; f < 3; ++f) buf[f][o] = I[f][off];
    }
    __syncthreads();

#pragma unroll 1
    for (int s = 0; s < K; ++s) {
        // cells that can still be advanced: staged rows / columns [s + 1, R - 2 - s],
        // split into one chunk of consecutive rows per wave
        const int lo = s + 1, hx = RX - 2 - s, hy = RY - 2 - s;
        const bool col_live = lane >= lo && lane <= hx;
        const int chunk = (hy - lo + NW) / NW;
        const int r0 = lo + wave * chunk, r1 = min(r0 + chunk, hy + 1);
        const bool active = r0 < r1;
        T E0[3], E1[3];
        if (active) {
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                E0[kk] = buf[kk][(r0 - 1) * RX + lane];
                E1[kk] = buf[kk][r1 * RX + lane];
            }
        }
        __syncthreads();        // the neighbours' edge rows are read before anyone writes
        if (active)
            tb_march<T, RX>(Bf, E0, E1, r0, r1, TbCols{col_live && col_in, col_live && col_lo_wall,
                                                       col_live && col_hi_wall},
                            xwall, gy0, ny, pery, k, lx, ly, mx, my);
        __syncthreads();
    }

    // the tile's own cells: U^{n+K}, their ghost images, the sticky flag
    bool bad = false;
    const bool col_out = lane >= K && lane < K + TX && x < nx;
    for (int r = K + wave; r < K + TY; r += NW) {
        const int y = gy0 + r;
        if (!col_out || y >= ny) continue;
        const int o = r * RX + lane;
        const U3<T> v = {buf[0][o], buf[1][o], buf[2][o]};
        const int64_t off = (int64_t)y * pitch + x;
        O[0][off] = v.h;
        O[1][off] = v.p;
        O[2][off] = v.q;
        if (x == 0 || x == nx - 1 || y == 0 || y == ny - 1) write_ghosts(O, pitch, nx, ny, a.bc_x, a.bc_y, x, y, v);
        bad |= !(signal_speed(v, g) <= finite_max<T>());
    }
    if (__ballot(bad) && lane == 0) atomicOr(&a.sc->unstable, 1u);
    if (blockIdx.x == 0 && blockIdx.y == 0 && threadIdx.x == 0) {
#pragma unroll 1
        for (int s = 0; s < K; ++s) a.sc->t += dt;   // as K single steps accumulate it
        a.sc->last_dt = dt;
        a.sc->steps += K;
    }
}

template <typename T, int K> hipError_t launch_tb(const SwLaunch &a, int waves, hipStream_t s) {
    constexpr int TX = kTbCols - 2 * K, TY = tb_staged_rows<T>() - 2 * K;
    dim3 grid((a.nx + TX - 1) / TX, (a.ny + TY - 1) / TY);
    if (grid.y > 65535u) return hipErrorInvalidValue;   // refused earlier by the tuning check
    if (waves == 16) k_step_tb<T, K, 16><<<grid, 1024, 0, s>>>(a);
    else if (waves == 12) k_step_tb<T, K, 12><<<grid, 768, 0, s>>>(a);
    else if (waves == 8) k_step_tb<T, K, 8><<<grid, 512, 0, s>>>(a);
    else k_step_tb<T, K, 4><<<grid, 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

bool sw_tb_supported(int dtype, int k) { return k == 3 || k == 5 || (dtype == 0 && k == 7); }

int sw_tb_tile_rows(int dtype, int k) { return (dtype == 0 ? tb_staged_rows<float>() : tb_staged_rows<double>()) - 2 * k; }

hipError_t sw_launch_tb(const SwLaunch &a, int k, int waves, hipStream_t s) {
    if (a.dt_fixed <= 0 || a.scheme != 0) return hipErrorInvalidValue;
    if (a.dtype == 0) {
        if (k == 3) return launch_tb<float, 3>(a, waves, s);
        if (k == 5) return launch_tb<float, 5>(a, waves, s);
        if (k == 7) return launch_tb<float, 7>(a, waves, s);
    } else {
        if (k == 3) return launch_tb<double, 3>(a, waves, s);
        if (k == 5) return launch_tb<double, 5>(a, waves, s);
    }
    return hipErrorInvalidValue;
}
