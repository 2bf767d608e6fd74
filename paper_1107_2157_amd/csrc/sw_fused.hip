// Single-grid fused step kernel for gfx950 (per-tile body in sw_tile.h; with
// the transverse term in sw_tile_tr.h).
#include "sw_tile_tr.h"

using namespace sw;
using namespace sw::tile;

namespace {

// MINW: register budget expressed as waves per SIMD (0 = compiler's choice).
// PD: rows loaded ahead of the row being processed (software pipeline depth).
// TR: the transverse scheme.
template <typename T, int VEC, int MINW, int PD, bool TR>
__global__ __launch_bounds__(256, (MINW > 0 ? MINW : 1)) void k_step_fused(SwLaunch a, int rows, int nstrips, int nrb,
                                                                           int order) {
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    // Tile order.  Blocks are dispatched round-robin over the 8 XCDs (block
    // b on XCD b % 8); orders 0 and 1 give every XCD a contiguous run of the
    // tile sequence so that tiles sharing halo rows and edge columns meet in
    // the same L2.  Order 0: row-block-major sequence.  Order 1: groups of 4
    // row blocks, strip-major inside a group, so the 4 waves of a block take
    // 4 vertically adjacent tiles of one strip.  Order 2: plain block order.
    const int per_xcd = gridDim.x >> 3;
    const int seq = order == 2 ? (int)blockIdx.x : (int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3);
    const int tile = (seq << 2) + wave;
    int s, rb;
    if (order == 1) {
        const int grp = tile / (nstrips * 4), rem = tile - grp * (nstrips * 4);
        s = rem >> 2;
        rb = grp * 4 + (rem & 3);
    } else {
        s = tile % nstrips;
        rb = tile / nstrips;
    }
    const double stripe = step_dt_stripe(a);   // issued first; waited for after the tile's first row loads
    double dt = 0.0;
    T smax = T(0);
    bool bad = false;
    if (rb < nrb) {
        TileArgs t;
        for (int kk = 0; kk < 3; ++kk) { t.in[kk] = a.in[kk]; t.out[kk] = a.out[kk]; }
        t.pitch = a.pitch;
        t.nx = a.nx; t.ny = a.ny; t.bc_x = a.bc_x; t.bc_y = a.bc_y;
        t.s = s; t.rb = rb; t.rows = rows; t.ghosts = a.ghosts;
        if constexpr (TR)
            fused_tile_tr<T, VEC, PD>(t, [&] { return step_dt_finish(a, stripe); }, a.g, a.dx, a.dy, smax, bad, dt);
        else
            fused_tile<T, VEC, PD>(t, [&] { return step_dt_finish(a, stripe); }, a.g, a.dx, a.dy, smax, bad, dt);
    } else {
        dt = step_dt_finish(a, stripe);
    }

    step_epilogue(a, (double)smax, bad, dt, blockIdx.x == 0 && wave == 0, (int)blockIdx.x * 4 + wave);
}

template <typename T, int VEC, int MINW, int PD, bool TR>
hipError_t launch_fused_t(const SwLaunch &a, int rows, int order, hipStream_t s) {
    constexpr int W = 64 * VEC;
    const int nstrips = (a.nx + W - 1) / W;
    const int nrb = (a.ny + rows - 1) / rows;
    // tiles covered by the grid: order 1 rounds the row blocks up to groups of 4
    const int64_t ntiles = (int64_t)nstrips * (order == 1 ? (nrb + 3) / 4 * 4 : nrb);
    int64_t blocks = (ntiles + 3) / 4;
    blocks = (blocks + 7) / 8 * 8;
    if (blocks > 0x3fffffff) return hipErrorInvalidValue;
    k_step_fused<T, VEC, MINW, PD, TR><<<(unsigned)blocks, 256, 0, s>>>(a, rows, nstrips, nrb, order);
    return hipGetLastError();
}

}  // namespace

// Rows per tile: 2 up to 256 cells a side, 4 up to 512, 8 beyond.  A wave
// marches its rows one after another, so on small grids short marches keep
// the step from being latency-bound; 8 rows hold the halo re-reads to 1.25x
// and were best or within 3 % of best from 1024^2 to 16384^2 (FP32,
// measured per width over 1-64 rows).
int sw_fused_default_rows(int nx, int ny, int vec) {
    (void)vec;
    const int side = nx > ny ? nx : ny;
    int rows = 2;
    while (rows < 8 && rows * 128 < side) rows <<= 1;
    return rows;
}

// Cells per lane: wide vectors where the rows are long enough to fill them.
int sw_fused_default_vec(int dtype, int nx) {
    if (dtype) return nx >= 1024 ? 2 : 1;
    return nx >= 2048 ? 4 : (nx >= 512 ? 2 : 1);
}

bool sw_fused_tile_fits(int rows, int64_t pitch, int elem_bytes) {
    return rows >= 1 && ((int64_t)rows + 2) * pitch * (int64_t)elem_bytes <= 0x7fffffff;
}

bool sw_fused_supported(int dtype, int scheme, int vec, int minw, int pd) {
#define SW_FUSED_SUP(T, V, M, P) \
    if ((dtype == 1) == (sizeof(T) == 8) && vec == V && minw == M && pd == P) return true;
    if (scheme == 0) {
        SW_FUSED_SHAPES(SW_FUSED_SUP)
    } else if (scheme == 1) {
        SW_FUSED_TR_SHAPES(SW_FUSED_SUP)
    }
#undef SW_FUSED_SUP
    return false;
}

hipError_t sw_launch_fused_cfg(const SwLaunch &a, int rows, int vec, int minw, int pd, int order, hipStream_t s) {
    if (a.scheme < 0 || a.scheme > 1 || rows < 1 || order < 0 || order > 2) return hipErrorInvalidValue;
#define SW_FUSED_CASE(T, V, M, P) \
    if ((a.dtype == 1) == (sizeof(T) == 8) && vec == V && minw == M && pd == P) \
        return launch_fused_t<T, V, M, P, false>(a, rows, order, s);
#define SW_FUSED_TR_CASE(T, V, M, P) \
    if ((a.dtype == 1) == (sizeof(T) == 8) && vec == V && minw == M && pd == P) \
        return launch_fused_t<T, V, M, P, true>(a, rows, order, s);
    if (a.scheme == 0) {
        SW_FUSED_SHAPES(SW_FUSED_CASE)
    } else {
        SW_FUSED_TR_SHAPES(SW_FUSED_TR_CASE)
    }
#undef SW_FUSED_CASE
#undef SW_FUSED_TR_CASE
    return hipErrorInvalidValue;
}
