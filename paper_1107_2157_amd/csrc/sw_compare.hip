// The paper's own comparison points, rebuilt on gfx950 (section "Performance
// Measurements"): the generated code kept the face states of the first
// half-step in array temporaries, and the hand-optimised kernel it was
// measured against packed H, U and V into one vector type.  Two step
// variants reproduce those two designs so that their cost on MI355X can be
// set against the fused kernel:
//
//  * unfused: the first half-step writes the face states (x faces and y
//    faces, three planes each) to HBM; a second kernel reads them back,
//    forms the face fluxes and updates the cells (with the ghost writes and
//    the CFL reduction of the fused kernel's epilogue);
//  * AoS: the state lives as one 4-vector (h, hu, hv, 0) per cell; a wave
//    marches a strip of 64 cells (one 16- or 32-byte vector per lane and
//    row) the way the fused kernel does.
//
// Both repeat the fused kernel's arithmetic operation for operation (face
// state = L_left + R_right and B_below + T_above, the same fluxes and
// reciprocal, the same update order), so their states equal the fused
// kernel's bitwise.
#include "sw_tile.h"

using namespace sw;
using namespace sw::tile;

namespace {

// Per-cell parts of the half-step, as the fused kernel forms them: half
// the state, the nonlinear flux components (x flux of hu, the shared
// hu hv / h, y flux of hv) and the momenta.
template <typename T> struct CellParts {
    T hh, hp, hq, fp, fq, gq, p, q;
};
template <typename T> __device__ __forceinline__ CellParts<T> cell_parts(T h, T p, T q, T k) {
    CellParts<T> c;
    const T r = fast_rcp(h);
    const T u = p * r, v = q * r;
    const T kh = k * h;
    c.fp = fma(kh, h, p * u);
    c.fq = q * u;
    c.gq = fma(kh, h, q * v);
    c.hh = T(0.5) * h;
    c.hp = T(0.5) * p;
    c.hq = T(0.5) * q;
    c.p = p;
    c.q = q;
    return c;
}

// ---------------------------------------------------------------------------
// Unfused: face states through HBM.

// x face i (0..nx) of row j lies between cells (i-1, j) and (i, j), at
// f.x[k][j * pitch + i]; y face j (0..ny) of column i lies between cells
// (i, j-1) and (i, j), at f.y[k][j * pitch + i].  Thread (i, j) of a 2-D
// grid writes x face i of row j and y face j of
// column i, from cells (i-1, j), (i, j) and (i, j-1); each block walks a
// band of consecutive rows, so the row below is still in cache.
template <typename T>
__global__ __launch_bounds__(256) void k_faces(SwLaunch a, SwFaces f) {
    const T *P[3] = {(const T *)a.in[0], (const T *)a.in[1], (const T *)a.in[2]};
    T *X[3] = {(T *)f.x[0], (T *)f.x[1], (T *)f.x[2]};
    T *Y[3] = {(T *)f.y[0], (T *)f.y[1], (T *)f.y[2]};
    const int nx = a.nx, ny = a.ny;
    const double dt = step_dt(a);
    const T k = (T)(0.5 * a.g);
    const T lx = (T)(0.5 * dt / a.dx), ly = (T)(0.5 * dt / a.dy);
    const int64_t pitch = a.pitch, fp_ = f.pitch;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (i > nx) return;
    const int band = (ny + 1 + (int)gridDim.y - 1) / (int)gridDim.y;   // consecutive rows per block
    const int jb = (int)blockIdx.y * band, je = min(jb + band, ny + 1);
    for (int j = jb; j < je; ++j) {
        const int64_t oc = (int64_t)j * pitch + i, o = (int64_t)j * fp_ + i;
        const CellParts<T> c = cell_parts(P[0][oc], P[1][oc], P[2][oc], k);
        if (j < ny) {
            const CellParts<T> l = cell_parts(P[0][oc - 1], P[1][oc - 1], P[2][oc - 1], k);
            X[0][o] = fma(lx, l.p, l.hh) + fma(-lx, c.p, c.hh);
            X[1][o] = fma(lx, l.fp, l.hp) + fma(-lx, c.fp, c.hp);
            X[2][o] = fma(lx, l.fq, l.hq) + fma(-lx, c.fq, c.hq);
        }
        if (i < nx) {
            const CellParts<T> b = cell_parts(P[0][oc - pitch], P[1][oc - pitch], P[2][oc - pitch], k);
            Y[0][o] = fma(ly, b.q, b.hh) + fma(-ly, c.q, c.hh);
            Y[1][o] = fma(ly, b.fq, b.hp) + fma(-ly, c.fq, c.hp);
            Y[2][o] = fma(ly, b.gq, b.hq) + fma(-ly, c.gq, c.hq);
        }
    }
}

// Second half-step from the stored face states (thread (i, j), one band of
// consecutive rows per block); epilogue as the fused kernel's.
template <typename T>
__global__ __launch_bounds__(256) void k_update(SwLaunch a, SwFaces f) {
    const T *P[3] = {(const T *)a.in[0], (const T *)a.in[1], (const T *)a.in[2]};
    T *O[3] = {(T *)a.out[0], (T *)a.out[1], (T *)a.out[2]};
    const T *X[3] = {(const T *)f.x[0], (const T *)f.x[1], (const T *)f.x[2]};
    const T *Y[3] = {(const T *)f.y[0], (const T *)f.y[1], (const T *)f.y[2]};
    const int nx = a.nx, ny = a.ny;
    const double dt = step_dt(a);
    const T k = (T)(0.5 * a.g), g = (T)a.g;
    const T mx = (T)(dt / a.dx), my = (T)(dt / a.dy);
    const int64_t pitch = a.pitch, fp_ = f.pitch;
    const int i = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    T smax = T(0);
    bool bad = false;
    if (i < nx) {
        const int band = (ny + (int)gridDim.y - 1) / (int)gridDim.y;    // consecutive rows per block
        const int jb = (int)blockIdx.y * band, je = min(jb + band, ny);
        for (int j = jb; j < je; ++j) {
            const int64_t of = (int64_t)j * fp_ + i;
            T fl[3], fr[3], gd[3], gu[3];
            xface_flux<T>(X[0][of], X[1][of], X[2][of], k, fl);
            xface_flux<T>(X[0][of + 1], X[1][of + 1], X[2][of + 1], k, fr);
            yface_flux<T>(Y[0][of], Y[1][of], Y[2][of], k, gd);
            yface_flux<T>(Y[0][of + fp_], Y[1][of + fp_], Y[2][of + fp_], k, gu);
            const int64_t o = (int64_t)j * pitch + i;
            U3<T> v;
            v.h = fma(-my, gu[0] - gd[0], fma(-mx, fr[0] - fl[0], P[0][o]));
            v.p = fma(-my, gu[1] - gd[1], fma(-mx, fr[1] - fl[1], P[1][o]));
            v.q = fma(-my, gu[2] - gd[2], fma(-mx, fr[2] - fl[2], P[2][o]));
            O[0][o] = v.h;
            O[1][o] = v.p;
            O[2][o] = v.q;
            if (i == 0 || i == nx - 1 || j == 0 || j == ny - 1)
                write_ghosts(O, pitch, nx, ny, a.bc_x, a.bc_y, i, j, v);
            const T sp = signal_speed(v, g);
            bad |= !(sp <= finite_max<T>());
            smax = fmax(smax, sp);
        }
    }
    const int wave = threadIdx.x >> 6;
    const bool first = blockIdx.x == 0 && blockIdx.y == 0 && wave == 0;
    step_epilogue(a, (double)smax, bad, dt, first, (int)(blockIdx.y * gridDim.x + blockIdx.x) * 4 + wave);
}

// ---------------------------------------------------------------------------
// AoS: one (h, hu, hv, 0) vector per cell.

template <typename T> struct alignas(4 * sizeof(T)) V4 {
    T h, p, q, z;
};

// Rows (halo and padding included) between the two layouts: element i of row
// j is s[j * sp + i] in each plane and o[j * op + i] in the AoS array.
template <typename T>
__global__ __launch_bounds__(256) void k_to_aos(const T *h, const T *p, const T *q, int64_t sp, V4<T> *o, int64_t op,
                                                int64_t row, int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / row, i = t - j * row, so = j * sp + i;
        o[j * op + i] = V4<T>{h[so], p[so], q[so], T(0)};
    }
}
template <typename T>
__global__ __launch_bounds__(256) void k_from_aos(const V4<T> *a, int64_t op, T *h, T *p, T *q, int64_t sp, int64_t row,
                                                  int64_t n) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t j = t / row, i = t - j * row, so = j * sp + i;
        const V4<T> v = a[j * op + i];
        h[so] = v.h;
        p[so] = v.p;
        q[so] = v.q;
    }
}

template <typename T>
__device__ __forceinline__ void write_ghosts_aos(V4<T> *o, int64_t pitch, int nx, int ny, int bcx, int bcy, int i,
                                                 int j, U3<T> c) {
    int xt[2], yt[2];
    T xs[2], ys[2];
    int nxt = 0, nyt = 0;
    if (i == 0) { xt[nxt] = bcx ? nx : -1; xs[nxt++] = bcx ? T(1) : T(-1); }
    if (i == nx - 1) { xt[nxt] = bcx ? -1 : nx; xs[nxt++] = bcx ? T(1) : T(-1); }
    if (j == 0) { yt[nyt] = bcy ? ny : -1; ys[nyt++] = bcy ? T(1) : T(-1); }
    if (j == ny - 1) { yt[nyt] = bcy ? -1 : ny; ys[nyt++] = bcy ? T(1) : T(-1); }
    for (int a = 0; a < nxt; ++a) o[(int64_t)j * pitch + xt[a]] = V4<T>{c.h, xs[a] * c.p, c.q, T(0)};
    for (int b = 0; b < nyt; ++b) {
        o[(int64_t)yt[b] * pitch + i] = V4<T>{c.h, c.p, ys[b] * c.q, T(0)};
        for (int a = 0; a < nxt; ++a) o[(int64_t)yt[b] * pitch + xt[a]] = V4<T>{c.h, xs[a] * c.p, ys[b] * c.q, T(0)};
    }
}

// One wave: rows [rb * rows, ...) of the 64-cell strip s; lane l owns
// column s * 64 + l.  Rows are loaded two ahead; the x neighbours of lane 0
// and lane 63 come from one extra vector per row (lanes 0..31 load the
// column left of the strip, lanes 32..63 the one right of it).
template <typename T>
__global__ __launch_bounds__(256) void k_step_aos(SwLaunch a, const V4<T> *in, V4<T> *out, int rows, int nstrips,
                                                  int nrb) {
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int tile = (int)blockIdx.x * 4 + wave;
    const int s = tile % nstrips, rb = tile / nstrips;
    const double dt = step_dt(a);
    const T k = (T)(0.5 * a.g), g = (T)a.g;
    const T lx = (T)(0.5 * dt / a.dx), ly = (T)(0.5 * dt / a.dy);
    const T mx = (T)(dt / a.dx), my = (T)(dt / a.dy);
    const int nx = a.nx, ny = a.ny;
    const int64_t pitch = a.pitch;
    T smax = T(0);
    bool bad = false;
    if (rb < nrb) {
        const int c0 = s * 64, j0 = rb * rows, j1 = min(j0 + rows, ny);
        const int c = c0 + lane;
        const int cl = c <= nx ? c : c0;                       // lanes past the row read the strip's first cell
        const bool right_ok = c0 + 64 <= nx;
        const int ec = (lane < 32 || !right_ok) ? c0 - 1 : c0 + 64;
        const T elx = lane == 0 ? lx : -lx;
        const bool tile_at_wall = s == 0 || c0 + 64 >= nx || j0 == 0 || j1 >= ny;
        auto load = [&](int j, V4<T> &v, V4<T> &e) {
            v = in[(int64_t)j * pitch + cl];
            e = in[(int64_t)j * pitch + ec];
        };
        T S[3], Bp[3], Gd[3];
        auto row = [&](bool face, bool emit, const V4<T> &v, const V4<T> &e, bool want_x, int jout) {
            const CellParts<T> cp = cell_parts(v.h, v.p, v.q, k);
            if (face) {
                T f[3];
                yface_flux<T>(Bp[0] + fma(-ly, cp.q, cp.hh), Bp[1] + fma(-ly, cp.fq, cp.hp),
                              Bp[2] + fma(-ly, cp.gq, cp.hq), k, f);
                if (emit) {
                    U3<T> o3;
                    o3.h = fma(-my, f[0] - Gd[0], S[0]);
                    o3.p = fma(-my, f[1] - Gd[1], S[1]);
                    o3.q = fma(-my, f[2] - Gd[2], S[2]);
                    if (c < nx) {
                        out[(int64_t)jout * pitch + c] = V4<T>{o3.h, o3.p, o3.q, T(0)};
                        const T sp = signal_speed(o3, g);
                        bad |= !(sp <= finite_max<T>());
                        smax = fmax(smax, sp);
                        if (tile_at_wall && (c == 0 || c == nx - 1 || jout == 0 || jout == ny - 1))
                            write_ghosts_aos(out, pitch, nx, ny, a.bc_x, a.bc_y, c, jout, o3);
                    }
                }
#pragma unroll
                for (int kk = 0; kk < 3; ++kk) Gd[kk] = f[kk];
            }
            Bp[0] = fma(ly, cp.q, cp.hh);
            Bp[1] = fma(ly, cp.fq, cp.hp);
            Bp[2] = fma(ly, cp.gq, cp.hq);
            if (!want_x) return;
            T L[3], R[3], E[3];
            L[0] = fma(lx, cp.p, cp.hh);
            L[1] = fma(lx, cp.fp, cp.hp);
            L[2] = fma(lx, cp.fq, cp.hq);
            R[0] = fma(-lx, cp.p, cp.hh);
            R[1] = fma(-lx, cp.fp, cp.hp);
            R[2] = fma(-lx, cp.fq, cp.hq);
            {   // the lane's edge cell: L (lane 0) or R (lane 63) of the column outside the strip
                const T r = fast_rcp(e.h);
                const T u = e.p * r;
                const T fp = fma(k * e.h, e.h, e.p * u);
                const T fq = e.q * u;
                E[0] = fma(elx, e.p, T(0.5) * e.h);
                E[1] = fma(elx, fp, T(0.5) * e.p);
                E[2] = fma(elx, fq, T(0.5) * e.q);
            }
            T Lm[3], Rp[3], fl[3], fr[3];
#pragma unroll
            for (int kk = 0; kk < 3; ++kk) {
                Lm[kk] = from_prev_lane(L[kk], E[kk]);
                Rp[kk] = from_next_lane(R[kk], E[kk]);
            }
            xface_flux<T>(Lm[0] + R[0], Lm[1] + R[1], Lm[2] + R[2], k, fl);
            xface_flux<T>(L[0] + Rp[0], L[1] + Rp[1], L[2] + Rp[2], k, fr);
            S[0] = fma(-mx, fr[0] - fl[0], v.h);
            S[1] = fma(-mx, fr[1] - fl[1], v.p);
            S[2] = fma(-mx, fr[2] - fl[2], v.q);
        };
        // rows j0 - 1 (B only) and j0 (face below, B, x part); then one row
        // finished per row loaded, two rows in flight
        V4<T> v0, e0, v1, e1, v2, e2;
        load(j0 - 1, v0, e0);
        load(j0, v1, e1);
        load(min(j0 + 1, j1), v2, e2);
        row(false, false, v0, e0, false, 0);
        row(true, false, v1, e1, true, 0);
        for (int j = j0; j < j1; ++j) {
            // v2 holds row j + 1
            const V4<T> vc = v2, ec_ = e2;
            load(min(j + 2, j1), v2, e2);
            row(true, true, vc, ec_, j + 1 < j1, j);
        }
    }
    step_epilogue(a, (double)smax, bad, dt, blockIdx.x == 0 && wave == 0, (int)blockIdx.x * 4 + wave);
}

unsigned grid_for(int64_t n) {
    int64_t b = (n + 255) / 256;
    return (unsigned)(b < 65536 ? (b > 0 ? b : 1) : 65536);
}

}  // namespace

hipError_t sw_launch_unfused(const SwLaunch &a, const SwFaces &f, hipStream_t s) {
    if (a.scheme != 0) return hipErrorInvalidValue;
    // about 4096 blocks, each thread looping over rows: the update's CFL
    // epilogue takes one atomic per wave, so the wave count stays bounded
    auto grid2d = [](int cols, int rows) {
        const int gx = (cols + 255) / 256;
        int gy = 4096 / gx;
        gy = gy < 1 ? 1 : (gy > rows ? rows : gy);
        return dim3((unsigned)gx, (unsigned)gy);
    };
    const dim3 gf = grid2d(a.nx + 1, a.ny + 1), gu = grid2d(a.nx, a.ny);
    if (a.dtype == 0) {
        k_faces<float><<<gf, 256, 0, s>>>(a, f);
        k_update<float><<<gu, 256, 0, s>>>(a, f);
    } else {
        k_faces<double><<<gf, 256, 0, s>>>(a, f);
        k_update<double><<<gu, 256, 0, s>>>(a, f);
    }
    return hipGetLastError();
}

hipError_t sw_launch_aos_convert(int dtype, const void *const soa[3], int64_t soa_pitch, void *aos, int64_t aos_pitch,
                                 int64_t rows, bool to_aos, hipStream_t s) {
    // each plane's row is aos_pitch elements: the AoS rows hold exactly one plane row
    const int64_t row = aos_pitch, n = rows * row;
    if (rows < 0 || row < 1 || soa_pitch < row) return hipErrorInvalidValue;
    const unsigned gb = grid_for(n);
    if (dtype == 0) {
        const float *const *q = (const float *const *)soa;
        if (to_aos) k_to_aos<float><<<gb, 256, 0, s>>>(q[0], q[1], q[2], soa_pitch, (V4<float> *)aos, aos_pitch, row, n);
        else k_from_aos<float><<<gb, 256, 0, s>>>((const V4<float> *)aos, aos_pitch, (float *)soa[0], (float *)soa[1],
                                                   (float *)soa[2], soa_pitch, row, n);
    } else {
        const double *const *q = (const double *const *)soa;
        if (to_aos) k_to_aos<double><<<gb, 256, 0, s>>>(q[0], q[1], q[2], soa_pitch, (V4<double> *)aos, aos_pitch, row, n);
        else k_from_aos<double><<<gb, 256, 0, s>>>((const V4<double> *)aos, aos_pitch, (double *)soa[0],
                                                    (double *)soa[1], (double *)soa[2], soa_pitch, row, n);
    }
    return hipGetLastError();
}

hipError_t sw_launch_aos_step(const SwLaunch &a, const void *in, void *out, int rows, hipStream_t s) {
    if (a.scheme != 0 || rows < 1) return hipErrorInvalidValue;
    const int nstrips = (a.nx + 63) / 64;
    const int nrb = (a.ny + rows - 1) / rows;
    const int64_t blocks = ((int64_t)nstrips * nrb + 3) / 4;
    if (blocks > 0x3fffffff) return hipErrorInvalidValue;
    if (a.dtype == 0)
        k_step_aos<float><<<(unsigned)blocks, 256, 0, s>>>(a, (const V4<float> *)in, (V4<float> *)out, rows, nstrips, nrb);
    else
        k_step_aos<double><<<(unsigned)blocks, 256, 0, s>>>(a, (const V4<double> *)in, (V4<double> *)out, rows, nstrips,
                                                            nrb);
    return hipGetLastError();
}
