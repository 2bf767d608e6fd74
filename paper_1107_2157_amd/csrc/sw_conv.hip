// 3x3 "same" convolution on MFMA (gfx950, v_mfma_f32_16x16x32_bf16), the
// building block of the learned surrogate's forward and input-gradient passes.
//
// Tensors are NHWC BF16 with a one-pixel halo: X[b][y + 1][x + 1][c] over
// (H + 2) x (W + 2) pixels per image.  The convolution is an implicit GEMM
//     out[co][p] = sum_k Wk[co][k] * X[p + tap(k)][ci(k)],   k = tap * CIN + ci
// with the weights as the M x K operand and 16 output pixels as the K x N
// operand, so after an MFMA each lane holds 4 consecutive output channels of
// one pixel (one 8-byte store).  Per 32-wide K step, CIN = 32 covers one tap
// (lane group g = lane / 16 takes channels 8g..8g+7), CIN = 8 covers four taps
// (lane group g takes tap 4 * kstep + g, all 8 channels).  Taps beyond 8 and
// channels beyond the real ones are zero in Wk.
//
// Operand layouts of v_mfma_f32_16x16x32_bf16 (checked on the GPU by a lane
// probe): A[m][k] in lane m + 16 * (k / 8), element k % 8; B[k][n] in lane
// n + 16 * (k / 8), element k % 8; D[m][n] in lane n + 16 * (m / 4), element
// m % 4.
#include "sw_conv.h"
#include "sw_dma.h"

#include <algorithm>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int CIN> constexpr int ksteps() { return CIN == 32 ? 9 : 3; }

constexpr int kTileCols = 64;               // output pixels per tile row (4 MFMA N blocks)
constexpr int kStageCols = kTileCols + 2;   // staged pixels per row (halo)

// Offset (BF16 elements) of 16-byte chunk c (channels 8c .. 8c + 7) of pixel
// p in an LDS area of 32-channel pixels.  The chunk index is XORed with bits
// 1-2 of the pixel index.  A ds_read_b128 is served 8 lanes (128 bytes, 32
// banks) at a time, and 8 lanes of an MFMA operand read the same chunk of 8
// consecutive pixels: at a plain 64-byte pixel stride those fall on 2 of the
// 8 bank quads, a 4-way conflict (measured: about 70 % of the convolutions'
// LDS cycles were bank-conflict cycles); swizzled they cover all 8.
__device__ __forceinline__ int chunk_off(int p, int c) { return p * 32 + ((c ^ ((p >> 1) & 3)) << 3); }

// Persistent, LDS-staged 3x3 convolution.  Each block owns a contiguous run
// of ROWS-row x 64-pixel output tiles (ROWS = waves per block), numbered down
// the columns of tiles, so the tile a block takes next is the one below the
// last and re-reads two of its staged rows while they are still in L2 (with
// the run along the rows, counters showed 1.5x the input bytes coming from
// HBM), and keeps the layer's weights (the MFMA A operands of every K step)
// in registers for its whole life.  A tile's input
// rows ((ROWS + 2) x 66 pixels x CIN channels, halo included) are staged in LDS, double
// buffered: the global loads of tile t + 1 are in flight while the MFMAs of
// tile t read LDS.  Wave w computes output row w of the tile: per K step one
// 16-byte LDS read per 16-pixel block gives the B operand (16 pixels x 64 B
// per wave, chunks swizzled by chunk_off so that the reads are conflict
// free).  Runs the 8-channel input layer and the input-gradient mode; the
// 32-channel forward modes run k_conv3x3_dma below, which keeps two tiles'
// loads in flight.
template <int CIN, int COUT, int MODE, int ROWS>
__global__ __launch_bounds__(64 * ROWS, 2) void k_conv3x3(SwConvArgs a, int tiles_y, int tiles_x, int ntiles) {
    constexpr int NT = 64 * ROWS;
    constexpr int MB = (COUT + 15) / 16;
    constexpr int KS = ksteps<CIN>();
    constexpr int KP = KS * 32;
    constexpr int NPB = kTileCols / 16;
    constexpr int STAGE = (ROWS + 2) * kStageCols * CIN;          // bf16 per buffer
    constexpr int CHUNKS = STAGE / 8;                             // 16-byte chunks per tile
    constexpr int PER = (CHUNKS + NT - 1) / NT;                   // per thread
    __shared__ __attribute__((aligned(16))) __bf16 tile[2][STAGE];
    __shared__ __attribute__((aligned(16))) __bf16 ostage[ROWS][kTileCols * (COUT > 16 ? COUT : 16)];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int g = lane >> 4, n = lane & 15;
    const int Wp = a.W + 2;
    const int per_block = (ntiles + gridDim.x - 1) / gridDim.x;
    const int t0 = blockIdx.x * per_block;
    const int t1 = min(ntiles, t0 + per_block);
    if (t0 >= t1) return;                                          // uniform per block: no barrier is skipped by part of it

    // weights: A operand of K step ks, M block mb (row mb*16 + n, k = ks*32 + 8g .. + 7)
    bf16x8 wa[KS][MB];
    const __bf16 *Wk = (const __bf16 *)a.w;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            wa[ks][mb] = *reinterpret_cast<const bf16x8 *>(Wk + (int64_t)(mb * 16 + n) * KP + ks * 32 + 8 * g);

    const __bf16 *X = (const __bf16 *)a.x;
    bf16x8 stg[PER];
    auto load_tile = [&](int t) {
        const int b = t / (tiles_y * tiles_x);
        const int r = t - b * tiles_y * tiles_x;
        const int tx = r / tiles_y, ty = r - tx * tiles_y;        // column-major: the next tile is the one below
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int c = threadIdx.x + k * NT;
            const int row = c / (kStageCols * CIN / 8), rem = c - row * (kStageCols * CIN / 8);
            const int yy = ty * ROWS + row;                        // halo row of the input
            stg[k] = bf16x8{};
            if (c < CHUNKS && yy < a.H + 2) {
                if constexpr (MODE == SW_CONV_RELU_PLANES) {
                    // CIN = 8: one chunk is one pixel (h, hu, hv, 0 ...) of grid b's
                    // buffer cur, normalised as the dense input preparation does
                    const SwBatchGrid &gd = a.grids[b];
                    const int64_t off = (int64_t)(yy - 1) * gd.pitch + (tx * kTileCols + rem - 1);
                    const float h = ((const float *)gd.plane[a.cur][0])[off];
                    const float hu = ((const float *)gd.plane[a.cur][1])[off];
                    const float hv = ((const float *)gd.plane[a.cur][2])[off];
                    stg[k] = bf16x8{(__bf16)((h - a.nrm.in_off[0]) / a.nrm.in_scale[0]),
                                    (__bf16)((hu - a.nrm.in_off[1]) / a.nrm.in_scale[1]),
                                    (__bf16)((hv - a.nrm.in_off[2]) / a.nrm.in_scale[2]),
                                    (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
                } else {
                    stg[k] = *reinterpret_cast<const bf16x8 *>(
                        X + (((int64_t)b * (a.H + 2) + yy) * Wp + tx * kTileCols) * CIN + rem * 8);
                }
            }
        }
    };
    auto store_tile = [&](int buf) {   // chunk c: pixel c / 4, chunk c % 4 (CIN = 32, swizzled) or pixel c (CIN = 8)
#pragma unroll
        for (int k = 0; k < PER; ++k) {
            const int c = threadIdx.x + k * NT;
            if (c < CHUNKS)
                *reinterpret_cast<bf16x8 *>(&tile[buf][CIN == 32 ? chunk_off(c >> 2, c & 3) : c * 8]) = stg[k];
        }
    };

    load_tile(t0);
    store_tile(0);
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        const int buf = (t - t0) & 1;
        if (t + 1 < t1) load_tile(t + 1);                         // in flight during the MFMAs below
        const int b = t / (tiles_y * tiles_x);
        const int r = t - b * tiles_y * tiles_x;
        const int tx = r / tiles_y, ty = r - tx * tiles_y;        // column-major: the next tile is the one below
        const int y = ty * ROWS + w;                               // output row of this wave
        const int x0 = tx * kTileCols;
        const __bf16 *T = tile[buf];
        if constexpr (MODE == SW_CONV_RELU_PLANES) {                // a grid's first tile clears its statistics
            if (a.clear_stats && ty == 0 && tx == 0 && threadIdx.x == 0) {
                SwGateStats &st = a.clear_stats[b];
                st.mass_old = 0.0;
                st.mass_new = 0.0;
                st.hmin = 3.0e38f;
                st.nonfinite = 0u;
            }
        }

        f32x4 acc[MB][NPB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) acc[mb][pb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int tap = CIN == 32 ? ks : 4 * ks + g;
            const int ci0 = CIN == 32 ? 8 * g : 0;
            const bool live = tap < 9;
            const int dy = live ? tap / 3 : 1, dx = live ? tap % 3 : 1;
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                const int px = (w + dy) * kStageCols + pb * 16 + n + dx;
                bf16x8 xb = *reinterpret_cast<const bf16x8 *>(T + (CIN == 32 ? chunk_off(px, g) : px * CIN + ci0));
                if (!live) xb = bf16x8{};
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ks][mb], xb, acc[mb][pb], 0, 0, 0);
            }
        }

        // epilogue: lane holds channels co = mb*16 + 4g .. +3 of pixel x0 + pb*16 + n
        if (y < a.H) {
            if (MODE == SW_CONV_F32) {   // channels 0..3 (COUT <= 4) with bias, FP32, no halo
                double dh = 0.0;         // this lane's channel-0 outputs, for the row sums
#pragma unroll
                for (int pb = 0; pb < NPB; ++pb) {
                    if (g != 0) continue;
                    f32x4 v = acc[0][pb];
                    float *Y = a.yf + (((int64_t)b * a.H + y) * a.W + x0 + pb * 16 + n) * 4;
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = q < COUT ? v[q] + a.bias[q] : 0.f;
                    *reinterpret_cast<f32x4 *>(Y) = v;
                    dh += (double)v[0];
                }
                if (a.dh_part) {         // fixed-order sum of the wave's 64 pixels (one tile row)
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) dh += __shfl_xor(dh, o);
                    if (lane == 0) a.dh_part[((int64_t)b * a.H + y) * tiles_x + tx] = dh;
                }
            } else {
                // The wave's 64 output pixels x COUT channels are one contiguous run of the
                // NHWC row: values go to the wave's LDS area, then out as 16 contiguous bytes
                // per lane.  Two outputs (RESID's ReLU part, DGRAD's dZ) reuse the area in turn.
                const int64_t row0 = (((int64_t)b * (a.H + 2) + y + 1) * Wp + x0 + 1) * COUT;
                // the area holds the wave's 64 pixels x 32 channels, chunks swizzled as the input tile's
                auto slot = [&](int mb, int pb) -> bf16x4 & {
                    return *reinterpret_cast<bf16x4 *>(&ostage[w][chunk_off(pb * 16 + n, 2 * mb + (g >> 1)) + 4 * (g & 1)]);
                };
                auto wave_sync = [] {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                };
                auto flush = [&](__bf16 *dst) {
                    wave_sync();
#pragma unroll
                    for (int k = 0; k < kTileCols * COUT / 512; ++k) {   // non-temporal: GB-sized tensors
                        const int e = k * 512 + lane * 8;                 // chunk (e / 8) % 4 of pixel e / 32
                        __builtin_nontemporal_store(
                            *reinterpret_cast<const bf16x8 *>(&ostage[w][chunk_off(e >> 5, (e >> 3) & 3)]),
                            reinterpret_cast<bf16x8 *>(dst + row0 + e));
                    }
                    wave_sync();   // the copy's reads are done before the area is written again
                };
                auto relu_part = [&](int mb, int pb) {
                    f32x4 v = acc[mb][pb];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q] + a.bias[mb * 16 + 4 * g + q], 0.f);
                    return v;
                };
                if (MODE == SW_CONV_RELU_BF16 || MODE == SW_CONV_RELU_PLANES || MODE == SW_CONV_RESID_BF16) {
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int pb = 0; pb < NPB; ++pb) {
                            f32x4 v = relu_part(mb, pb);
                            if (MODE == SW_CONV_RESID_BF16) {   // CIN == COUT: the block's input at this pixel, from LDS
                                const bf16x4 xin = *reinterpret_cast<const bf16x4 *>(
                                    T + chunk_off((w + 1) * kStageCols + pb * 16 + n + 1, 2 * mb + (g >> 1)) + 4 * (g & 1));
#pragma unroll
                                for (int q = 0; q < 4; ++q) v[q] += (float)xin[q];
                            }
                            slot(mb, pb) = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                        }
                    flush((__bf16 *)a.y);
                    if (MODE == SW_CONV_RESID_BF16 && a.y2) {
#pragma unroll
                        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                            for (int pb = 0; pb < NPB; ++pb) {
                                const f32x4 v = relu_part(mb, pb);
                                slot(mb, pb) = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                            }
                        flush((__bf16 *)a.y2);
                    }
                } else {   // SW_CONV_DGRAD: G = conv + add into y (if set), dZ = G where mask > 0 into y2
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int pb = 0; pb < NPB; ++pb) {
                            f32x4 v = acc[mb][pb];
                            if (a.add) {
                                const bf16x4 ad = *reinterpret_cast<const bf16x4 *>(
                                    (const __bf16 *)a.add + row0 + (pb * 16 + n) * COUT + mb * 16 + 4 * g);
#pragma unroll
                                for (int q = 0; q < 4; ++q) v[q] += (float)ad[q];
                            }
                            slot(mb, pb) = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                        }
                    if (a.y) flush((__bf16 *)a.y);
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int pb = 0; pb < NPB; ++pb) {   // each lane rewrites only its own values
                            const bf16x4 mk = *reinterpret_cast<const bf16x4 *>(
                                (const __bf16 *)a.mask + row0 + (pb * 16 + n) * COUT + mb * 16 + 4 * g);
                            bf16x4 gv = slot(mb, pb);
#pragma unroll
                            for (int q = 0; q < 4; ++q) gv[q] = (float)mk[q] > 0.f ? gv[q] : (__bf16)0.f;
                            slot(mb, pb) = gv;
                        }
                    flush((__bf16 *)a.y2);
                }
            }
        }
        if (t + 1 < t1) store_tile(buf ^ 1);                      // buffer buf ^ 1 was last read before the previous barrier
        __syncthreads();
    }
}

}  // namespace

// Compute units of the current device (queried once; thread-safe initialisation).
int sw_device_cus() {
    static const int cus = [] {
        int dev = 0;
        hipDeviceProp_t p;
        return (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) ? p.multiProcessorCount
                                                                                                   : 256;
    }();
    return cus;
}

namespace {

constexpr int kDmaRows = 8;   // tile height of the LDS DMA kernel

// The forward 32-channel modes (residual block, output layer) with the
// input tiles brought in by LDS DMA, three buffers deep: while tile t is
// computed, the loads of tiles t + 1 and t + 2 are in flight and hold no
// registers.  With 8-row tiles (one workgroup of 8 waves per CU: three
// 43 KB input buffers and the waves' 4 KB output staging areas fill the
// 160 KB of LDS) two tiles' loads, 86 KB, are in flight per CU.  Same
// operands, MFMA order and output staging as k_conv3x3, hence the same
// results.
//
// A tile's (ROWS + 2) x 66 staged pixels are 16-byte slots; slot s holds
// chunk (s & 3) ^ ((p >> 1) & 3) of pixel p = s >> 2 (the chunk_off
// layout), so one DMA instruction fills 64 consecutive slots.  The slots
// are padded to whole instructions; the padding lanes load a slot of the
// window again and land past its end.  Rows past the image's bottom halo
// row (below the last tile of an image whose height is not a multiple of
// ROWS) are loaded from that halo row: they feed only outputs that are
// never stored.
template <int COUT, int MODE, int ROWS>
__global__ __launch_bounds__(64 * ROWS, 1) void k_conv3x3_dma(SwConvArgs a, int tiles_y, int tiles_x, int ntiles) {
    constexpr int CIN = 32;
    constexpr int OST = MODE == SW_CONV_RESID_BF16 ? kTileCols * COUT : 8;   // output staging per wave (bf16)
    constexpr int MB = (COUT + 15) / 16;
    constexpr int KS = ksteps<CIN>();
    constexpr int KP = KS * 32;
    constexpr int NPB = kTileCols / 16;
    constexpr int SLOTS = (ROWS + 2) * kStageCols * 4;
    constexpr int NI = (SLOTS + 63) / 64;          // DMA instructions per tile
    constexpr int BUF = NI * 64 * 8;               // bf16 per buffer
    constexpr int PERW = (NI + ROWS - 1) / ROWS;   // most instructions of one wave
    constexpr int NBUF = 3;
    static_assert(MODE == SW_CONV_RESID_BF16 || MODE == SW_CONV_F32, "forward 32-channel modes only");
    __shared__ __attribute__((aligned(16))) __bf16 tile[NBUF][BUF];
    __shared__ __attribute__((aligned(16))) __bf16 ostage[ROWS][OST];

    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, n = lane & 15;
    const int Wp = a.W + 2;
    const int per_block = (ntiles + gridDim.x - 1) / gridDim.x;
    const int t0 = blockIdx.x * per_block;
    const int t1 = min(ntiles, t0 + per_block);
    if (t0 >= t1) return;                          // uniform per block: no barrier is skipped by part of it

    bf16x8 wa[KS][MB];
    const __bf16 *Wk = (const __bf16 *)a.w;
#pragma unroll
    for (int ks = 0; ks < KS; ++ks)
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            wa[ks][mb] = *reinterpret_cast<const bf16x8 *>(Wk + (int64_t)(mb * 16 + n) * KP + ks * 32 + 8 * g);
    float bias[MB][4];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q)
            bias[mb][q] = MODE == SW_CONV_F32 ? (q < COUT ? a.bias[q] : 0.f) : a.bias[mb * 16 + 4 * g + q];

    // this wave's DMA instructions i = w + ROWS k (k < nw): per lane the
    // slot's byte offset from the window's first pixel, and its window row
    const int nw = (NI - w + ROWS - 1) / ROWS;
    unsigned soff[PERW];
    int srow[PERW];
#pragma unroll
    for (int k = 0; k < PERW; ++k) {
        int sl = (w + ROWS * k) * 64 + lane;
        if (sl >= SLOTS) sl = lane;                // padding: reload a slot of the window
        const int p = sl >> 2, c = (sl & 3) ^ ((p >> 1) & 3);
        const int row = p / kStageCols, col = p - row * kStageCols;
        soff[k] = (unsigned)(((row * Wp + col) * CIN + c * 8) * 2);
        srow[k] = row;
    }
    const char *X = (const char *)a.x;
    auto issue = [&](int t, int buf) {
        const int b = t / (tiles_y * tiles_x);
        const int r = t - b * tiles_y * tiles_x;
        const int tx = r / tiles_y, ty = r - tx * tiles_y;
        const char *base = X + ((((int64_t)b * (a.H + 2) + ty * ROWS) * Wp + tx * kTileCols) * CIN) * 2;
        const int rmax = a.H + 1 - ty * ROWS;      // last window row inside the image's halo
        const unsigned l0 = lds_addr(&tile[0][0]) + (unsigned)(buf * BUF * 2);
#pragma unroll
        for (int k = 0; k < PERW; ++k) {
            if (k < nw) {
                const unsigned off =
                    srow[k] > rmax ? soff[k] - (unsigned)((srow[k] - rmax) * Wp * CIN * 2) : soff[k];
                lds_dma16(base, off, l0 + (unsigned)((w + ROWS * k) * 1024));
            }
        }
    };

    issue(t0, 0);
    if (t0 + 1 < t1) issue(t0 + 1, 1);
    wait_vm_upto<PERW>(t0 + 1 < t1 ? nw : 0);      // tile t0 has landed (t0 + 1 may be in flight)
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        const int buf = (t - t0) % NBUF;
        if (t + 2 < t1) issue(t + 2, (t - t0 + 2) % NBUF);   // its buffer was last read before the barrier
        const int b = t / (tiles_y * tiles_x);
        const int r = t - b * tiles_y * tiles_x;
        const int tx = r / tiles_y, ty = r - tx * tiles_y;
        const int y = ty * ROWS + w;
        const int x0 = tx * kTileCols;
        const __bf16 *T = tile[buf];

        f32x4 acc[MB][NPB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) acc[mb][pb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
            const int dy = ks / 3, dx = ks % 3;
#pragma unroll
            for (int pb = 0; pb < NPB; ++pb) {
                const int px = (w + dy) * kStageCols + pb * 16 + n + dx;
                const bf16x8 xb = *reinterpret_cast<const bf16x8 *>(T + chunk_off(px, g));
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    acc[mb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ks][mb], xb, acc[mb][pb], 0, 0, 0);
            }
        }

        int stores = 0;                            // vector memory operations issued below
        if (y < a.H) {
            if constexpr (MODE == SW_CONV_F32) {
                double dh = 0.0;
                if (g == 0) {
#pragma unroll
                    for (int pb = 0; pb < NPB; ++pb) {
                        f32x4 v = acc[0][pb];
                        float *Y = a.yf + (((int64_t)b * a.H + y) * a.W + x0 + pb * 16 + n) * 4;
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] = q < COUT ? v[q] + bias[0][q] : 0.f;
                        *reinterpret_cast<f32x4 *>(Y) = v;
                        dh += (double)v[0];
                    }
                }
                stores = NPB;
                if (a.dh_part) {
#pragma unroll
                    for (int o = 32; o > 0; o >>= 1) dh += __shfl_xor(dh, o);
                    if (lane == 0) a.dh_part[((int64_t)b * a.H + y) * tiles_x + tx] = dh;
                    stores += 1;
                }
            } else {
                // the wave's 64 pixels x 32 channels are one contiguous run of the
                // NHWC row: staged in the wave's LDS area (chunks swizzled as the
                // input tile's), then stored as 16 contiguous bytes per lane
                const int64_t row0 = (((int64_t)b * (a.H + 2) + y + 1) * Wp + x0 + 1) * COUT;
                auto slot = [&](int mb, int pb) -> bf16x4 & {
                    return *reinterpret_cast<bf16x4 *>(&ostage[w][chunk_off(pb * 16 + n, 2 * mb + (g >> 1)) + 4 * (g & 1)]);
                };
                auto wave_sync = [] {
                    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                    __builtin_amdgcn_wave_barrier();
                    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                };
                constexpr int FL = kTileCols * COUT / 512;    // 16-byte stores per lane per output
                auto flush = [&](__bf16 *dst) {
                    wave_sync();
#pragma unroll
                    for (int k = 0; k < FL; ++k) {
                        const int e = k * 512 + lane * 8;
                        __builtin_nontemporal_store(
                            *reinterpret_cast<const bf16x8 *>(&ostage[w][chunk_off(e >> 5, (e >> 3) & 3)]),
                            reinterpret_cast<bf16x8 *>(dst + row0 + e));
                    }
                    wave_sync();
                };
                auto relu_part = [&](int mb, int pb) {
                    f32x4 v = acc[mb][pb];
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q] + bias[mb][q], 0.f);
                    return v;
                };
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int pb = 0; pb < NPB; ++pb) {
                        f32x4 v = relu_part(mb, pb);
                        const bf16x4 xin = *reinterpret_cast<const bf16x4 *>(
                            T + chunk_off((w + 1) * kStageCols + pb * 16 + n + 1, 2 * mb + (g >> 1)) + 4 * (g & 1));
#pragma unroll
                        for (int q = 0; q < 4; ++q) v[q] += (float)xin[q];
                        slot(mb, pb) = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                    }
                flush((__bf16 *)a.y);
                stores = FL;
                if (a.y2) {
#pragma unroll
                    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                        for (int pb = 0; pb < NPB; ++pb) {
                            const f32x4 v = relu_part(mb, pb);
                            slot(mb, pb) = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                        }
                    flush((__bf16 *)a.y2);
                    stores += FL;
                }
            }
        }
        // tile t + 1 has landed: newer than its loads are tile t + 2's loads
        // and this tile's stores (the previous tile's stores are older still).
        // `stores` counts the store instructions issued above (one per
        // 16-byte lane store of a flush, one per f32x4 store, the row sum);
        // the loop issues no other vector memory operation.  A count below
        // the true one only waits longer.
        if (t + 1 < t1) wait_vm_upto<PERW + (MODE == SW_CONV_F32 ? NPB + 1 : 2 * kTileCols * COUT / 512)>(
            (t + 2 < t1 ? nw : 0) + stores);
        __syncthreads();
    }
}

template <int COUT, int MODE>
hipError_t launch_dma(const SwConvArgs &a, hipStream_t s) {
    constexpr int ROWS = kDmaRows;
    if (a.W % kTileCols != 0) return hipErrorInvalidValue;
    const int tiles_y = (a.H + ROWS - 1) / ROWS, tiles_x = a.W / kTileCols;
    const int64_t ntiles = (int64_t)a.B * tiles_y * tiles_x;
    if (ntiles > (int64_t)1 << 30) return hipErrorInvalidValue;
    static const int resident = [] {
        int r = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_conv3x3_dma<COUT, MODE, ROWS>, 64 * ROWS, 0) == hipSuccess &&
                       r > 0
                   ? r
                   : 1;
    }();
    int64_t blocks = std::min<int64_t>(ntiles, (int64_t)sw_device_cus() * resident);
    if (a.max_blocks > 0) blocks = std::min<int64_t>(blocks, a.max_blocks);
    k_conv3x3_dma<COUT, MODE, ROWS><<<(unsigned)blocks, 64 * ROWS, 0, s>>>(a, tiles_y, tiles_x, (int)ntiles);
    return hipGetLastError();
}

template <int CIN, int COUT, int MODE, int ROWS>
hipError_t launch(const SwConvArgs &a, hipStream_t s) {
    if (a.W % kTileCols != 0) return hipErrorInvalidValue;
    const int tiles_y = (a.H + ROWS - 1) / ROWS, tiles_x = a.W / kTileCols;
    const int64_t ntiles = (int64_t)a.B * tiles_y * tiles_x;
    if (ntiles > (int64_t)1 << 30) return hipErrorInvalidValue;
    static const int resident = [] {   // blocks of this instance that fit on one CU at once
        int r = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_conv3x3<CIN, COUT, MODE, ROWS>, 64 * ROWS, 0) ==
                               hipSuccess &&
                       r > 0
                   ? r
                   : 1;
    }();
    int64_t blocks = std::min<int64_t>(ntiles, (int64_t)sw_device_cus() * resident);
    if (a.max_blocks > 0) blocks = std::min<int64_t>(blocks, a.max_blocks);
    k_conv3x3<CIN, COUT, MODE, ROWS><<<(unsigned)blocks, 64 * ROWS, 0, s>>>(a, tiles_y, tiles_x, (int)ntiles);
    return hipGetLastError();
}

// Tile height of the 8-channel forward modes (register-staged kernel).
// 8-row tiles (staged input rows 1.25x the rows written instead of 1.5x, one
// block of 8 waves per CU instead of two of 4) measured the same forward
// time at 256 x 256 x 256: the halo rows are served by L2, not HBM.
constexpr int kFwdRows = 4;

}  // namespace

hipError_t sw_conv3x3(const SwConvArgs &a, int cin, int cout, int mode, hipStream_t s) {
    if (a.B < 1 || a.H < 1 || a.W < 1 || (!a.x && mode != SW_CONV_RELU_PLANES) || !a.w) return hipErrorInvalidValue;
    if (mode == SW_CONV_F32 ? !a.yf || !a.bias : mode == SW_CONV_DGRAD ? !a.y2 || !a.mask : !a.y || !a.bias)
        return hipErrorInvalidValue;
    if (cin == 8 && cout == 32 && mode == SW_CONV_RELU_BF16) return launch<8, 32, SW_CONV_RELU_BF16, kFwdRows>(a, s);
    if (cin == 8 && cout == 32 && mode == SW_CONV_RELU_PLANES) {
        if (!a.grids || a.cur < 0 || a.cur > 1) return hipErrorInvalidValue;
        return launch<8, 32, SW_CONV_RELU_PLANES, kFwdRows>(a, s);
    }
    if (cin == 32 && cout == 32 && mode == SW_CONV_RESID_BF16)
        return launch_dma<32, SW_CONV_RESID_BF16>(a, s);
    if (cin == 32 && cout == 3 && mode == SW_CONV_F32) return launch_dma<3, SW_CONV_F32>(a, s);
    if (cin == 32 && cout == 32 && mode == SW_CONV_DGRAD) return launch<32, 32, SW_CONV_DGRAD, 4>(a, s);
    if (cin == 8 && cout == 32 && mode == SW_CONV_DGRAD) return launch<8, 32, SW_CONV_DGRAD, 4>(a, s);
    return hipErrorInvalidValue;
}
