// Learned-surrogate kernels other than the convolution: input preparation,
// loss and its gradient seed, weight gradients, Adam with the BF16 weight
// re-layout, and the gated rollout (apply, gate statistics, accept).
#include <algorithm>

#include "sw_dma.h"

#include "sw_common.h"
#include "sw_conv.h"

using namespace sw;

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wave_sum_d(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// Source cell of halo pixel index t in [0, n + 2) along one axis (halo
// coordinates): interior t - 1, or the boundary image; *flip = -1 where the
// reflective wall negates that axis' momentum.
__device__ __forceinline__ int src_index(int t, int n, int bc, float *flip) {
    *flip = 1.f;
    if (t == 0) {
        if (bc) return n - 1;
        *flip = -1.f;
        return 0;
    }
    if (t == n + 1) {
        if (bc) return 0;
        *flip = -1.f;
        return n - 1;
    }
    return t - 1;
}

__device__ __forceinline__ void store_x0(__bf16 *x0, float a, float b, float c) {
    bf16x8 v = {(__bf16)a, (__bf16)b, (__bf16)c, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
    *reinterpret_cast<bf16x8 *>(x0) = v;
}

__global__ __launch_bounds__(256) void k_prep_dense(const float *u, const float *u8, int B, int H, int W, int bcx,
                                                    int bcy, SwNorm nrm, __bf16 *x0, float *target) {
    const int Wp = W + 2, Hp = H + 2;
    const int64_t n = (int64_t)B * Hp * Wp;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(idx / ((int64_t)Hp * Wp));
        const int r = (int)(idx - (int64_t)b * Hp * Wp);
        const int yy = r / Wp, xx = r - yy * Wp;
        float fx, fy;
        const int x = src_index(xx, W, bcx, &fx), y = src_index(yy, H, bcy, &fy);
        const int64_t plane = (int64_t)H * W;
        const float *ub = u + (int64_t)b * 3 * plane + (int64_t)y * W + x;
        const float h = ub[0], hu = fx * ub[plane], hv = fy * ub[2 * plane];
        const float c0 = (h - nrm.in_off[0]) / nrm.in_scale[0], c1 = (hu - nrm.in_off[1]) / nrm.in_scale[1],
                    c2 = (hv - nrm.in_off[2]) / nrm.in_scale[2];
        store_x0(x0 + idx * 8, c0, c1, c2);
        if (target && xx >= 1 && xx <= W && yy >= 1 && yy <= H) {
            const float *vb = u8 + (int64_t)b * 3 * plane + (int64_t)y * W + x;
            float *tg = target + (((int64_t)b * H + y) * W + x) * 4;
            tg[0] = (vb[0] - ub[0]) / nrm.out_scale[0];
            tg[1] = (vb[plane] - ub[plane]) / nrm.out_scale[1];
            tg[2] = (vb[2 * plane] - ub[2 * plane]) / nrm.out_scale[2];
            tg[3] = 0.f;
        }
    }
}

__global__ __launch_bounds__(256) void k_loss(const float *pred, const float *target, int B, int H, int W,
                                              float *partial, __bf16 *dz) {
    const int64_t n = (int64_t)B * H * W;
    const float scale = 2.f / (3.f * (float)n);
    float acc = 0.f;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const float4 pr = *reinterpret_cast<const float4 *>(pred + p * 4);
        const float4 tg = *reinterpret_cast<const float4 *>(target + p * 4);
        const float d0 = pr.x - tg.x, d1 = pr.y - tg.y, d2 = pr.z - tg.z;
        acc += d0 * d0 + d1 * d1 + d2 * d2;
        const int b = (int)(p / ((int64_t)H * W));
        const int r = (int)(p - (int64_t)b * H * W);
        const int y = r / W, x = r - y * W;
        const float g0 = scale * d0, g1 = scale * d1, g2 = scale * d2;
        store_x0(dz + (((int64_t)b * (H + 2) + y + 1) * (W + 2) + x + 1) * 8, g0, g1, g2);
    }
    __shared__ float red[4];
    acc = wave_sum_f(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = (red[0] + red[1] + red[2] + red[3]) / (3.f * (float)n);
}

__global__ void k_reduce_sum(const float *partial, int n, float *out) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += blockDim.x) acc += partial[i];
    __shared__ double red[4];
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[0] = (float)(red[0] + red[1] + red[2] + red[3]);
}

// Weight gradient partials on MFMA (v_mfma_f32_16x16x32_bf16), K = pixels:
//     dW[co][(tap, ci)] = sum_p dZ[p][co] A[p + off(tap)][ci]
// read from the NHWC tensors.  Persistent blocks walk contiguous runs of
// 4-row x 64-pixel tiles, numbered down the columns of tiles (the next tile's
// halo rows are still in L2), and keep dW in registers.  A tile's dZ (4 x 64
// pixels) and input rows (6 x 66 pixels, halo included) are staged in LDS
// transposed, channel-major with the pixels contiguous, so 8 consecutive
// pixels of one channel are one 16-byte LDS read (row strides padded so the
// reads of 16 channels are conflict free); the next tile's global loads are
// in flight during the MFMAs.  A K step is 32 pixels of one row: lane
// (n, kg) = (lane % 16, lane / 16) takes pixels j0 = 8 kg .. + 7 of the step.
// Wave w owns input row dy = w / CH and, for CINP = 32, channel half w % CH,
// i.e. the taps (dy, 0..2) of 16 input channels: two aligned reads give all
// three column shifts (dx = 1 by a 16-bit funnel shift, dx = 2 by a dword
// shift).  For CINP = 8 a 16-wide N tile holds two taps of 8 channels.  Wave
// 0 also forms db with an all-ones operand.
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

constexpr int kWgRows = 4, kWgCols = 64;

template <int CINP, int COUTP>
__global__ __launch_bounds__(CINP == 32 ? 384 : 192) void k_wgrad(const __bf16 *dz, const __bf16 *a, int cout, int cin,
                                                                  int H, int W, int tiles_y, int tiles_x, int ntiles,
                                                                  float *partial, int nent) {
    constexpr int CH = CINP == 32 ? 2 : 1;
    constexpr int NTH = 64 * 3 * CH;
    constexpr int MB = (COUTP + 15) / 16;
    constexpr int NT = CINP == 32 ? 3 : 2;
    constexpr int DZS = kWgRows * kWgCols + 8;               // per output channel (padded)
    constexpr int AROW = 72, AS = (kWgRows + 2) * AROW + 8;  // per input channel (padded)
    constexpr int NKO = COUTP / 8, NKI = CINP / 8;
    constexpr int DZ_CH = kWgRows * NKO * kWgCols, A_CH = (kWgRows + 2) * NKI * (kWgCols + 2);
    constexpr int DZ_PER = (DZ_CH + NTH - 1) / NTH, A_PER = (A_CH + NTH - 1) / NTH;
    __shared__ __attribute__((aligned(16))) __bf16 dzT[COUTP * DZS];
    __shared__ __attribute__((aligned(16))) __bf16 aT[CINP * AS];

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int n = lane & 15, kg = lane >> 4;
    const int dy = w / CH, chalf = w % CH;
    const int ci = CINP == 32 ? chalf * 16 + n : (n & 7);
    const int Wp = W + 2;
    const int per_block = (ntiles + gridDim.x - 1) / gridDim.x;
    const int t0 = blockIdx.x * per_block, t1 = min(ntiles, t0 + per_block);
    const u32x4 ones = {0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u};   // bf16 1.0 pairs

    f32x4 acc[MB][NT], accb[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        accb[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[mb][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    bf16x8 sdz[DZ_PER], sa[A_PER];
    auto load_tile = [&](int t) {
        const int b = t / (tiles_y * tiles_x);
        const int r = t - b * tiles_y * tiles_x;
        const int tx = r / tiles_y, ty = r - tx * tiles_y;   // column-major: the next tile is the one below
#pragma unroll
        for (int k = 0; k < DZ_PER; ++k) {   // chunk c = (row * NKO + part) * 64 + p
            const int c = threadIdx.x + k * NTH;
            const int p = c % kWgCols, rp = c / kWgCols;
            const int row = rp / NKO, part = rp - row * NKO;
            const int y = ty * kWgRows + row;
            sdz[k] = bf16x8{};
            if (c < DZ_CH && y < H)
                sdz[k] = *reinterpret_cast<const bf16x8 *>(
                    dz + (((int64_t)b * (H + 2) + y + 1) * Wp + tx * kWgCols + 1 + p) * COUTP + part * 8);
        }
#pragma unroll
        for (int k = 0; k < A_PER; ++k) {    // chunk c = (row * NKI + part) * 66 + p, halo coordinates
            const int c = threadIdx.x + k * NTH;
            const int p = c % (kWgCols + 2), rp = c / (kWgCols + 2);
            const int row = rp / NKI, part = rp - row * NKI;
            const int yy = ty * kWgRows + row;
            sa[k] = bf16x8{};
            if (c < A_CH && yy < H + 2)
                sa[k] = *reinterpret_cast<const bf16x8 *>(
                    a + (((int64_t)b * (H + 2) + yy) * Wp + tx * kWgCols + p) * CINP + part * 8);
        }
    };
    auto store_tile = [&]() {   // transposing writes: lanes of a wave take consecutive pixels
#pragma unroll
        for (int k = 0; k < DZ_PER; ++k) {
            const int c = threadIdx.x + k * NTH;
            if (c >= DZ_CH) continue;
            const int p = c % kWgCols, rp = c / kWgCols;
            const int row = rp / NKO, part = rp - row * NKO;
#pragma unroll
            for (int e = 0; e < 8; ++e) dzT[(part * 8 + e) * DZS + row * kWgCols + p] = sdz[k][e];
        }
#pragma unroll
        for (int k = 0; k < A_PER; ++k) {
            const int c = threadIdx.x + k * NTH;
            if (c >= A_CH) continue;
            const int p = c % (kWgCols + 2), rp = c / (kWgCols + 2);
            const int row = rp / NKI, part = rp - row * NKI;
#pragma unroll
            for (int e = 0; e < 8; ++e) aT[(part * 8 + e) * AS + row * AROW + p] = sa[k][e];
        }
    };

    if (t0 < t1) load_tile(t0);
    for (int t = t0; t < t1; ++t) {
        __syncthreads();                  // the previous tile's reads of LDS are done
        store_tile();
        __syncthreads();
        if (t + 1 < t1) load_tile(t + 1); // in flight during the MFMAs below
#pragma unroll
        for (int kc = 0; kc < 2 * kWgRows; ++kc) {
            const int r = kc >> 1, j0 = (kc & 1) * 32 + 8 * kg;
            bf16x8 aop[MB];
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                const int co = mb * 16 + n;
                aop[mb] = co < COUTP ? *reinterpret_cast<const bf16x8 *>(&dzT[co * DZS + r * kWgCols + j0]) : bf16x8{};
            }
            const __bf16 *row = &aT[ci * AS + (r + dy) * AROW + j0];
            const u32x4 v0 = *reinterpret_cast<const u32x4 *>(row);
            const u32x4 v1 = *reinterpret_cast<const u32x4 *>(row + 8);
            // staged pixel j0 + dx + e is input pixel x0 + j0 + e + dx - 1: dx = 0, 1, 2
            const u32x4 s1 = {__builtin_amdgcn_alignbit(v0[1], v0[0], 16), __builtin_amdgcn_alignbit(v0[2], v0[1], 16),
                              __builtin_amdgcn_alignbit(v0[3], v0[2], 16), __builtin_amdgcn_alignbit(v1[0], v0[3], 16)};
            const u32x4 s2 = {v0[1], v0[2], v0[3], v1[0]};
            bf16x8 bop[NT];
            if (CINP == 32) {
                bop[0] = as_bf16x8(v0);
                bop[1] = as_bf16x8(s1);
                bop[2] = as_bf16x8(s2);
            } else {
                bop[0] = as_bf16x8(n < 8 ? v0 : s1);
                bop[1] = n < 8 ? as_bf16x8(s2) : bf16x8{};
            }
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
                    acc[mb][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[mb], bop[tt], acc[mb][tt], 0, 0, 0);
                if (w == 0) accb[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[mb], as_bf16x8(ones), accb[mb], 0, 0, 0);
            }
        }
    }
    // D[m][n] in lane n + 16 (m / 4), element m % 4
    float *P = partial + (int64_t)blockIdx.x * nent;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int co = mb * 16 + 4 * kg + q;
            if (co >= cout) continue;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) {
                int tap, cc;
                if (CINP == 32) {
                    tap = 3 * dy + tt;
                    cc = ci;
                } else {
                    tap = 3 * dy + (tt == 0 ? (n >> 3) : 2);
                    cc = n & 7;
                    if (tt == 1 && n >= 8) continue;
                }
                if (cc < cin) P[(co * 9 + tap) * cin + cc] = acc[mb][tt][q];
            }
            if (w == 0 && n == 0) P[cout * 9 * cin + co] = accb[mb][q];
        }
}

typedef short i16x4 __attribute__((ext_vector_type(4)));

// Offset (BF16 elements) of 16-byte chunk c (channels 8c .. 8c + 7) of pixel
// p in a pixel-major 32-channel LDS tile.  The chunk index is XORed with
// pixel bits 1-2 (the same chunk of 8 consecutive pixels covers all bank
// quads) and with pixel bit 3 into chunk bit 1 (a transposing read takes two
// chunks of pixels p .. p + 3 and p + 8 .. p + 11 in one pass; they then fall
// on disjoint banks).
__device__ __forceinline__ int wg_chunk(int p, int c) {
    return p * 32 + ((c ^ ((p >> 1) & 3) ^ ((p >> 2) & 2)) << 3);
}

// Channel-major read of a pixel-major tile with ds_read_b64_tr_b16 (gfx950):
// within each group of 16 lanes, lane i reads 4 16-bit elements and lane j
// receives element (j & 3) of the reads of lanes 4 e + (j >> 2), e = 0..3
// (probed on MI355X).  With lane i reading channels c0 + 4 (i & 3) .. + 3 of
// pixel p0 + (i >> 2), lane j of the group receives channel c0 + j of pixels
// p0 .. p0 + 3.  Two reads give the 8 consecutive pixels of one channel that
// an MFMA operand lane holds (i: the lane's index in its group).
__device__ __forceinline__ bf16x8 wg_pixels8(const __bf16 *tile, int p0, int c0, int i) {
    const int ch = c0 + 4 * (i & 3);
    const __bf16 *lo = tile + wg_chunk(p0 + (i >> 2), ch >> 3) + (ch & 7);
    const __bf16 *hi = tile + wg_chunk(p0 + 4 + (i >> 2), ch >> 3) + (ch & 7);
    const i16x4 x = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4 *)lo);
    const i16x4 y = __builtin_amdgcn_ds_read_tr16_b64_v4i16((__attribute__((address_space(3))) i16x4 *)hi);
    const i16x4 v[2] = {x, y};
    return __builtin_bit_cast(bf16x8, v);
}

// Weight gradient of a 32 -> 32 layer: k_wgrad's tile walk and MFMA
// operands for 32 channels, with the tiles brought in by LDS DMA,
// pixel-major as they lie in HBM, three buffers deep (two tiles' loads in
// flight while one is computed; one workgroup per CU, the buffers fill 123 KB
// of LDS), and the operands read channel-major with transposing LDS reads
// instead of staged transposed.  12 waves: wave w takes input row dy = u / 2
// and channel half u % 2 (u = w % 6) of the K steps over pixel half w / 6 of
// each tile row (three waves per SIMD hide each other's LDS latency); the
// two halves' sums meet in LDS at the end.  A tile's 16-byte slots: dZ (4 x
// 64 pixels) then the input (6 x 66 pixels, padded to whole DMA
// instructions; padding lanes reload a slot of the window and land past its
// end); slot s holds chunk (s & 3) ^ swizzle of pixel s >> 2 (wg_chunk).  dZ
// rows below the image (the last tile row of an image whose height is not a
// multiple of 4) are loaded from its last row and their K steps skipped;
// input rows below the bottom halo row feed only those steps.  The loop
// issues no vector memory operation other than the DMA, so waiting for all
// but the newest tile's DMA instructions leaves exactly that tile in flight.
__global__ __launch_bounds__(768) void k_wgrad_dma(const __bf16 *dz, const __bf16 *a, int cout, int cin, int H, int W,
                                                    int tiles_y, int tiles_x, int ntiles, float *partial, int nent) {
    constexpr int NWV = 12, MB = 2, NT = 3;
    constexpr int DZ_SLOTS = kWgRows * kWgCols * 4;
    constexpr int A_SLOTS = (kWgRows + 2) * (kWgCols + 2) * 4;
    constexpr int DZ_NI = DZ_SLOTS / 64;
    constexpr int A_NI = (A_SLOTS + 63) / 64;
    constexpr int NI = DZ_NI + A_NI;                 // DMA instructions per tile
    constexpr int BUF = NI * 64 * 8;                 // bf16 per buffer
    constexpr int PERW = (NI + NWV - 1) / NWV;       // most instructions of one wave
    constexpr int NBUF = 3;
    constexpr int NACC = MB * NT * 4 + MB * 4;       // a lane's sums (with the bias's)
    static_assert(6 * 64 * NACC * 4 <= NBUF * BUF * 2, "the halves' sums fit the tile buffers");
    __shared__ __attribute__((aligned(16))) __bf16 tiles[NBUF][BUF];

    const int lane = threadIdx.x & 63, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int n = lane & 15, kg = lane >> 4;
    const int u = w % 6, half = w / 6;
    const int dy = u >> 1, chalf = u & 1;
    const bool bias_wave = u == 0;
    const int Wp = W + 2;
    const int per_block = (ntiles + gridDim.x - 1) / gridDim.x;
    const int t0 = blockIdx.x * per_block, t1 = min(ntiles, t0 + per_block);
    const u32x4 ones = {0x3F803F80u, 0x3F803F80u, 0x3F803F80u, 0x3F803F80u};   // bf16 1.0 pairs

    f32x4 acc[MB][NT], accb[MB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        accb[mb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[mb][t] = f32x4{0.f, 0.f, 0.f, 0.f};
    }

    // this wave's DMA instructions i = w + 12 k (k < nw): per lane the slot's
    // byte offset from its window's first pixel, and its window row
    const int nw = (NI - w + NWV - 1) / NWV;
    unsigned soff[PERW];
    int srow[PERW];
#pragma unroll
    for (int k = 0; k < PERW; ++k) {
        const int i = w + NWV * k;
        const bool isdz = i < DZ_NI;
        const int cols = isdz ? kWgCols : kWgCols + 2;
        int sl = (isdz ? i : i - DZ_NI) * 64 + lane;
        if (!isdz && sl >= A_SLOTS) sl = lane;
        const int p = sl >> 2, c = (sl & 3) ^ ((p >> 1) & 3) ^ ((p >> 2) & 2);
        const int row = p / cols, col = p - row * cols;
        soff[k] = (unsigned)(((row * Wp + col) * 32 + c * 8) * 2);
        srow[k] = row;
    }
    const unsigned lds0 = lds_addr(&tiles[0][0]);
    auto issue = [&](int t, int buf) {
        const int b = t / (tiles_y * tiles_x);
        const int r = t - b * tiles_y * tiles_x;
        const int tx = r / tiles_y, ty = r - tx * tiles_y;   // column-major: the next tile is the one below
        const char *zb = (const char *)(dz + ((((int64_t)b * (H + 2) + ty * kWgRows + 1) * Wp + tx * kWgCols + 1) * 32));
        const char *ab = (const char *)(a + ((((int64_t)b * (H + 2) + ty * kWgRows) * Wp + tx * kWgCols) * 32));
        const int rz = H - 1 - ty * kWgRows, ra = H + 1 - ty * kWgRows;   // last window rows inside the image
        const unsigned l0 = lds0 + (unsigned)(buf * BUF * 2);
#pragma unroll
        for (int k = 0; k < PERW; ++k) {
            if (k < nw) {
                const int i = w + NWV * k;
                const bool isdz = i < DZ_NI;
                const int rm = isdz ? rz : ra;
                const unsigned off = srow[k] > rm ? soff[k] - (unsigned)((srow[k] - rm) * Wp * 64) : soff[k];
                lds_dma16(isdz ? zb : ab, off, l0 + (unsigned)(i * 1024));
            }
        }
    };

    if (t0 < t1) {
        issue(t0, 0);
        if (t0 + 1 < t1) issue(t0 + 1, 1);
        wait_vm_upto<PERW>(t0 + 1 < t1 ? nw : 0);      // tile t0 has landed
    }
    __syncthreads();
    for (int t = t0; t < t1; ++t) {
        const int buf = (t - t0) % NBUF;
        if (t + 2 < t1) issue(t + 2, (t - t0 + 2) % NBUF);   // its buffer was last read before the barrier
        const int r0 = t - (t / (tiles_y * tiles_x)) * tiles_y * tiles_x;
        const int ty = r0 - (r0 / tiles_y) * tiles_y;
        const int rows = min(kWgRows, H - ty * kWgRows);
        const __bf16 *DZ = tiles[buf];
        const __bf16 *AT = tiles[buf] + DZ_SLOTS * 8;
#pragma unroll
        for (int r = 0; r < kWgRows; ++r) {
            if (r >= rows) break;
            const int j0 = half * 32 + 8 * kg;
            bf16x8 aop[MB], bop[NT];
            // dZ: channel mb * 16 + n of pixels j0 .. j0 + 7 of row r; the
            // input: channel 16 chalf + n of staged pixels j0 + dx .. + 7 of row r + dy
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) aop[mb] = wg_pixels8(DZ, r * kWgCols + j0, mb * 16, n);
#pragma unroll
            for (int dx = 0; dx < NT; ++dx) bop[dx] = wg_pixels8(AT, (r + dy) * (kWgCols + 2) + j0 + dx, chalf * 16, n);
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
                    acc[mb][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[mb], bop[tt], acc[mb][tt], 0, 0, 0);
                if (bias_wave)
                    accb[mb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(aop[mb], as_bf16x8(ones), accb[mb], 0, 0, 0);
            }
        }
        if (t + 1 < t1) wait_vm_upto<PERW>(t + 2 < t1 ? nw : 0);   // tile t + 1 has landed
        __syncthreads();
    }
    // the second pixel half's sums join the first's (the tile buffers are free)
    float *X = reinterpret_cast<float *>(&tiles[0][0]) + (u * 64 + lane) * NACC;
    if (half == 1) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
#pragma unroll
                for (int q = 0; q < 4; ++q) X[(mb * NT + tt) * 4 + q] = acc[mb][tt][q];
#pragma unroll
            for (int q = 0; q < 4; ++q) X[MB * NT * 4 + mb * 4 + q] = accb[mb][q];
        }
    }
    __syncthreads();
    if (half == 1) return;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
#pragma unroll
        for (int tt = 0; tt < NT; ++tt)
#pragma unroll
            for (int q = 0; q < 4; ++q) acc[mb][tt][q] += X[(mb * NT + tt) * 4 + q];
#pragma unroll
        for (int q = 0; q < 4; ++q) accb[mb][q] += X[MB * NT * 4 + mb * 4 + q];
    }
    // D[m][n] in lane n + 16 (m / 4), element m % 4
    float *P = partial + (int64_t)blockIdx.x * nent;
    const int ci = chalf * 16 + n;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int co = mb * 16 + 4 * kg + q;
            if (co >= cout) continue;
#pragma unroll
            for (int tt = 0; tt < NT; ++tt)
                if (ci < cin) P[(co * 9 + 3 * dy + tt) * cin + ci] = acc[mb][tt][q];
            if (bias_wave && n == 0) P[cout * 9 * cin + co] = accb[mb][q];
        }
}

// Sum of the block partials per entry: 64 entries per block, four partial
// sums per entry over interleaved blocks, combined in LDS (FP64).
__global__ __launch_bounds__(256) void k_wgrad_reduce(const float *partial, int nblocks, int nent, int nw, float *grad_w,
                                                      float *grad_b) {
    const int e = blockIdx.x * 64 + (threadIdx.x & 63), part = threadIdx.x >> 6;
    double acc = 0.0;
    if (e < nent) {
        int k = part;
        for (; k + 12 < nblocks; k += 16) {
            const float a0 = partial[(int64_t)k * nent + e], a1 = partial[(int64_t)(k + 4) * nent + e];
            const float a2 = partial[(int64_t)(k + 8) * nent + e], a3 = partial[(int64_t)(k + 12) * nent + e];
            acc += ((double)a0 + (double)a1) + ((double)a2 + (double)a3);
        }
        for (; k < nblocks; k += 4) acc += partial[(int64_t)k * nent + e];
    }
    __shared__ double red[4][64];
    red[part][threadIdx.x & 63] = acc;
    __syncthreads();
    if (part == 0 && e < nent) {
        const double sum = (red[0][threadIdx.x] + red[1][threadIdx.x]) + (red[2][threadIdx.x] + red[3][threadIdx.x]);
        if (e < nw) grad_w[e] = (float)sum;
        else grad_b[e - nw] = (float)sum;
    }
}

__global__ void k_adam(float *master, float *m, float *v, const float *grad, int64_t n, SwAdam ad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = grad[i];
    const float mi = ad.beta1 * m[i] + (1.f - ad.beta1) * g;
    const float vi = ad.beta2 * v[i] + (1.f - ad.beta2) * g * g;
    m[i] = mi;
    v[i] = vi;
    master[i] -= ad.lr * (mi * ad.c1) / (sqrtf(vi * ad.c2) + ad.eps);
}

// One thread per weight of every layer: write its BF16 copies.
__global__ void k_relayout(const float *master, const SwLayerDesc *layers, int nlayers, int64_t total) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    int l = 0;
    while (l < nlayers) {
        const int64_t nw = (int64_t)layers[l].cout * 9 * layers[l].cin;
        if (i < nw) break;
        i -= nw;
        ++l;
    }
    if (l >= nlayers) return;
    const SwLayerDesc &L = layers[l];
    const int ci = (int)(i % L.cin), tap = (int)((i / L.cin) % 9), co = (int)(i / (9 * L.cin));
    const float w = master[L.w_off + i];
    reinterpret_cast<__bf16 *>(L.wk)[(int64_t)co * L.kp + tap * L.cinp + ci] = (__bf16)w;
    if (L.wd) reinterpret_cast<__bf16 *>(L.wd)[(int64_t)ci * L.kpd + (8 - tap) * L.cdp + co] = (__bf16)w;
}

// Per grid (blockIdx.y): U' = U + denorm(delta) (less the mean dh when
// projecting) into buffer cur ^ 1 with its ghosts, and the gate statistics.
// The mean dh comes from the output layer's per-row sums, added by every
// block in the same fixed order (so every block, and every run, gets the
// same value).
__global__ __launch_bounds__(256) void k_apply(const float *delta, const double *dh_part, int nparts,
                                               const SwBatchGrid *grids, int cur, int H, int W, SwNorm nrm, int project,
                                               int bcx, int bcy, SwGateStats *st, SwApplyPart *part,
                                               unsigned *ticket) {
    const int b = blockIdx.y;
    const SwBatchGrid &g = grids[b];
    const int64_t n = (int64_t)H * W;
    const float *U[3] = {(const float *)g.plane[cur][0], (const float *)g.plane[cur][1], (const float *)g.plane[cur][2]};
    float *O[3] = {(float *)g.plane[cur ^ 1][0], (float *)g.plane[cur ^ 1][1], (float *)g.plane[cur ^ 1][2]};
    // a thread's pixels in pairs, a pair's loads issued together (the first
    // pair's before the projection's sum, which they do not need)
    struct Px {
        float4 d;
        float h, hu, hv;
        int x, y;
        int64_t off;
        bool live;
    };
    auto fetch = [&](int64_t q, Px &v) {
        v.live = q < n;
        if (!v.live) return;
        if (n <= 0x7fffffff) {
            v.y = (int)q / W;
            v.x = (int)q - v.y * W;
        } else {
            v.y = (int)(q / W);
            v.x = (int)(q - (int64_t)v.y * W);
        }
        v.off = (int64_t)v.y * g.pitch + v.x;
        v.d = *reinterpret_cast<const float4 *>(delta + ((int64_t)b * n + q) * 4);
        v.h = U[0][v.off];
        v.hu = U[1][v.off];
        v.hv = U[2][v.off];
    };
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Px pa, pb;
    fetch(p, pa);
    fetch(p + stride, pb);
    float dh_mean = 0.f;
    if (project) {
        __shared__ double s_part[4];
        const double *part = dh_part + (int64_t)b * nparts;
        double acc = 0.0;
        for (int k = threadIdx.x; k < nparts; k += blockDim.x) acc += part[k];
        acc = wave_sum_d(acc);
        if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
        __syncthreads();
        dh_mean = (float)(((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])) / (double)n);
    }
    double mo = 0.0, mn = 0.0;
    float hmin = 3.0e38f;
    bool bad = false;
    auto emit = [&](const Px &v) {
        U3<float> c = {v.h + (v.d.x - dh_mean) * nrm.out_scale[0], v.hu + v.d.y * nrm.out_scale[1],
                       v.hv + v.d.z * nrm.out_scale[2]};
        O[0][v.off] = c.h;
        O[1][v.off] = c.p;
        O[2][v.off] = c.q;
        if (v.x == 0 || v.x == W - 1 || v.y == 0 || v.y == H - 1) write_ghosts(O, g.pitch, W, H, bcx, bcy, v.x, v.y, c);
        mo += v.h;
        mn += c.h;
        hmin = fminf(hmin, c.h);
        bad |= !(fabsf(c.h) <= 3.0e38f) || !(fabsf(c.p) <= 3.0e38f) || !(fabsf(c.q) <= 3.0e38f);
    };
    while (pa.live) {
        emit(pa);
        if (!pb.live) break;
        emit(pb);
        p += 2 * stride;
        fetch(p, pa);
        fetch(p + stride, pb);
    }
    mo = wave_sum_d(mo);
    mn = wave_sum_d(mn);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) hmin = fminf(hmin, __shfl_xor(hmin, o));
    const unsigned long long anybad = __ballot(bad);
    // The four waves' partial results meet in LDS; each block then publishes
    // its partials in its own slot with device-scope atomic exchanges
    // (performed where every XCD sees them) and takes a ticket; the block
    // with the last ticket sums the slots in block order and writes the
    // grid's statistics, then clears the ticket.  Per grid that is one
    // contended atomic per block, where atomics on the statistics themselves
    // (four per block, one cache line) serialised into microseconds for the
    // few grids of a small batch.
    __shared__ double s_mo[4], s_mn[4];
    __shared__ float s_hmin[4];
    __shared__ int s_bad[4];
    __shared__ int s_last;
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_mo[w] = mo;
        s_mn[w] = mn;
        s_hmin[w] = hmin;
        s_bad[w] = anybad != 0;
    }
    __syncthreads();
    const unsigned nb = gridDim.x;
    SwApplyPart *P = part + (int64_t)b * nb;
    if (threadIdx.x == 0) {
        const double bmo = (s_mo[0] + s_mo[1]) + (s_mo[2] + s_mo[3]);
        const double bmn = (s_mn[0] + s_mn[1]) + (s_mn[2] + s_mn[3]);
        const float hm = fminf(fminf(s_hmin[0], s_hmin[1]), fminf(s_hmin[2], s_hmin[3]));
        const unsigned bd = (unsigned)(s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]);
        unsigned long long r = atomicExch(&P[blockIdx.x].mo, (unsigned long long)__double_as_longlong(bmo));
        r ^= atomicExch(&P[blockIdx.x].mn, (unsigned long long)__double_as_longlong(bmn));
        r ^= atomicExch(&P[blockIdx.x].hmin_bad, ((unsigned long long)__float_as_uint(hm) << 32) | bd);
        // the exchanges have returned (so are performed) before the ticket is taken
        asm volatile("" : "+v"(r)::"memory");
        const unsigned t = atomicAdd(&ticket[b], 1u);
        s_last = t == nb - 1;
    }
    __syncthreads();
    if (!s_last) return;                              // uniform per block
    // every block's slot is published: per thread a strided run of slots in
    // block order, then the waves and the block in a fixed order
    double tmo = 0.0, tmn = 0.0;
    float thm = 3.0e38f;
    unsigned tbad = 0u;
    for (unsigned k = threadIdx.x; k < nb; k += blockDim.x) {
        tmo += __longlong_as_double((long long)atomicAdd(&P[k].mo, 0ull));
        tmn += __longlong_as_double((long long)atomicAdd(&P[k].mn, 0ull));
        const unsigned long long hb = atomicAdd(&P[k].hmin_bad, 0ull);
        thm = fminf(thm, __uint_as_float((unsigned)(hb >> 32)));
        tbad |= (unsigned)hb;
    }
    tmo = wave_sum_d(tmo);
    tmn = wave_sum_d(tmn);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) thm = fminf(thm, __shfl_xor(thm, o));
    const unsigned long long wbad = __ballot(tbad != 0u);
    __syncthreads();                                  // the LDS slots are reused
    if ((threadIdx.x & 63) == 0) {
        s_mo[w] = tmo;
        s_mn[w] = tmn;
        s_hmin[w] = thm;
        s_bad[w] = wbad != 0ull;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        st[b].mass_old = (s_mo[0] + s_mo[1]) + (s_mo[2] + s_mo[3]);
        st[b].mass_new = (s_mn[0] + s_mn[1]) + (s_mn[2] + s_mn[3]);
        const float hm = fminf(fminf(s_hmin[0], s_hmin[1]), fminf(s_hmin[2], s_hmin[3]));
        st[b].hmin = hm > 0.f ? hm : 0.f;             // a non-positive depth is recorded as 0
        st[b].nonfinite = (unsigned)(s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]);
        atomicExch(&ticket[b], 0u);                   // ready for the next launch
    }
}

// Per grid (blockIdx.y): the gate's verdict on the jump from its statistics
// (mass drift, least depth, non-finite values; every block derives it, block
// 0 records it in active, st and fallbacks), then for a rejected grid the
// whole halo'd rectangle of buffer cur copied into cur ^ 1.
__global__ __launch_bounds__(256) void k_gate_restore(const SwBatchGrid *grids, int cur, int H, int W, SwGateStats *st,
                                                      double mass_tol, double hmin, int *active, int *fallbacks) {
    const int b = blockIdx.y;
    const double mass_old = st[b].mass_old, mass_new = st[b].mass_new;
    const double drift = fabs(mass_new - mass_old) / fabs(mass_old);
    const int reject = !(drift <= mass_tol) || !((double)st[b].hmin > hmin) || st[b].nonfinite != 0u;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        st[b].fallback = reject;
        active[b] = reject;
        if (fallbacks) fallbacks[b] += reject;
    }
    if (!reject) return;
    const SwBatchGrid &g = grids[b];
    const int64_t n = (int64_t)(H + 2) * (W + 2);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int yy = (int)(p / (W + 2)), xx = (int)(p - (int64_t)yy * (W + 2));
        const int64_t off = (int64_t)(yy - 1) * g.pitch + (xx - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) ((float *)g.plane[cur ^ 1][k])[off] = ((const float *)g.plane[cur][k])[off];
    }
}

// Judge, before the rollout: remember every grid's time and step count and
// clear the sums.
__global__ void k_judge_begin(const SwBatchScalars *sc, int B, SwJudge *j) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    j[b].d2 = 0.0;
    j[b].r2 = 0.0;
    j[b].t0 = sc[b].t;
    j[b].steps0 = sc[b].steps;
}

// Per grid (blockIdx.y): sums of (h - h_ref)^2 and h_ref^2 over the interior.
__global__ __launch_bounds__(256) void k_judge_sums(const SwBatchGrid *ga, int cur_a, const SwBatchGrid *gr,
                                                    int cur_r, int H, int W, SwJudge *j) {
    const int b = blockIdx.y;
    const float *A = (const float *)ga[b].plane[cur_a][0];
    const float *R = (const float *)gr[b].plane[cur_r][0];
    const int64_t pa = ga[b].pitch, pr = gr[b].pitch, n = (int64_t)H * W;
    double d2 = 0.0, r2 = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const double r = R[y * pr + x], d = (double)A[y * pa + x] - r;
        d2 += d * d;
        r2 += r * r;
    }
    d2 = wave_sum_d(d2);
    r2 = wave_sum_d(r2);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&j[b].d2, d2);
        atomicAdd(&j[b].r2, r2);
    }
}

__global__ void k_judge_decide(SwJudge *j, int B, SwBatchScalars *sc, const SwBatchScalars *rsc, double l2_tol,
                               int jumps, int *reject, int *fallbacks, double *l2) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const double e = sqrt(j[b].d2 / j[b].r2);
    const int rej = !(e <= l2_tol);
    reject[b] = rej;
    if (l2) l2[b] = e;
    if (rej) {
        if (fallbacks) fallbacks[b] = jumps;
        sc[b].t = j[b].t0 + rsc[b].t;
        sc[b].last_dt = rsc[b].last_dt;
        sc[b].steps = j[b].steps0 + rsc[b].steps;
        sc[b].unstable = rsc[b].unstable;   // the rollout's history is discarded
    }
}

// Rejected grids: copy the solver's halo'd rectangle (buffer cur) over the rollout's.
__global__ __launch_bounds__(256) void k_judge_copy(const SwBatchGrid *ga, int cur_a, const SwBatchGrid *gr,
                                                    int cur_r, int H, int W, const int *reject) {
    const int b = blockIdx.y;
    if (!reject[b]) return;
    const int64_t n = (int64_t)(H + 2) * (W + 2);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int yy = (int)(p / (W + 2)), xx = (int)(p - (int64_t)yy * (W + 2));
        const int64_t oa = (int64_t)(yy - 1) * ga[b].pitch + (xx - 1), orr = (int64_t)(yy - 1) * gr[b].pitch + (xx - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) ((float *)ga[b].plane[cur_a][k])[oa] = ((const float *)gr[b].plane[cur_r][k])[orr];
    }
}

unsigned grid_for(int64_t n, int cap = 16384) {
    int64_t b = (n + 255) / 256;
    if (b > cap) b = cap;
    if (b < 1) b = 1;
    return (unsigned)b;
}

}  // namespace

hipError_t sw_sur_prep_dense(const float *u, const float *u8, int B, int H, int W, int bc_x, int bc_y, SwNorm nrm,
                             void *x0, float *target, hipStream_t s) {
    k_prep_dense<<<grid_for((int64_t)B * (H + 2) * (W + 2)), 256, 0, s>>>(u, u8, B, H, W, bc_x, bc_y, nrm,
                                                                           (__bf16 *)x0, u8 ? target : nullptr);
    return hipGetLastError();
}


hipError_t sw_sur_loss(const float *pred, const float *target, int B, int H, int W, float *partial, int nblocks,
                       void *dz, hipStream_t s) {
    k_loss<<<nblocks, 256, 0, s>>>(pred, target, B, H, W, partial, (__bf16 *)dz);
    return hipGetLastError();
}

hipError_t sw_sur_reduce_sum(const float *partial, int n, float *out, hipStream_t s) {
    k_reduce_sum<<<1, 256, 0, s>>>(partial, n, out);
    return hipGetLastError();
}

template <int CINP, int COUTP>
hipError_t launch_wgrad(const __bf16 *dz, const __bf16 *a, int cout, int cin, int B, int H, int W, float *partial,
                        int maxblocks, int nent, int *used, hipStream_t s) {
    constexpr int threads = CINP == 32 ? 384 : 192;
    static const int resident = [] {   // blocks of this instance that fit on one CU at once
        int r = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_wgrad<CINP, COUTP>, threads, 0) == hipSuccess && r > 0
                   ? r
                   : 1;
    }();
    const int cus = sw_device_cus();
    const int tiles_y = (H + kWgRows - 1) / kWgRows, tiles_x = W / kWgCols;
    const int64_t ntiles = (int64_t)B * tiles_y * tiles_x;
    if (ntiles > (int64_t)1 << 30) return hipErrorInvalidValue;
    const int nb = (int)std::min<int64_t>({ntiles, (int64_t)cus * resident, (int64_t)maxblocks});
    k_wgrad<CINP, COUTP><<<nb, threads, 0, s>>>(dz, a, cout, cin, H, W, tiles_y, tiles_x, (int)ntiles, partial, nent);
    *used = nb;
    return hipGetLastError();
}

hipError_t launch_wgrad_dma(const __bf16 *dz, const __bf16 *a, int cout, int cin, int B, int H, int W, float *partial,
                            int maxblocks, int nent, int *used, hipStream_t s) {
    const int tiles_y = (H + kWgRows - 1) / kWgRows, tiles_x = W / kWgCols;
    const int64_t ntiles = (int64_t)B * tiles_y * tiles_x;
    if (ntiles > (int64_t)1 << 30) return hipErrorInvalidValue;
    const int nb = (int)std::min<int64_t>({ntiles, (int64_t)sw_device_cus(), (int64_t)maxblocks});   // one per CU (LDS)
    k_wgrad_dma<<<nb, 768, 0, s>>>(dz, a, cout, cin, H, W, tiles_y, tiles_x, (int)ntiles, partial, nent);
    *used = nb;
    return hipGetLastError();
}

hipError_t sw_sur_wgrad(const void *dzv, int coutp, int cout, const void *av, int cinp, int cin, int B, int H, int W,
                        float *partial, int nblocks, float *grad_w, float *grad_b, hipStream_t s) {
    if (W % kWgCols != 0 || nblocks < 1 || cout > coutp || cin > cinp) return hipErrorInvalidValue;
    const int nent = cout * 9 * cin + cout;
    const __bf16 *dz = (const __bf16 *)dzv, *a = (const __bf16 *)av;
    int used = 0;
    hipError_t e;
    if (cinp == 32 && coutp == 32)
        e = launch_wgrad_dma(dz, a, cout, cin, B, H, W, partial, nblocks, nent, &used, s);
    else if (cinp == 8 && coutp == 32)
        e = launch_wgrad<8, 32>(dz, a, cout, cin, B, H, W, partial, nblocks, nent, &used, s);
    else if (cinp == 32 && coutp == 8)
        e = launch_wgrad<32, 8>(dz, a, cout, cin, B, H, W, partial, nblocks, nent, &used, s);
    else
        return hipErrorInvalidValue;
    if (e != hipSuccess) return e;
    k_wgrad_reduce<<<(nent + 63) / 64, 256, 0, s>>>(partial, used, nent, cout * 9 * cin, grad_w, grad_b);
    return hipGetLastError();
}

hipError_t sw_sur_adam(float *master, float *m, float *v, const float *grad, int64_t n, SwAdam ad, hipStream_t s) {
    k_adam<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(master, m, v, grad, n, ad);
    return hipGetLastError();
}

hipError_t sw_sur_relayout(const float *master, const SwLayerDesc *layers, int nlayers, int64_t total_weights,
                           hipStream_t s) {
    k_relayout<<<(unsigned)((total_weights + 255) / 256), 256, 0, s>>>(master, layers, nlayers, total_weights);
    return hipGetLastError();
}

// Blocks per grid of the per-grid passes: up to one element per thread for
// small batches (their few grids would otherwise leave most CUs idle and
// walk the pixels serially), 64 per grid from 256 grids up.
unsigned per_grid_blocks(int64_t n, int B) {
    const int cap = B >= 256 ? 64 : std::max(64, 16384 / std::max(B, 1));
    return grid_for(n, cap);
}


unsigned sw_sur_apply_slots(int64_t pixels, int B) { return per_grid_blocks(pixels, 1) * (unsigned)B; }

hipError_t sw_sur_apply(const float *delta, const double *dh_part, int nparts, const SwBatchGrid *grids, int cur,
                        int B, int H, int W, SwNorm nrm, int project, int bcx, int bcy, SwGateStats *st,
                        SwApplyPart *part, unsigned *ticket, hipStream_t s) {
    if (project && (!dh_part || nparts < 1)) return hipErrorInvalidValue;
    if (!part || !ticket) return hipErrorInvalidValue;
    // at most 128 blocks per grid (two pixels per thread on a 256^2 grid):
    // the blocks of one grid meet on its ticket
    dim3 grid(std::min(per_grid_blocks((int64_t)H * W, B), 128u), B);
    k_apply<<<grid, 256, 0, s>>>(delta, dh_part, nparts, grids, cur, H, W, nrm, project, bcx, bcy, st, part, ticket);
    return hipGetLastError();
}

hipError_t sw_sur_gate_restore(const SwBatchGrid *grids, int cur, int B, int H, int W, SwGateStats *st,
                               double mass_tol, double hmin, int *active, int *fallbacks, hipStream_t s) {
    dim3 grid(per_grid_blocks((int64_t)(H + 2) * (W + 2), B), B);
    k_gate_restore<<<grid, 256, 0, s>>>(grids, cur, H, W, st, mass_tol, hmin, active, fallbacks);
    return hipGetLastError();
}

hipError_t sw_sur_judge_begin(const SwBatchScalars *sc, int B, SwJudge *j, hipStream_t s) {
    k_judge_begin<<<(B + 255) / 256, 256, 0, s>>>(sc, B, j);
    return hipGetLastError();
}

hipError_t sw_sur_judge(const SwBatchGrid *a, int cur_a, const SwBatchGrid *ref, int cur_ref, int B, int H, int W,
                        SwJudge *j, SwBatchScalars *sc, const SwBatchScalars *ref_sc, double l2_tol, int jumps,
                        int *reject, int *fallbacks, double *l2, hipStream_t s) {
    k_judge_sums<<<dim3(grid_for((int64_t)H * W, 64), B), 256, 0, s>>>(a, cur_a, ref, cur_ref, H, W, j);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_judge_decide<<<(B + 255) / 256, 256, 0, s>>>(j, B, sc, ref_sc, l2_tol, jumps, reject, fallbacks, l2);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    k_judge_copy<<<dim3(grid_for((int64_t)(H + 2) * (W + 2), 64), B), 256, 0, s>>>(a, cur_a, ref, cur_ref, H, W, reject);
    return hipGetLastError();
}
