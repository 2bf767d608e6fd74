// The rollout's whole network in one kernel: each workgroup takes a TH x TW
// output tile and runs all six layers on it with the activations in LDS, so
// the only HBM traffic of a jump's forward pass is the state read once (with
// a 6-pixel border) and the FP32 prediction written once.
//
// Layer l (1..6) is evaluated over the tile grown by 6 - l pixels on every
// side, so that layer l + 1 finds all its 3x3 inputs: the input region is
// (TH + 12) x (TW + 12) pixels, layer 1 writes (TH + 10) x (TW + 10), ...,
// layer 6 only the tile.  Hidden activations outside the grid are set to
// zero, which is the zero padding of the layer that reads them; the input's
// one-pixel ring outside the grid comes from the state's ghost cells (the
// boundary conditions), as in the per-layer path.  Every MFMA takes the same
// operands in the same order as the per-layer kernel (k_conv3x3): weights as
// the 16-row A operand per K step, 16 pixels as the B operand, FP32
// accumulation tap by tap, then bias, ReLU, the residual add and the BF16
// rounding in the same expression order.  The prediction is therefore
// bitwise that of the per-layer path; only the recomputed border costs
// extra (1.77x the flops at 16 x 16 tiles, 1.54x at 16 x 32).
//
// LDS regions are dense, row-major, with their own widths: X (input, 8
// channels, 16 B per pixel), A (layers 1, 3, 5) and B (layers 2, 4), 32
// channels (64 B per pixel, its 16-byte chunks swizzled by chunk_off); X and
// B share one area (X is dead once layer 1 has run), so a 16 x 16 tile needs
// 80 KB and two workgroups fit on a CU.  Per K step a lane reads one 16-byte
// chunk; the 64 lanes of a wave read 16 pixels x 64 B.
#include "sw_conv.h"

#include <algorithm>

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBorder = 6;   // one pixel per 3x3 layer

// Offset (BF16 elements) of 16-byte chunk c (channels 8c .. 8c + 7) of pixel
// p in a 32-channel LDS region.  The chunk index is XORed with bits 1-2 of
// the pixel index: a ds_read_b128 is served 8 lanes (128 bytes, 32 banks) at
// a time, and those 8 lanes read the same chunk of 8 consecutive pixels,
// which at a plain 64-byte pixel stride fall on 2 of the 8 bank quads (a
// 4-way conflict); swizzled they cover all 8.
__device__ __forceinline__ int chunk_off(int p, int c) { return p * 32 + ((c ^ ((p >> 1) & 3)) << 3); }

template <int TH, int TW> struct Geo {
    static constexpr int h(int l) { return TH + 2 * (kBorder - l); }   // rows of layer l's region (l = 0: input)
    static constexpr int w(int l) { return TW + 2 * (kBorder - l); }
    static constexpr int X_ELEMS = h(0) * w(0) * 8;
    static constexpr int A_ELEMS = h(1) * w(1) * 32;
    static constexpr int B_ELEMS = h(2) * w(2) * 32;
    // X is read only by layer 1 and B first written by layer 2: they share one area
    static constexpr int XB_ELEMS = X_ELEMS > B_ELEMS ? X_ELEMS : B_ELEMS;
};

// The A operand of M block mb, K step ks of a layer with KS K steps (forward
// layout: row mb * 16 + n, K elements ks * 32 + 8 g .. + 7).
template <int KS>
__device__ __forceinline__ bf16x8 load_wk(const __bf16 *Wk, int mb, int ks, int n, int g) {
    return *reinterpret_cast<const bf16x8 *>(Wk + (int64_t)(mb * 16 + n) * (KS * 32) + ks * 32 + 8 * g);
}

// One layer over its region.  Wave w owns the pixel blocks w, w + NW, ...
// (NB of them, the last possibly a padding block that stores nothing) and
// keeps an accumulator per block; the K steps run outermost, so only one K
// step's weights (the A operands of the M blocks, from the forward layout
// in global memory: row mb * 16 + n, K elements ks * 32 + 8 g .. + 7) and
// its B operands are live, and the next step's are loaded while this step's
// MFMAs run.  Each accumulator still sums its K steps in order, as the
// per-layer kernel does.  MODE 0: A = relu(Z) (first layer), 1: A = A_prev +
// relu(Z) (residual blocks), 2: FP32 Z to the prediction (output layer,
// channels 0..2; returns this lane's sum of channel 0 over the pixels it
// stored).  (gy0, gx0): grid coordinates of the region's first pixel; bias:
// the layer's biases in LDS.  wcur holds the weights of K step 0 on entry
// and, on return, those of the next layer (next_wk), loaded during this
// layer's last K steps, after which at_last() issues the caller's own loads
// (the next tile's input), so that no wait for this layer's operands waits
// for them.
template <int CIN, int COUT, int MODE, int WOUT, int HOUT, int NW, int MBN, int KSN, typename AtLast>
__device__ __forceinline__ double run_layer(const __bf16 *src, __bf16 *dst, const void *wk, bf16x8 (&wcur)[2],
                                            const void *next_wk, const float *bias, int gy0, int gx0, int H, int W,
                                            float *out, int64_t out_row0, AtLast &&at_last) {
    constexpr int KS = CIN == 32 ? 9 : 3;
    constexpr int MB = (COUT + 15) / 16;
    constexpr int NPIX = WOUT * HOUT;
    constexpr int NBLK = (NPIX + 15) / 16;
    constexpr int NB = (NBLK + NW - 1) / NW;     // blocks per wave
    constexpr int WIN = WOUT + 2;                // source region width
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int g = lane >> 4, n = lane & 15;
    const __bf16 *Wk = (const __bf16 *)wk;
    int sb[NB], pp[NB];
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        const int p = (wave + k * NW) * 16 + n;
        pp[k] = p;
        const int pc = p < NPIX ? p : NPIX - 1;  // padding lanes and blocks read a real pixel, store nothing
        const int r = pc / WOUT;
        sb[k] = r * WIN + (pc - r * WOUT);
    }
    auto load_w = [&](int ks, bf16x8 (&wa)[MB]) {
#pragma unroll
        for (int mb = 0; mb < MB; ++mb) wa[mb] = load_wk<KS>(Wk, mb, ks, n, g);
    };
    auto load_b = [&](int ks, bf16x8 (&xb)[NB]) {
        const int tap = CIN == 32 ? ks : 4 * ks + g;
        const bool live = tap < 9;
        const int off = live ? (tap / 3) * WIN + tap % 3 : 0;
#pragma unroll
        for (int k = 0; k < NB; ++k) {
            if (CIN == 32)
                xb[k] = *reinterpret_cast<const bf16x8 *>(src + chunk_off(sb[k] + off, g));
            else
                xb[k] = *reinterpret_cast<const bf16x8 *>(src + (sb[k] + off) * 8);
            if (!live) xb[k] = bf16x8{};
        }
    };
    f32x4 acc[MB][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int k = 0; k < NB; ++k) acc[mb][k] = f32x4{0.f, 0.f, 0.f, 0.f};
    // weights run WD K steps ahead (a global load's latency is longer than one
    // K step's MFMAs), B operands one step ahead
    constexpr int WD = KS > 2 ? 2 : 1;
    bf16x8 wa[WD + 1][MB], xb[2][NB];
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) wa[0][mb] = wcur[mb];
#pragma unroll
    for (int d = 1; d < WD; ++d) load_w(d, wa[d]);
    load_b(0, xb[0]);
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        if (ks + WD < KS) load_w(ks + WD, wa[(ks + WD) % (WD + 1)]);
        if (ks + WD == KS) {   // the next layer's first weights (MBN M blocks, KSN K steps)
#pragma unroll
            for (int mb = 0; mb < MBN; ++mb) wcur[mb] = load_wk<KSN>((const __bf16 *)next_wk, mb, 0, n, g);
        }
        if (ks + 1 < KS) load_b(ks + 1, xb[(ks + 1) & 1]);
        else at_last();        // then what the caller issues last
#pragma unroll
        for (int k = 0; k < NB; ++k)
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                acc[mb][k] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[ks % (WD + 1)][mb], xb[ks & 1][k], acc[mb][k],
                                                                     0, 0, 0);
    }
    // epilogue: lane holds channels mb * 16 + 4 g .. + 3 of pixel pp[k]
    double dh = 0.0;
#pragma unroll
    for (int k = 0; k < NB; ++k) {
        if (pp[k] >= NPIX) continue;
        const int r = pp[k] / WOUT, c = pp[k] - (pp[k] / WOUT) * WOUT;
        const int gy = gy0 + r, gx = gx0 + c;
        if constexpr (MODE == 2) {
            if (g != 0 || gy >= H) continue;                    // lanes of group 0 hold channels 0..3
            f32x4 v = acc[0][k];
#pragma unroll
            for (int q = 0; q < 4; ++q) v[q] = q < COUT ? v[q] + bias[q] : 0.f;
            *reinterpret_cast<f32x4 *>(out + (out_row0 + (int64_t)r * W + c) * 4) = v;
            dh += (double)v[0];
        } else {
            const bool inside = gy >= 0 && gy < H && gx >= 0 && gx < W;
#pragma unroll
            for (int mb = 0; mb < MB; ++mb) {
                f32x4 v = acc[mb][k];
#pragma unroll
                for (int q = 0; q < 4; ++q) v[q] = fmaxf(v[q] + bias[mb * 16 + 4 * g + q], 0.f);
                if (MODE == 1) {
                    const bf16x4 xin = *reinterpret_cast<const bf16x4 *>(
                        src + chunk_off(sb[k] + WIN + 1, 2 * mb + (g >> 1)) + 4 * (g & 1));
#pragma unroll
                    for (int q = 0; q < 4; ++q) v[q] += (float)xin[q];
                }
                bf16x4 o = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                if (!inside) o = bf16x4{};
                *reinterpret_cast<bf16x4 *>(dst + chunk_off(pp[k], 2 * mb + (g >> 1)) + 4 * (g & 1)) = o;
            }
        }
    }
    return dh;
}

// NW waves per workgroup.
template <int TH, int TW, int NW>
__global__ __launch_bounds__(64 * NW) void k_net_fused(SwNetFusedArgs a, int tiles_y, int tiles_x, int ntiles) {
    using G = Geo<TH, TW>;
    __shared__ __attribute__((aligned(16))) __bf16 sa[G::A_ELEMS];
    __shared__ __attribute__((aligned(16))) __bf16 sxb[G::XB_ELEMS];
    __bf16 *const sx = sxb, *const sbf = sxb;   // input (layer 1 reads it), then layers 2 and 4
    __shared__ double s_dh[NW];
    __shared__ float s_bias[6][32];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < 6 * 32; i += 64 * NW) {   // the layers' biases (output layer: 3)
        const int l = i >> 5, co = i & 31;
        s_bias[l][co] = (l < 5 || co < 3) ? a.bias[l][co] : 0.f;
    }
    const int H = a.H, W = a.W;

    // the input of tile tt: raw state values of this thread's pixels of the
    // (TH + 12) x (TW + 12) region, loaded into registers ahead of use (the
    // ghost ring of the grid included; pixels further out are zero)
    constexpr int NPIN = G::h(0) * G::w(0);
    constexpr int PER = (NPIN + 64 * NW - 1) / (64 * NW);
    float rh[PER], rp[PER], rq[PER];
    unsigned ok = 0u;
    auto stage_load = [&](int tt) {
        const int b = tt / (tiles_y * tiles_x);
        const int rem = tt - b * tiles_y * tiles_x;
        const int ty = rem / tiles_x, tx = rem - ty * tiles_x;
        const SwBatchGrid &gd = a.grids[b];
        const float *P0 = (const float *)gd.plane[a.cur][0], *P1 = (const float *)gd.plane[a.cur][1],
                    *P2 = (const float *)gd.plane[a.cur][2];
        ok = 0u;
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * 64 * NW;
            const int r = i / G::w(0), c = i - r * G::w(0);
            const int gy = ty * TH - kBorder + r, gx = tx * TW - kBorder + c;
            rh[j] = rp[j] = rq[j] = 0.f;
            if (i < NPIN && gy >= -1 && gy <= H && gx >= -1 && gx <= W) {
                const int64_t off = (int64_t)gy * gd.pitch + gx;
                rh[j] = P0[off];
                rp[j] = P1[off];
                rq[j] = P2[off];
                ok |= 1u << j;
            }
        }
    };
    auto stage_store = [&] {
#pragma unroll
        for (int j = 0; j < PER; ++j) {
            const int i = threadIdx.x + j * 64 * NW;
            if (i >= NPIN) continue;
            bf16x8 v = bf16x8{};
            if (ok >> j & 1u)
                v = bf16x8{(__bf16)((rh[j] - a.nrm.in_off[0]) / a.nrm.in_scale[0]),
                           (__bf16)((rp[j] - a.nrm.in_off[1]) / a.nrm.in_scale[1]),
                           (__bf16)((rq[j] - a.nrm.in_off[2]) / a.nrm.in_scale[2]),
                           (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f, (__bf16)0.f};
            *reinterpret_cast<bf16x8 *>(sx + i * 8) = v;
        }
    };
    auto nothing = [] {};
    const int lane16 = lane & 15, g4 = lane >> 4;
    bf16x8 wcur[2];
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) wcur[mb] = load_wk<3>((const __bf16 *)a.wk[0], mb, 0, lane16, g4);
    if (blockIdx.x < ntiles) stage_load(blockIdx.x);

    for (int t = blockIdx.x; t < ntiles; t += gridDim.x) {   // uniform per block
        const int b = t / (tiles_y * tiles_x);
        const int rem = t - b * tiles_y * tiles_x;
        const int ty = rem / tiles_x, tx = rem - ty * tiles_x;
        const int y0 = ty * TH, x0 = tx * TW;               // tile origin in the grid
        if (a.clear_stats && ty == 0 && tx == 0 && threadIdx.x == 0) {   // the grid's first tile clears its statistics
            SwGateStats &st = a.clear_stats[b];
            st.mass_old = 0.0;
            st.mass_new = 0.0;
            st.hmin = 3.0e38f;
            st.nonfinite = 0u;
        }
        stage_store();
        __syncthreads();
        run_layer<8, 32, 0, G::w(1), G::h(1), NW, 2, 9>(sx, sa, a.wk[0], wcur, a.wk[1], s_bias[0], y0 - 5, x0 - 5, H,
                                                        W, nullptr, 0, nothing);
        __syncthreads();
        run_layer<32, 32, 1, G::w(2), G::h(2), NW, 2, 9>(sa, sbf, a.wk[1], wcur, a.wk[2], s_bias[1], y0 - 4, x0 - 4,
                                                         H, W, nullptr, 0, nothing);
        __syncthreads();
        run_layer<32, 32, 1, G::w(3), G::h(3), NW, 2, 9>(sbf, sa, a.wk[2], wcur, a.wk[3], s_bias[2], y0 - 3, x0 - 3,
                                                         H, W, nullptr, 0, nothing);
        __syncthreads();
        run_layer<32, 32, 1, G::w(4), G::h(4), NW, 2, 9>(sa, sbf, a.wk[3], wcur, a.wk[4], s_bias[3], y0 - 2, x0 - 2,
                                                         H, W, nullptr, 0, nothing);
        __syncthreads();
        run_layer<32, 32, 1, G::w(5), G::h(5), NW, 1, 9>(sbf, sa, a.wk[4], wcur, a.wk[5], s_bias[4], y0 - 1, x0 - 1,
                                                         H, W, nullptr, 0, nothing);
        __syncthreads();
        const int tn = t + gridDim.x;
        double dh = run_layer<32, 3, 2, TW, TH, NW, 2, 3>(sa, nullptr, a.wk[5], wcur, a.wk[0], s_bias[5], y0, x0, H, W,
                                                          a.delta, ((int64_t)b * H + y0) * W + x0, [&] {
                                                              if (tn < ntiles) stage_load(tn);
                                                          });
        // the tile's sum of predicted dh in a fixed order: lanes, then waves
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) dh += __shfl_xor(dh, o);
        if (lane == 0) s_dh[wave] = dh;
        __syncthreads();                                     // also: the next tile's staging may overwrite sx / sa
        if (threadIdx.x == 0 && a.dh_tile) {
            double s = 0.0;
            for (int k = 0; k < NW; ++k) s += s_dh[k];
            a.dh_tile[(int64_t)b * tiles_y * tiles_x + rem] = s;
        }
    }
}

#ifndef SW_NET_WAVES
#define SW_NET_WAVES 8
#endif
constexpr int kNetWaves = SW_NET_WAVES;

template <int TH, int TW>
hipError_t launch_net(const SwNetFusedArgs &a, hipStream_t s) {
    const int tiles_y = (a.H + TH - 1) / TH, tiles_x = a.W / TW;
    const int64_t ntiles = (int64_t)a.B * tiles_y * tiles_x;
    if (ntiles > (int64_t)1 << 30) return hipErrorInvalidValue;
    static const int resident = [] {   // workgroups that fit on one CU at once (LDS and registers)
        int r = 0;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(&r, k_net_fused<TH, TW, kNetWaves>, 64 * kNetWaves,
                                                            0) == hipSuccess &&
                       r > 0
                   ? r
                   : 1;
    }();
    int64_t blocks = std::min<int64_t>(ntiles, (int64_t)sw_device_cus() * resident);
    if (a.max_blocks > 0) blocks = std::min<int64_t>(blocks, a.max_blocks);
    k_net_fused<TH, TW, kNetWaves><<<(unsigned)blocks, 64 * kNetWaves, 0, s>>>(a, tiles_y, tiles_x, (int)ntiles);
    return hipGetLastError();
}

}  // namespace

// Tile shape: 16 x 32 when the batch has at least two such tiles per CU
// (less recomputed border), else 16 x 16 (more workgroups for small batches).
#ifndef SW_NET_WIDE
#define SW_NET_WIDE 1
#endif
void sw_net_fused_tile(int B, int H, int W, int *th, int *tw) {
    const int64_t wide = (int64_t)B * ((H + 15) / 16) * (W / 32);
    *th = 16;
    *tw = SW_NET_WIDE && wide >= 2 * (int64_t)sw_device_cus() ? 32 : 16;
}

hipError_t sw_net_fused(const SwNetFusedArgs &a, hipStream_t s) {
    if (a.B < 1 || a.H < 1 || a.W < 64 || a.W % 64 != 0 || !a.grids || a.cur < 0 || a.cur > 1 || !a.delta)
        return hipErrorInvalidValue;
    for (int l = 0; l < 6; ++l)
        if (!a.wk[l] || !a.bias[l]) return hipErrorInvalidValue;
    int th, tw;
    sw_net_fused_tile(a.B, a.H, a.W, &th, &tw);
    return tw == 32 ? launch_net<16, 32>(a, s) : launch_net<16, 16>(a, s);
}
