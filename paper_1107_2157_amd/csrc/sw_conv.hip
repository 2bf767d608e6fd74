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

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int CIN> constexpr int ksteps() { return CIN == 32 ? 9 : 3; }

// One wave: NPB blocks of 16 pixels of one image row, all COUT channels.
template <int CIN, int COUT, int MODE, int NPB>
__global__ __launch_bounds__(256) void k_conv3x3(SwConvArgs a) {
    constexpr int MB = (COUT + 15) / 16;
    constexpr int KS = ksteps<CIN>();
    constexpr int KP = KS * 32;
    const int lane = threadIdx.x & 63;
    const int wave = (int)(blockIdx.x * 4 + (threadIdx.x >> 6));
    const int segs = a.W / (16 * NPB);
    const int total = a.B * a.H * segs;
    if (wave >= total) return;
    const int b = wave / (a.H * segs);
    const int rem = wave - b * a.H * segs;
    const int y = rem / segs;
    const int x0 = (rem - y * segs) * 16 * NPB;
    const int Wp = a.W + 2;
    const __bf16 *X = (const __bf16 *)a.x + ((int64_t)b * (a.H + 2) * Wp) * CIN;
    const __bf16 *Wk = (const __bf16 *)a.w;
    const int g = lane >> 4, n = lane & 15;

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
        const int dy = live ? tap / 3 : 1, dx = live ? tap % 3 : 1;   // offsets into the halo'd image
        bf16x8 wa[MB];
#pragma unroll
        for (int mb = 0; mb < MB; ++mb)
            wa[mb] = *reinterpret_cast<const bf16x8 *>(Wk + (int64_t)(mb * 16 + n) * KP + ks * 32 + 8 * g);
#pragma unroll
        for (int pb = 0; pb < NPB; ++pb) {
            const int px = x0 + pb * 16 + n;
            bf16x8 xb = *reinterpret_cast<const bf16x8 *>(X + ((int64_t)(y + dy) * Wp + px + dx) * CIN + ci0);
            if (!live) xb = bf16x8{};
#pragma unroll
            for (int mb = 0; mb < MB; ++mb)
                acc[mb][pb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wa[mb], xb, acc[mb][pb], 0, 0, 0);
        }
    }

    // epilogue: lane holds channels co = mb*16 + 4g .. +3 of pixel x0 + pb*16 + n
    const int Wq = sw_planar_pitch(a.W);
#pragma unroll
    for (int mb = 0; mb < MB; ++mb) {
        const int co0 = mb * 16 + 4 * g;
        if (co0 >= COUT && MODE != SW_CONV_F32) continue;
#pragma unroll
        for (int pb = 0; pb < NPB; ++pb) {
            const int px = x0 + pb * 16 + n;
            f32x4 v = acc[mb][pb];
            if (MODE == SW_CONV_F32) {   // channels 0..3 (COUT <= 4) with bias, FP32, no halo
                if (g != 0) continue;
                float *Y = a.yf + (((int64_t)b * a.H + y) * a.W + px) * 4;
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = r < COUT ? v[r] + a.bias[r] : 0.f;
                *reinterpret_cast<f32x4 *>(Y) = v;
                continue;
            }
            const int64_t at = (((int64_t)b * (a.H + 2) + y + 1) * Wp + px + 1) * COUT + co0;   // NHWC, halo'd
            bf16x4 o, o2;
            if (MODE == SW_CONV_RELU_BF16 || MODE == SW_CONV_RESID_BF16) {
#pragma unroll
                for (int r = 0; r < 4; ++r) v[r] = fmaxf(v[r] + a.bias[co0 + r], 0.f);
                if (MODE == SW_CONV_RESID_BF16) {   // CIN == COUT: the block's input at this pixel
                    const bf16x4 xin = *reinterpret_cast<const bf16x4 *>((const __bf16 *)a.x + at);
                    o2 = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] += (float)xin[r];
                    if (a.y2) *reinterpret_cast<bf16x4 *>((__bf16 *)a.y2 + at) = o2;
                }
                o = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                *reinterpret_cast<bf16x4 *>((__bf16 *)a.y + at) = o;
            } else {   // SW_CONV_DGRAD
                if (a.add) {
                    const bf16x4 ad = *reinterpret_cast<const bf16x4 *>((const __bf16 *)a.add + at);
#pragma unroll
                    for (int r = 0; r < 4; ++r) v[r] += (float)ad[r];
                }
                o2 = bf16x4{(__bf16)v[0], (__bf16)v[1], (__bf16)v[2], (__bf16)v[3]};
                if (a.y) *reinterpret_cast<bf16x4 *>((__bf16 *)a.y + at) = o2;
                const bf16x4 mk = *reinterpret_cast<const bf16x4 *>((const __bf16 *)a.mask + at);
#pragma unroll
                for (int r = 0; r < 4; ++r) o[r] = (float)mk[r] > 0.f ? o2[r] : (__bf16)0.f;
                *reinterpret_cast<bf16x4 *>((__bf16 *)a.y2 + at) = o;
            }
            if (a.yp) {   // planar copy: 16 lanes of a channel write 16 consecutive pixels
                __bf16 *P = (__bf16 *)a.yp + (((int64_t)b * (a.H + 2) + y + 1) * COUT + co0) * Wq + px + 8;
#pragma unroll
                for (int r = 0; r < 4; ++r) P[(int64_t)r * Wq] = o[r];
            }
        }
    }
}

template <int CIN, int COUT, int MODE>
hipError_t launch(const SwConvArgs &a, hipStream_t s) {
    constexpr int NPB = 4;
    if (a.W % (16 * NPB) != 0) return hipErrorInvalidValue;
    const int64_t waves = (int64_t)a.B * a.H * (a.W / (16 * NPB));
    k_conv3x3<CIN, COUT, MODE, NPB><<<(unsigned)((waves + 3) / 4), 256, 0, s>>>(a);
    return hipGetLastError();
}

}  // namespace

hipError_t sw_conv3x3(const SwConvArgs &a, int cin, int cout, int mode, hipStream_t s) {
    if (a.B < 1 || a.H < 1 || a.W < 1 || !a.x || !a.w) return hipErrorInvalidValue;
    if (mode == SW_CONV_F32 ? !a.yf || !a.bias : mode == SW_CONV_DGRAD ? !a.y2 || !a.mask : !a.y || !a.bias)
        return hipErrorInvalidValue;
    if (cin == 8 && cout == 32 && mode == SW_CONV_RELU_BF16) return launch<8, 32, SW_CONV_RELU_BF16>(a, s);
    if (cin == 32 && cout == 32 && mode == SW_CONV_RESID_BF16) return launch<32, 32, SW_CONV_RESID_BF16>(a, s);
    if (cin == 32 && cout == 3 && mode == SW_CONV_F32) return launch<32, 3, SW_CONV_F32>(a, s);
    if (cin == 32 && cout == 32 && mode == SW_CONV_DGRAD) return launch<32, 32, SW_CONV_DGRAD>(a, s);
    if (cin == 8 && cout == 32 && mode == SW_CONV_DGRAD) return launch<8, 32, SW_CONV_DGRAD>(a, s);
    return hipErrorInvalidValue;
}
