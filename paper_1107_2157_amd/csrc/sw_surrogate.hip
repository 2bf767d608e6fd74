// Learned-surrogate kernels other than the convolution: input preparation,
// loss and its gradient seed, weight gradients, Adam with the BF16 weight
// re-layout, and the gated rollout (apply, gate statistics, accept).
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
        store_x0(x0 + idx * 8, (h - nrm.in_off[0]) / nrm.in_scale[0], (hu - nrm.in_off[1]) / nrm.in_scale[1],
                 (hv - nrm.in_off[2]) / nrm.in_scale[2]);
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

__global__ __launch_bounds__(256) void k_prep_planes(const SwBatchGrid *grids, int cur, int B, int H, int W, SwNorm nrm,
                                                     __bf16 *x0) {
    const int Wp = W + 2, Hp = H + 2;
    const int64_t n = (int64_t)B * Hp * Wp;
    for (int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; idx < n; idx += (int64_t)gridDim.x * blockDim.x) {
        const int b = (int)(idx / ((int64_t)Hp * Wp));
        const int r = (int)(idx - (int64_t)b * Hp * Wp);
        const int yy = r / Wp, xx = r - yy * Wp;
        const SwBatchGrid &g = grids[b];
        const int64_t off = (int64_t)(yy - 1) * g.pitch + (xx - 1);   // halo cells are materialised
        const float h = ((const float *)g.plane[cur][0])[off];
        const float hu = ((const float *)g.plane[cur][1])[off];
        const float hv = ((const float *)g.plane[cur][2])[off];
        store_x0(x0 + idx * 8, (h - nrm.in_off[0]) / nrm.in_scale[0], (hu - nrm.in_off[1]) / nrm.in_scale[1],
                 (hv - nrm.in_off[2]) / nrm.in_scale[2]);
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
        store_x0(dz + (((int64_t)b * (H + 2) + y + 1) * (W + 2) + x + 1) * 8, scale * d0, scale * d1, scale * d2);
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

// Weight gradient partials: each block walks 64-pixel row segments; LDS holds
// the segment's dZ (64 x COUTP) and the three input rows it needs
// (3 x 66 x CINP).  Thread (co, ci group of 4) accumulates all 9 taps.
template <int CINP, int COUTP>
__global__ __launch_bounds__(256) void k_wgrad(const __bf16 *dz, const __bf16 *a, int cout, int cin, int B, int H,
                                               int W, float *partial, int nent) {
    __shared__ __bf16 sdz[64 * COUTP];
    __shared__ __bf16 sa[3 * 66 * CINP];
    constexpr int CG = CINP / 4;
    const int t = threadIdx.x;
    const int co = t / CG, cg = t % CG;
    float acc[9][4];
#pragma unroll
    for (int k = 0; k < 9; ++k)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[k][r] = 0.f;
    float bacc = 0.f;
    const int segs = W / 64;
    const int64_t nseg = (int64_t)B * H * segs;
    const int Wp = W + 2;
    for (int64_t seg = blockIdx.x; seg < nseg; seg += gridDim.x) {
        const int b = (int)(seg / ((int64_t)H * segs));
        const int rem = (int)(seg - (int64_t)b * H * segs);
        const int y = rem / segs, x0 = (rem - y * segs) * 64;
        __syncthreads();
        for (int i = t; i < 64 * COUTP / 8; i += 256) {
            const int px = i / (COUTP / 8), part = i % (COUTP / 8);
            *reinterpret_cast<bf16x8 *>(&sdz[px * COUTP + part * 8]) = *reinterpret_cast<const bf16x8 *>(
                dz + (((int64_t)b * (H + 2) + y + 1) * Wp + x0 + 1 + px) * COUTP + part * 8);
        }
        for (int i = t; i < 3 * 66 * CINP / 8; i += 256) {
            const int rr = i / (66 * CINP / 8), rem2 = i % (66 * CINP / 8);
            const int px = rem2 / (CINP / 8), part = rem2 % (CINP / 8);
            *reinterpret_cast<bf16x8 *>(&sa[(rr * 66 + px) * CINP + part * 8]) = *reinterpret_cast<const bf16x8 *>(
                a + (((int64_t)b * (H + 2) + y + rr) * Wp + x0 + px) * CINP + part * 8);
        }
        __syncthreads();
        if (co < cout) {
            for (int p = 0; p < 64; ++p) {
                const float d = (float)sdz[p * COUTP + co];
                bacc += d;
#pragma unroll
                for (int tap = 0; tap < 9; ++tap) {
                    const bf16x4 av = *reinterpret_cast<const bf16x4 *>(&sa[((tap / 3) * 66 + p + tap % 3) * CINP + 4 * cg]);
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc[tap][r] = fmaf(d, (float)av[r], acc[tap][r]);
                }
            }
        }
    }
    float *P = partial + (int64_t)blockIdx.x * nent;
    if (co < cout) {
#pragma unroll
        for (int tap = 0; tap < 9; ++tap)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int ci = 4 * cg + r;
                if (ci < cin) P[(co * 9 + tap) * cin + ci] = acc[tap][r];
            }
        if (cg == 0) P[cout * 9 * cin + co] = bacc;
    }
}

__global__ void k_wgrad_reduce(const float *partial, int nblocks, int nent, int nw, float *grad_w, float *grad_b) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nent) return;
    double acc = 0.0;
    for (int k = 0; k < nblocks; ++k) acc += partial[(int64_t)k * nent + e];
    if (e < nw) grad_w[e] = (float)acc;
    else grad_b[e - nw] = (float)acc;
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

__global__ void k_zero_stats(SwGateStats *st, int B) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    st[b].mass_old = 0.0;
    st[b].mass_new = 0.0;
    st[b].dh_sum = 0.0;
    st[b].hmin = 3.0e38f;
    st[b].nonfinite = 0u;
}

// Per grid (blockIdx.y): sum of the normalised dh over its pixels.
__global__ __launch_bounds__(256) void k_delta_sum(const float *delta, int H, int W, SwGateStats *st) {
    const int b = blockIdx.y;
    const int64_t n = (int64_t)H * W;
    double acc = 0.0;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x)
        acc += delta[((int64_t)b * n + p) * 4];
    acc = wave_sum_d(acc);
    if ((threadIdx.x & 63) == 0) atomicAdd(&st[b].dh_sum, acc);
}

__global__ __launch_bounds__(256) void k_apply(const float *delta, const SwBatchGrid *grids, int cur, int H, int W,
                                               SwNorm nrm, int project, int bcx, int bcy, SwGateStats *st) {
    const int b = blockIdx.y;
    const SwBatchGrid &g = grids[b];
    const int64_t n = (int64_t)H * W;
    const float dh_mean = project ? (float)(st[b].dh_sum / (double)n) : 0.f;
    const float *U[3] = {(const float *)g.plane[cur][0], (const float *)g.plane[cur][1], (const float *)g.plane[cur][2]};
    float *O[3] = {(float *)g.plane[cur ^ 1][0], (float *)g.plane[cur ^ 1][1], (float *)g.plane[cur ^ 1][2]};
    double mo = 0.0, mn = 0.0;
    float hmin = 3.0e38f;
    bool bad = false;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int y = (int)(p / W), x = (int)(p - (int64_t)y * W);
        const int64_t off = (int64_t)y * g.pitch + x;
        const float4 d = *reinterpret_cast<const float4 *>(delta + ((int64_t)b * n + p) * 4);
        const float h = U[0][off], hu = U[1][off], hv = U[2][off];
        U3<float> c = {h + (d.x - dh_mean) * nrm.out_scale[0], hu + d.y * nrm.out_scale[1], hv + d.z * nrm.out_scale[2]};
        O[0][off] = c.h;
        O[1][off] = c.p;
        O[2][off] = c.q;
        if (x == 0 || x == W - 1 || y == 0 || y == H - 1) write_ghosts(O, g.pitch, W, H, bcx, bcy, x, y, c);
        mo += h;
        mn += c.h;
        hmin = fminf(hmin, c.h);
        bad |= !(fabsf(c.h) <= 3.0e38f) || !(fabsf(c.p) <= 3.0e38f) || !(fabsf(c.q) <= 3.0e38f);
    }
    mo = wave_sum_d(mo);
    mn = wave_sum_d(mn);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) hmin = fminf(hmin, __shfl_xor(hmin, o));
    const unsigned long long anybad = __ballot(bad);
    if ((threadIdx.x & 63) == 0) {
        atomicAdd(&st[b].mass_old, mo);
        atomicAdd(&st[b].mass_new, mn);
        // min over non-negative values by integer order; a non-positive depth is recorded as 0
        atomicMin(reinterpret_cast<int *>(&st[b].hmin), __float_as_int(hmin > 0.f ? hmin : 0.f));
        if (anybad) atomicOr(&st[b].nonfinite, 1u);
    }
}

__global__ void k_gate(SwGateStats *st, int B, double mass_tol, double hmin, int *active, int *fallbacks) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B) return;
    const SwGateStats s = st[b];
    const double drift = fabs(s.mass_new - s.mass_old) / fabs(s.mass_old);
    const int reject = !(drift <= mass_tol) || !((double)s.hmin > hmin) || s.nonfinite != 0u;
    st[b].fallback = reject;
    active[b] = reject;
    if (fallbacks) fallbacks[b] += reject;
}

// Accepted grids: copy the whole halo'd rectangle of buffer cur ^ 1 into cur.
__global__ __launch_bounds__(256) void k_accept(const SwBatchGrid *grids, int cur, int H, int W, const int *active) {
    const int b = blockIdx.y;
    if (active[b]) return;
    const SwBatchGrid &g = grids[b];
    const int64_t n = (int64_t)(H + 2) * (W + 2);
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n; p += (int64_t)gridDim.x * blockDim.x) {
        const int yy = (int)(p / (W + 2)), xx = (int)(p - (int64_t)yy * (W + 2));
        const int64_t off = (int64_t)(yy - 1) * g.pitch + (xx - 1);
#pragma unroll
        for (int k = 0; k < 3; ++k) ((float *)g.plane[cur][k])[off] = ((const float *)g.plane[cur ^ 1][k])[off];
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

hipError_t sw_sur_prep_planes(const SwBatchGrid *grids, int cur, int B, int H, int W, SwNorm nrm, void *x0,
                              hipStream_t s) {
    k_prep_planes<<<grid_for((int64_t)B * (H + 2) * (W + 2)), 256, 0, s>>>(grids, cur, B, H, W, nrm, (__bf16 *)x0);
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

hipError_t sw_sur_wgrad(const void *dz, int coutp, int cout, const void *a, int cinp, int cin, int B, int H, int W,
                        float *partial, int nblocks, float *grad_w, float *grad_b, hipStream_t s) {
    if (W % 64 != 0) return hipErrorInvalidValue;
    const int nent = cout * 9 * cin + cout;
    if (cinp == 32 && coutp == 32)
        k_wgrad<32, 32><<<nblocks, 256, 0, s>>>((const __bf16 *)dz, (const __bf16 *)a, cout, cin, B, H, W, partial, nent);
    else if (cinp == 8 && coutp == 32)
        k_wgrad<8, 32><<<nblocks, 256, 0, s>>>((const __bf16 *)dz, (const __bf16 *)a, cout, cin, B, H, W, partial, nent);
    else if (cinp == 32 && coutp == 8)
        k_wgrad<32, 8><<<nblocks, 256, 0, s>>>((const __bf16 *)dz, (const __bf16 *)a, cout, cin, B, H, W, partial, nent);
    else
        return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_wgrad_reduce<<<(nent + 255) / 256, 256, 0, s>>>(partial, nblocks, nent, cout * 9 * cin, grad_w, grad_b);
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

hipError_t sw_sur_zero_stats(SwGateStats *st, int B, hipStream_t s) {
    k_zero_stats<<<(B + 255) / 256, 256, 0, s>>>(st, B);
    return hipGetLastError();
}

hipError_t sw_sur_delta_sum(const float *delta, int B, int H, int W, SwGateStats *st, hipStream_t s) {
    dim3 grid(grid_for((int64_t)H * W, 64), B);
    k_delta_sum<<<grid, 256, 0, s>>>(delta, H, W, st);
    return hipGetLastError();
}

hipError_t sw_sur_apply(const float *delta, const SwBatchGrid *grids, int cur, int B, int H, int W, SwNorm nrm,
                        int project, int bcx, int bcy, SwGateStats *st, hipStream_t s) {
    dim3 grid(grid_for((int64_t)H * W, 64), B);
    k_apply<<<grid, 256, 0, s>>>(delta, grids, cur, H, W, nrm, project, bcx, bcy, st);
    return hipGetLastError();
}

hipError_t sw_sur_gate(SwGateStats *st, int B, double mass_tol, double hmin, int *active, int *fallbacks,
                       hipStream_t s) {
    k_gate<<<(B + 255) / 256, 256, 0, s>>>(st, B, mass_tol, hmin, active, fallbacks);
    return hipGetLastError();
}

hipError_t sw_sur_accept(const SwBatchGrid *grids, int cur, int B, int H, int W, const int *active, hipStream_t s) {
    dim3 grid(grid_for((int64_t)(H + 2) * (W + 2), 64), B);
    k_accept<<<grid, 256, 0, s>>>(grids, cur, H, W, active);
    return hipGetLastError();
}
