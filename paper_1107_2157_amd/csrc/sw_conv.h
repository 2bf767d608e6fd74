// Internal interface of the learned surrogate's kernels (host <-> device).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

#include "sw_batch_internal.h"

enum { SW_CONV_RELU_BF16 = 0, SW_CONV_RESID_BF16 = 1, SW_CONV_F32 = 2, SW_CONV_DGRAD = 3, SW_CONV_RELU_PLANES = 4 };

// Per-channel affine normalisation of the state: x = (u - offset) / scale.
struct SwNorm {
    float in_off[3], in_scale[3], out_scale[3];
};

// One 3x3 convolution launch (see sw_conv.hip for layouts).  Modes:
//   RELU:  y = relu(conv(x) + b)                                (first layer)
//   RESID: y = x + relu(conv(x) + b), y2 = relu(conv(x) + b)     (residual blocks)
//   F32:   yf = conv(x) + b in FP32                              (output layer)
//   DGRAD: G = conv(x) + add, y = G, y2 = G where mask > 0       (input gradient)
//   RELU_PLANES: RELU with the input read from the FP32 planes of a batch of
//          grids (buffer cur, ghosts materialised) and normalised on the fly
//          (the rollout's first layer); the tile at a grid's origin also
//          clears that grid's gate statistics (clear_stats).
// Every BF16 output may be null except y in RELU / RESID and y2 in DGRAD.
// F32 with dh_part set also writes, per grid and output row, the sum of the
// row's channel-0 outputs (FP64, fixed order) at dh_part[b * H + y].
struct SwConvArgs {
    const void *x;       // BF16 NHWC input with halo, CIN channels
    const void *w;       // BF16 [COUT padded to 16][K padded to 32] implicit-GEMM weights
    const float *bias;   // FP32 [COUT] (RELU, RESID and F32 modes)
    void *y;             // BF16 NHWC output with halo, COUT channels
    void *y2;            // BF16 NHWC output with halo, COUT channels (RESID: relu part, DGRAD: masked)
    float *yf;           // FP32 [B][H][W][4] output (F32 mode)
    const void *add;     // BF16 NHWC with halo, COUT channels, added before rounding (DGRAD)
    const void *mask;    // BF16 NHWC with halo, COUT channels: y2 kept where mask > 0 (DGRAD)
    int B, H, W;
    int max_blocks;      // cap on the persistent grid (0: one block per resident slot)
    const SwBatchGrid *grids;   // RELU_PLANES: the batch's grids (all H x W)
    int cur;                    // RELU_PLANES: buffer holding the state
    SwNorm nrm;                 // RELU_PLANES: input normalisation
    SwGateStats *clear_stats;   // RELU_PLANES: gate statistics to clear (may be null)
    double *dh_part;            // F32: per-row sums of channel 0 (may be null)
};
hipError_t sw_conv3x3(const SwConvArgs &a, int cin, int cout, int mode, hipStream_t s);

// The rollout's whole network in one launch (sw_netfused.hip): from the
// batch's FP32 planes (buffer cur, ghosts materialised) to the FP32
// prediction [B][H][W][4], bitwise the per-layer forward pass, plus each
// output tile's sum of the predicted dh (FP64, fixed order) at
// dh_tile[b * tiles_per_grid + tile] (tiles row-major; sw_net_fused_tile
// gives the tile shape).  W a multiple of 64.
struct SwNetFusedArgs {
    const SwBatchGrid *grids;
    int cur;
    int B, H, W;
    SwNorm nrm;
    const void *wk[6];          // forward weight layouts of the six layers
    const float *bias[6];       // FP32 biases
    float *delta;               // [B][H][W][4]
    double *dh_tile;            // may be null
    SwGateStats *clear_stats;   // the jump's gate statistics, cleared per grid (may be null)
    int max_blocks;             // cap on the persistent grid (0: one workgroup per CU)
};
hipError_t sw_net_fused(const SwNetFusedArgs &a, hipStream_t s);
void sw_net_fused_tile(int B, int H, int W, int *th, int *tw);
// Compute units of the current device (for persistent grids).
int sw_device_cus();

// Dense FP32 frames [B][3][H][W] -> network input X0 (BF16 NHWC, 8 channels,
// halo = reflective / periodic ghost values) and, if u8 != nullptr, the
// target (u8 - u) / out_scale as FP32 [B][H][W][4].
hipError_t sw_sur_prep_dense(const float *u, const float *u8, int B, int H, int W, int bc_x, int bc_y, SwNorm nrm,
                             void *x0, float *target, hipStream_t s);
// MSE loss over the three channels: per-block partial sums into partial[nblocks],
// and dZ = 2 (pred - target) / (3 B H W) as BF16 NHWC with halo, 8 channels.
hipError_t sw_sur_loss(const float *pred, const float *target, int B, int H, int W, float *partial, int nblocks,
                       void *dz, hipStream_t s);
hipError_t sw_sur_reduce_sum(const float *partial, int n, float *out, hipStream_t s);
// Weight gradient of one layer (MFMA, K = pixels) from the NHWC tensors with
// halo: dW[co][tap][ci] = sum_p dZ[p][co] A[p + tap][ci], db[co] = sum_p dZ[p][co],
// written into grad (logical layout, W then b).  dz has coutp (8 or 32)
// channels, a cinp (8 or 32); W a multiple of 64; partial holds
// nblocks * (cout * 9 * cin + cout) floats (at most nblocks blocks are used).
hipError_t sw_sur_wgrad(const void *dz, int coutp, int cout, const void *a, int cinp, int cin, int B, int H, int W,
                        float *partial, int nblocks, float *grad_w, float *grad_b, hipStream_t s);
// Adam on the FP32 master parameters and refresh of the BF16 forward /
// input-gradient weight layouts.
struct SwLayerDesc {
    int cin, cinp, cout, coutp;   // real and padded channel counts
    int64_t w_off, b_off;         // offsets in the master vector
    void *wk;                     // BF16 [coutp16][kp] forward layout
    void *wd;                     // BF16 [cin padded to 32][kp'] input-gradient layout (nullptr for layer 1)
    int kp, kpd, cdp;             // forward K (padded), input-gradient K (padded), dgrad input channels (8 or 32)
};
struct SwAdam {
    float lr, beta1, beta2, eps;
    float c1, c2;                 // 1 / (1 - beta^t) bias corrections
};
hipError_t sw_sur_adam(float *master, float *m, float *v, const float *grad, int64_t n, SwAdam ad, hipStream_t s);
hipError_t sw_sur_relayout(const float *master, const SwLayerDesc *layers, int nlayers, int64_t total_weights,
                           hipStream_t s);

// Rollout: per grid, sum of predicted dh (for the mass projection), the
// update U' = U + denorm(delta) (- mean dh if projecting) written into the
// other buffer, and the gate's mass / min-h / finiteness statistics
// (SwGateStats, sw_batch_internal.h).
// dh_part: partial sums of the normalised dh, nparts per grid ([B][nparts]:
// the per-layer output layer's per-row-segment sums, or the fused network's
// per-tile sums), summed per grid in a fixed order for the mass projection.
// part / ticket: scratch of the statistics' reduction, sw_sur_apply_slots
// entries and one ticket per grid (zero before the first call; every call
// leaves the tickets at zero).
struct SwApplyPart {
    unsigned long long mo, mn;       // FP64 bits: the block's sums of h before and after
    unsigned long long hmin_bad;     // FP32 bits of the block's least h (high word), non-finite flag (low)
    unsigned long long pad;
};
unsigned sw_sur_apply_slots(int64_t pixels, int B);
hipError_t sw_sur_apply(const float *delta, const double *dh_part, int nparts, const SwBatchGrid *grids, int cur,
                        int B, int H, int W, SwNorm nrm, int project, int bcx, int bcy, SwGateStats *st,
                        SwApplyPart *part, unsigned *ticket, hipStream_t s);
// The gate's verdict per grid (active[b] = 1 and fallbacks[b] += 1 for a
// rejected jump); rejected grids get U^n (buffer cur, halos included) copied
// over the prediction in buffer cur ^ 1, where the solver then takes the jump.
hipError_t sw_sur_gate_restore(const SwBatchGrid *grids, int cur, int B, int H, int W, SwGateStats *st,
                               double mass_tol, double hmin, int *active, int *fallbacks, hipStream_t s);

// Judge: per grid, relative L2(h) of the rollout (batch grids `a`, current
// buffer cur_a) against the plain solver's run (`ref`, buffer cur_ref); grids
// above l2_tol take the solver's state (halos included), their fallback count
// becomes jumps, their time / step counters become start + the solver's, and
// their unstable flag the solver's.
struct SwJudge {
    double d2, r2;     // sum (h - h_ref)^2, sum h_ref^2
    double t0;         // time at the start of the advance
    long long steps0;  // step count at the start of the advance
};
hipError_t sw_sur_judge_begin(const SwBatchScalars *sc, int B, SwJudge *j, hipStream_t s);
hipError_t sw_sur_judge(const SwBatchGrid *a, int cur_a, const SwBatchGrid *ref, int cur_ref, int B, int H, int W,
                        SwJudge *j, SwBatchScalars *sc, const SwBatchScalars *ref_sc, double l2_tol, int jumps,
                        int *reject, int *fallbacks, double *l2, hipStream_t s);
