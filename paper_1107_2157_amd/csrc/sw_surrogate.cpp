// Learned surrogate, host side: a 6-layer 3x3 convolutional residual network
// (3 -> 32 -> 32 -> 32 -> 32 -> 32 -> 3: A1 = relu(Z1), four residual blocks
// A_l = A_{l-1} + relu(Z_l), delta = Z6; BF16 weights and activations, FP32
// accumulation) whose output is the normalised increment U^{n+8} - U^n,
// trained by the library's own forward / backward kernels, and its gated
// rollout on a batch of grids with the plain solver as fallback.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <random>
#include <vector>

#include "../../include/sw.h"
#include "sw_conv.h"

sw_status sw_fail(sw_status s, const char *fmt, ...);

#define SHIP(call)                                                                                  \
    do {                                                                                            \
        hipError_t e_ = (call);                                                                     \
        if (e_ != hipSuccess) return sw_fail(SW_EHIP, "%s: %s", #call, hipGetErrorString(e_));      \
    } while (0)

namespace {
constexpr int kLayers = 6;
constexpr int kHidden = 32;
constexpr int kLossBlocks = 1024;
constexpr int kWgradBlocks = 1024;
}  // namespace

struct sw_net {
    sw_net_cfg cfg{};
    int H = 0, W = 0, maxB = 0, device = 0;
    int64_t nparams = 0, nweights = 0;
    float *master = nullptr, *m = nullptr, *v = nullptr, *grad = nullptr;
    float *loss_partial = nullptr, *scratch_loss = nullptr;
    float *wpartial = nullptr;
    SwLayerDesc L[kLayers]{};
    SwLayerDesc *L_dev = nullptr;
    // NHWC BF16 tensors with halo; relu[k] = relu(Z) of residual block k + 1 (its mask)
    void *x0 = nullptr, *act[kLayers - 1] = {}, *relu[kLayers - 2] = {}, *g[2] = {}, *dz[2] = {}, *dz6 = nullptr;
    float *delta = nullptr, *target = nullptr;
    double *dh_part = nullptr;   // rollout: the output layer's per-row sums of dh ([B][H][W / 64])
    double *dh_tile = nullptr;   // fused rollout: per-tile sums of dh ([B][tiles per grid])
    // rollout network: 0 per-layer kernels, 1 one fused launch, 2 (default) the
    // form the batch size favours (rollout_fused)
    int fused_mode = 2;
    SwGateStats *stats = nullptr;
    SwApplyPart *apply_part = nullptr;   // the update's per-block statistics ([B][blocks per grid])
    unsigned *apply_ticket = nullptr;    // per grid, blocks of the update done (zero between launches)
    int32_t *active = nullptr;
    // judge mode: a clone of the advanced batch that runs the plain solver
    sw_batch *shadow = nullptr;
    void *shadow_arena = nullptr;
    SwJudge *judge = nullptr;
    int32_t *reject = nullptr;
    SwNorm nrm{};
    int block_cap = 0;   // cap on the persistent conv / weight-gradient grids (0: resident slots)
    int64_t adam_t = 0;
    std::vector<void *> allocs;
    // unjudged rollouts replay one hipGraph per (batch and its generation,
    // start buffer, nsteps, gate, fallbacks array), captured on the first call
    bool use_graph = true;
    hipStream_t cap = nullptr;
    struct Graph {
        const sw_batch *solver;
        uint64_t gen;
        int cur, nsteps;
        sw_gate gate;
        const int32_t *fallbacks;
        hipGraphExec_t exec;
    };
    std::vector<Graph> graphs;
};

namespace {

sw_status dalloc(sw_net *n, void **p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return sw_fail(e == hipErrorOutOfMemory ? SW_ENOMEM : SW_EHIP, "surrogate: %s", hipGetErrorString(e));
    n->allocs.push_back(*p);
    e = hipMemset(*p, 0, bytes);
    if (e != hipSuccess) return sw_fail(SW_EHIP, "surrogate: %s", hipGetErrorString(e));
    return SW_OK;
}

size_t act_bytes(const sw_net *n, int B, int ch) { return (size_t)B * (n->H + 2) * (n->W + 2) * ch * 2; }

void drop_graphs(sw_net *n) {
    for (auto &g : n->graphs) (void)hipGraphExecDestroy(g.exec);
    n->graphs.clear();
}

sw_status use_dev(const sw_net *n) {
    int d = -1;
    SHIP(hipGetDevice(&d));
    if (d != n->device) SHIP(hipSetDevice(n->device));
    return SW_OK;
}

bool residual(int l) { return l >= 1 && l <= kLayers - 2; }

SwConvArgs conv_args(const sw_net *n, int B, const void *x) {
    SwConvArgs a{};
    a.x = x;
    a.B = B;
    a.H = n->H;
    a.W = n->W;
    a.max_blocks = n->block_cap;
    return a;
}

// X0 -> act[0..4] -> delta; with train, also the ReLU parts (backward masks).
// With `planes` (a rollout) the first layer reads the batch's buffer directly
// (normalising it and clearing the jump's gate statistics) instead of X0, and
// the output layer also writes the per-row sums of dh when `dh_part` is set.
struct RolloutInput {
    const SwBatchGrid *grids;
    int cur;
    bool dh_sums;
};
sw_status forward(const sw_net *n, int B, bool train, hipStream_t s, const RolloutInput *planes = nullptr) {
    for (int l = 0; l < kLayers; ++l) {
        const SwLayerDesc &L = n->L[l];
        SwConvArgs a = conv_args(n, B, l == 0 ? n->x0 : n->act[l - 1]);
        a.w = L.wk;
        a.bias = n->master + L.b_off;
        int mode = SW_CONV_RELU_BF16;
        if (l == 0 && planes) {
            mode = SW_CONV_RELU_PLANES;
            a.x = nullptr;
            a.grids = planes->grids;
            a.cur = planes->cur;
            a.nrm = n->nrm;
            a.clear_stats = n->stats;
        }
        if (l == kLayers - 1) {
            a.yf = n->delta;
            if (planes && planes->dh_sums) a.dh_part = n->dh_part;
            mode = SW_CONV_F32;
        } else {
            a.y = n->act[l];
            if (residual(l)) {
                mode = SW_CONV_RESID_BF16;
                if (train) a.y2 = n->relu[l - 1];
            }
        }
        SHIP(sw_conv3x3(a, L.cinp, L.cout, mode, s));
    }
    return SW_OK;
}

// loss and gradients into n->grad (target and the training forward done):
// dZ of layer l gives dW_l, db_l, and G = dL/d(input of l) = conv^T(dZ) (+ G
// of l's output where l is residual), then dZ_{l-1} = G * (Z_{l-1} > 0)
sw_status backward(sw_net *n, int B, float *loss_out, hipStream_t s) {
    SHIP(sw_sur_loss(n->delta, n->target, B, n->H, n->W, n->loss_partial, kLossBlocks, n->dz6, s));
    if (loss_out) SHIP(sw_sur_reduce_sum(n->loss_partial, kLossBlocks, loss_out, s));
    const void *dz = n->dz6, *gout = nullptr;
    int dzc = 8;
    for (int l = kLayers - 1; l >= 0; --l) {
        const SwLayerDesc &L = n->L[l];
        SHIP(sw_sur_wgrad(dz, dzc, L.cout, l == 0 ? n->x0 : n->act[l - 1], L.cinp, L.cin, B, n->H, n->W,
                          n->wpartial, n->block_cap > 0 ? n->block_cap : kWgradBlocks, n->grad + L.w_off,
                          n->grad + L.b_off, s));
        if (l == 0) break;
        SwConvArgs a = conv_args(n, B, dz);
        a.w = L.wd;
        a.add = residual(l) ? gout : nullptr;
        a.mask = l == 1 ? n->act[0] : n->relu[l - 2];
        a.y = residual(l - 1) ? n->g[l & 1] : nullptr;
        a.y2 = n->dz[l & 1];
        SHIP(sw_conv3x3(a, L.cdp, L.cin, SW_CONV_DGRAD, s));
        gout = a.y;
        dz = a.y2;
        dzc = 32;
    }
    return SW_OK;
}

sw_status relayout(sw_net *n, hipStream_t s) {
    SHIP(sw_sur_relayout(n->master, n->L_dev, kLayers, n->nweights, s));
    return SW_OK;
}

void drop_shadow(sw_net *n) {
    if (n->shadow) sw_batch_destroy(n->shadow);
    if (n->shadow_arena) (void)hipFree(n->shadow_arena);
    n->shadow = nullptr;
    n->shadow_arena = nullptr;
}

sw_status check_net(const sw_net *n, int B) {
    if (!n) return sw_fail(SW_EINVAL, "surrogate: NULL network");
    if (B < 1 || B > n->maxB) return sw_fail(SW_EINVAL, "surrogate: batch %d outside [1, %d]", B, n->maxB);
    return use_dev(n);
}

}  // namespace

extern "C" {

sw_status sw_surrogate_create(const sw_net_cfg *cfg, int32_t H, int32_t W, int32_t max_batch, sw_net **out) {
    if (!out || !cfg) return sw_fail(SW_EINVAL, "surrogate_create: NULL argument");
    *out = nullptr;
    if (cfg->layers != kLayers || cfg->hidden != kHidden)
        return sw_fail(SW_ENOTSUP, "surrogate_create: only %d layers x %d channels", kLayers, kHidden);
    if (cfg->jump < 2 || (cfg->jump & 1)) return sw_fail(SW_EINVAL, "surrogate_create: jump %d must be even", cfg->jump);
    if ((cfg->bc_x != SW_BC_REFLECT && cfg->bc_x != SW_BC_PERIODIC) ||
        (cfg->bc_y != SW_BC_REFLECT && cfg->bc_y != SW_BC_PERIODIC))
        return sw_fail(SW_EINVAL, "surrogate_create: unknown boundary condition");
    if (H < 1 || W < 64 || W % 64 != 0 || max_batch < 1 || (int64_t)H * W * max_batch > (int64_t)1 << 31)
        return sw_fail(SW_EINVAL, "surrogate_create: grid %d x %d (W a multiple of 64), batch %d", H, W, max_batch);
    auto *n = new (std::nothrow) sw_net();
    if (!n) return sw_fail(SW_ENOMEM, "surrogate_create: host allocation");
    n->cfg = *cfg;
    n->H = H;
    n->W = W;
    n->maxB = max_batch;
    sw_status st = hipGetDevice(&n->device) == hipSuccess ? SW_OK : sw_fail(SW_EHIP, "surrogate_create: no device");
    // layer table: logical master layout W[co][tap][ci] then b[co], layer after layer
    const int cins[kLayers] = {3, 32, 32, 32, 32, 32}, couts[kLayers] = {32, 32, 32, 32, 32, 3};
    int64_t off = 0, nw = 0;
    for (int l = 0; l < kLayers && st == SW_OK; ++l) {
        SwLayerDesc &L = n->L[l];
        L.cin = cins[l];
        L.cout = couts[l];
        L.cinp = L.cin <= 8 ? 8 : 32;
        L.coutp = L.cout <= 8 ? 8 : 32;
        L.kp = (L.cinp == 32 ? 9 : 3) * 32;
        L.cdp = L.coutp;
        L.kpd = (L.cdp == 32 ? 9 : 3) * 32;
        L.w_off = off;
        off += (int64_t)L.cout * 9 * L.cin;
        nw += (int64_t)L.cout * 9 * L.cin;
        L.b_off = off;
        off += L.cout;
        const int rows = (L.cout + 15) / 16 * 16;
        st = dalloc(n, &L.wk, (size_t)rows * L.kp * 2);
        if (st == SW_OK && l > 0) st = dalloc(n, &L.wd, (size_t)32 * L.kpd * 2);
    }
    n->nparams = off;
    n->nweights = nw;
    if (st == SW_OK) st = dalloc(n, (void **)&n->master, off * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->m, off * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->v, off * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->grad, off * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->loss_partial, kLossBlocks * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->scratch_loss, 64);
    if (st == SW_OK) st = dalloc(n, (void **)&n->wpartial, (size_t)kWgradBlocks * (32 * 9 * 32 + 32) * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->L_dev, sizeof(n->L));
    if (st == SW_OK) st = dalloc(n, &n->x0, act_bytes(n, max_batch, 8));
    for (int l = 0; l < kLayers - 1 && st == SW_OK; ++l) st = dalloc(n, &n->act[l], act_bytes(n, max_batch, 32));
    for (int k = 0; k < kLayers - 2 && st == SW_OK; ++k) st = dalloc(n, &n->relu[k], act_bytes(n, max_batch, 32));
    for (int k = 0; k < 2 && st == SW_OK; ++k) {
        st = dalloc(n, &n->g[k], act_bytes(n, max_batch, 32));
        if (st == SW_OK) st = dalloc(n, &n->dz[k], act_bytes(n, max_batch, 32));
    }
    if (st == SW_OK) st = dalloc(n, &n->dz6, act_bytes(n, max_batch, 8));
    if (st == SW_OK) st = dalloc(n, (void **)&n->delta, (size_t)max_batch * H * W * 16);
    if (st == SW_OK) st = dalloc(n, (void **)&n->target, (size_t)max_batch * H * W * 16);
    if (st == SW_OK) st = dalloc(n, (void **)&n->stats, (size_t)max_batch * sizeof(SwGateStats));
    if (st == SW_OK) st = dalloc(n, (void **)&n->dh_part, (size_t)max_batch * H * (W / 64) * sizeof(double));
    if (st == SW_OK)
        st = dalloc(n, (void **)&n->apply_part, (size_t)sw_sur_apply_slots((int64_t)H * W, max_batch) * sizeof(SwApplyPart));
    if (st == SW_OK) st = dalloc(n, (void **)&n->apply_ticket, (size_t)max_batch * sizeof(unsigned));
    if (st == SW_OK)   // the smallest fused tile is 16 x 16
        st = dalloc(n, (void **)&n->dh_tile, (size_t)max_batch * ((H + 15) / 16) * (W / 16) * sizeof(double));
    if (st == SW_OK) st = dalloc(n, (void **)&n->active, (size_t)max_batch * 4);
    if (st == SW_OK) st = dalloc(n, (void **)&n->judge, (size_t)max_batch * sizeof(SwJudge));
    if (st == SW_OK) st = dalloc(n, (void **)&n->reject, (size_t)max_batch * 4);
    if (st == SW_OK && hipMemcpy(n->L_dev, n->L, sizeof(n->L), hipMemcpyHostToDevice) != hipSuccess)
        st = sw_fail(SW_EHIP, "surrogate_create: layer table upload");
    if (st == SW_OK) {
        // He-normal weights from the seed (fan-in 9 * cin); the output layer
        // starts 10x smaller so the untrained network is close to persistence
        std::mt19937_64 rng(cfg->seed);
        std::normal_distribution<double> nd(0.0, 1.0);
        std::vector<float> p((size_t)off, 0.f);
        for (int l = 0; l < kLayers; ++l) {
            const SwLayerDesc &L = n->L[l];
            const double sd = std::sqrt(2.0 / (9.0 * L.cin)) * (l == kLayers - 1 ? 0.1 : 1.0);
            for (int64_t i = 0; i < (int64_t)L.cout * 9 * L.cin; ++i) p[L.w_off + i] = (float)(sd * nd(rng));
        }
        if (hipMemcpy(n->master, p.data(), off * 4, hipMemcpyHostToDevice) != hipSuccess)
            st = sw_fail(SW_EHIP, "surrogate_create: weight upload");
    }
    if (st == SW_OK) st = relayout(n, nullptr);
    if (st == SW_OK && hipDeviceSynchronize() != hipSuccess) st = sw_fail(SW_EHIP, "surrogate_create: sync");
    for (int c = 0; c < 3; ++c) {
        n->nrm.in_off[c] = c == 0 ? 1.f : 0.f;
        n->nrm.in_scale[c] = c == 0 ? 0.25f : 0.25f * std::sqrt(9.8f);
        n->nrm.out_scale[c] = n->nrm.in_scale[c];
    }
    if (st != SW_OK) {
        sw_surrogate_destroy(n);
        return st;
    }
    *out = n;
    return SW_OK;
}

sw_status sw_surrogate_destroy(sw_net *n) {
    if (!n) return SW_OK;
    (void)use_dev(n);
    drop_graphs(n);
    if (n->cap) (void)hipStreamDestroy(n->cap);
    drop_shadow(n);
    for (void *p : n->allocs) (void)hipFree(p);
    delete n;
    return SW_OK;
}

sw_status sw_surrogate_params(sw_net *n, float **master, int64_t *count) {
    if (!n || !master || !count) return sw_fail(SW_EINVAL, "surrogate_params: NULL argument");
    *master = n->master;
    *count = n->nparams;
    return SW_OK;
}

sw_status sw_surrogate_set_norm(sw_net *n, const float in_offset[3], const float in_scale[3],
                                const float out_scale[3]) {
    if (!n || !in_offset || !in_scale || !out_scale) return sw_fail(SW_EINVAL, "surrogate_set_norm: NULL argument");
    for (int c = 0; c < 3; ++c) {
        if (!(in_scale[c] > 0) || !(out_scale[c] > 0)) return sw_fail(SW_EINVAL, "surrogate_set_norm: scale <= 0");
        n->nrm.in_off[c] = in_offset[c];
        n->nrm.in_scale[c] = in_scale[c];
        n->nrm.out_scale[c] = out_scale[c];
    }
    drop_graphs(n);   // captured rollouts hold the old values
    return SW_OK;
}

sw_status sw_surrogate_set_graph(sw_net *n, int32_t enable) {
    if (!n) return sw_fail(SW_EINVAL, "surrogate_set_graph: NULL network");
    n->use_graph = enable != 0;
    if (!n->use_graph) drop_graphs(n);
    return SW_OK;
}

sw_status sw_surrogate_set_block_cap(sw_net *n, int32_t max_blocks) {
    if (!n) return sw_fail(SW_EINVAL, "surrogate_set_block_cap: NULL network");
    if (max_blocks < 0 || max_blocks > kWgradBlocks)
        return sw_fail(SW_EINVAL, "surrogate_set_block_cap: %d outside [0, %d]", max_blocks, kWgradBlocks);
    n->block_cap = max_blocks;
    drop_graphs(n);   // captured rollouts hold the old launch shapes
    return SW_OK;
}

sw_status sw_surrogate_set_fused(sw_net *n, int32_t mode) {
    if (!n) return sw_fail(SW_EINVAL, "surrogate_set_fused: NULL network");
    if (mode < 0 || mode > 2) return sw_fail(SW_EINVAL, "surrogate_set_fused: mode %d (0, 1 or 2)", mode);
    n->fused_mode = mode;
    drop_graphs(n);
    return SW_OK;
}

sw_status sw_surrogate_sync_weights(sw_net *n, void *stream) {
    if (!n) return sw_fail(SW_EINVAL, "surrogate_sync_weights: NULL network");
    sw_status st = use_dev(n);
    if (st != SW_OK) return st;
    return relayout(n, (hipStream_t)stream);
}

sw_status sw_surrogate_forward(sw_net *n, const float *u, int32_t B, float *delta, void *stream) {
    sw_status st = check_net(n, B);
    if (st != SW_OK) return st;
    if (!u) return sw_fail(SW_EINVAL, "surrogate_forward: NULL input");
    hipStream_t s = (hipStream_t)stream;
    SHIP(sw_sur_prep_dense(u, nullptr, B, n->H, n->W, n->cfg.bc_x, n->cfg.bc_y, n->nrm, n->x0, nullptr, s));
    if ((st = forward(n, B, false, s)) != SW_OK) return st;
    if (delta) SHIP(hipMemcpyAsync(delta, n->delta, (size_t)B * n->H * n->W * 16, hipMemcpyDeviceToDevice, s));
    return SW_OK;
}

sw_status sw_surrogate_activation(sw_net *n, int32_t layer, const void **ptr, int64_t *bytes) {
    if (!n || !ptr) return sw_fail(SW_EINVAL, "surrogate_activation: NULL argument");
    if (layer < 0 || layer > kLayers) return sw_fail(SW_EINVAL, "surrogate_activation: layer %d", layer);
    if (layer == 0) *ptr = n->x0;
    else if (layer < kLayers) *ptr = n->act[layer - 1];
    else *ptr = n->delta;
    if (bytes)
        *bytes = layer == kLayers ? (int64_t)n->maxB * n->H * n->W * 16
                                  : (int64_t)act_bytes(n, n->maxB, layer == 0 ? 8 : 32);
    return SW_OK;
}

sw_status sw_surrogate_grad(sw_net *n, const float *u, const float *u8, int32_t B, float *grad, float *loss,
                            void *stream) {
    sw_status st = check_net(n, B);
    if (st != SW_OK) return st;
    if (!u || !u8) return sw_fail(SW_EINVAL, "surrogate_grad: NULL input");
    hipStream_t s = (hipStream_t)stream;
    SHIP(sw_sur_prep_dense(u, u8, B, n->H, n->W, n->cfg.bc_x, n->cfg.bc_y, n->nrm, n->x0, n->target, s));
    if ((st = forward(n, B, true, s)) != SW_OK) return st;
    if ((st = backward(n, B, loss, s)) != SW_OK) return st;
    if (grad) SHIP(hipMemcpyAsync(grad, n->grad, n->nparams * 4, hipMemcpyDeviceToDevice, s));
    return SW_OK;
}

sw_status sw_surrogate_train_step(sw_net *n, const float *u, const float *u8, int32_t B, float lr, float *loss,
                                  void *stream) {
    sw_status st = check_net(n, B);
    if (st != SW_OK) return st;
    if (!(lr > 0)) return sw_fail(SW_EINVAL, "surrogate_train_step: lr %g", lr);
    if ((st = sw_surrogate_grad(n, u, u8, B, nullptr, loss, stream)) != SW_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    n->adam_t += 1;
    SwAdam ad{lr, 0.9f, 0.999f, 1e-8f, 0.f, 0.f};
    ad.c1 = (float)(1.0 / (1.0 - std::pow(0.9, (double)n->adam_t)));
    ad.c2 = (float)(1.0 / (1.0 - std::pow(0.999, (double)n->adam_t)));
    SHIP(sw_sur_adam(n->master, n->m, n->v, n->grad, n->nparams, ad, s));
    return relayout(n, s);
}

namespace {
// The rollout's launches on stream s (no host sync, no allocation once the
// batch is prepared): halo fill, then per jump the network step, the gate, the
// restore of rejected grids and their masked solver steps.  Leaves the batch's
// current buffer at the final state.
// Whether a rollout of B grids runs the network as one fused launch.  In
// automatic mode: while the batch has at most kFusedMaxTiles 16 x 32 output
// tiles per CU.  The fused launch recomputes a 6-pixel border of every tile
// (1.5-1.8x the flops) but moves only the state and the prediction through
// HBM and takes one launch per jump instead of six; measured on MI355X with
// 256^2 grids (128 such tiles each), the whole 64-step rollout is 1.37x
// faster than with per-layer launches at batch 1, 1.05x at batch 4 (2 tiles
// per CU), and 0.94x at batch 8.
constexpr int kFusedMaxTiles = 2;
bool rollout_fused(const sw_net *n, int B) {
    if (n->fused_mode != 2) return n->fused_mode == 1;
    const int64_t tiles = (int64_t)B * ((n->H + 15) / 16) * (n->W / 32);
    return tiles <= (int64_t)kFusedMaxTiles * sw_device_cus();
}

sw_status enqueue_rollout(sw_net *n, sw_batch *solver, const SwBatchInfo &bi, int32_t nsteps, const sw_gate *gate,
                          int32_t *fallbacks, hipStream_t s) {
    const int B = bi.n;
    int cur = bi.cur;
    sw_status st;
    if ((st = sw_batch_fill_halo(solver, s)) != SW_OK) return st;
    const bool fused = rollout_fused(n, B);
    for (int j = 0; j < nsteps / n->cfg.jump; ++j) {
        if (fused) {
            // the network in one launch, the update with the gate's statistics, then the gate's verdict and
            // the rejected grids' solver steps in one launch
            SwNetFusedArgs fa{};
            fa.grids = bi.d_grids;
            fa.cur = cur;
            fa.B = B;
            fa.H = n->H;
            fa.W = n->W;
            fa.nrm = n->nrm;
            for (int l = 0; l < kLayers; ++l) {
                fa.wk[l] = n->L[l].wk;
                fa.bias[l] = n->master + n->L[l].b_off;
            }
            fa.delta = n->delta;
            fa.dh_tile = gate->project_mass ? n->dh_tile : nullptr;
            fa.clear_stats = n->stats;
            fa.max_blocks = n->block_cap;
            SHIP(sw_net_fused(fa, s));
            int th = 0, tw = 0;
            sw_net_fused_tile(B, n->H, n->W, &th, &tw);
            SHIP(sw_sur_apply(n->delta, n->dh_tile, ((n->H + th - 1) / th) * (n->W / tw), bi.d_grids, cur, B, n->H,
                              n->W, n->nrm, gate->project_mass, bi.bc_x, bi.bc_y, n->stats, n->apply_part,
                              n->apply_ticket, s));
            cur ^= 1;
            if ((st = (sw_status)sw_batch_internal_set_cur(solver, cur)) != SW_OK) return st;
            const SwFallbackGate fg{n->stats, gate->mass_rel_tol, gate->hmin, fallbacks};
            if ((st = (sw_status)sw_batch_internal_gated_fallback(solver, n->cfg.jump, fg, s)) != SW_OK) return st;
            continue;
        }
        // U^n in buffer cur; every grid's U^{n+jump} ends in buffer cur ^ 1
        const RolloutInput in{bi.d_grids, cur, gate->project_mass != 0};
        if ((st = forward(n, B, false, s, &in)) != SW_OK) return st;
        SHIP(sw_sur_apply(n->delta, n->dh_part, n->H * (n->W / 64), bi.d_grids, cur, B, n->H, n->W, n->nrm,
                          gate->project_mass, bi.bc_x, bi.bc_y, n->stats, n->apply_part, n->apply_ticket, s));
        // the gate; rejected grids: U^n over the prediction, then the plain solver takes the jump (an
        // even number of steps, so it ends where it started); accepted grids keep the prediction
        SHIP(sw_sur_gate_restore(bi.d_grids, cur, B, n->H, n->W, n->stats, gate->mass_rel_tol, gate->hmin, n->active,
                                 fallbacks, s));
        cur ^= 1;
        if ((st = (sw_status)sw_batch_internal_set_cur(solver, cur)) != SW_OK) return st;
        if ((st = (sw_status)sw_batch_internal_fallback(solver, n->cfg.jump, n->active, s)) != SW_OK) return st;
    }
    return SW_OK;
}
}  // namespace

sw_status sw_surrogate_advance(sw_net *n, sw_batch *solver, int32_t nsteps, const sw_gate *gate,
                               int32_t *fallbacks, double *l2, void *stream) {
    if (!n || !solver || !gate) return sw_fail(SW_EINVAL, "surrogate_advance: NULL argument");
    SwBatchInfo bi;
    sw_status st = (sw_status)sw_batch_internal_info(solver, &bi);
    if (st != SW_OK) return st;
    if ((st = check_net(n, bi.n)) != SW_OK) return st;
    if (bi.dtype != SW_F32) return sw_fail(SW_ENOTSUP, "surrogate_advance: the surrogate advances FP32 batches");
    if (bi.same_nx != n->W || bi.same_ny != n->H)
        return sw_fail(SW_EINVAL, "surrogate_advance: every grid must be %d x %d", n->W, n->H);
    if (nsteps < 0 || nsteps % n->cfg.jump)
        return sw_fail(SW_EINVAL, "surrogate_advance: nsteps %d is not a multiple of the jump %d", nsteps, n->cfg.jump);
    if (bi.bc_x != n->cfg.bc_x || bi.bc_y != n->cfg.bc_y)
        return sw_fail(SW_EINVAL, "surrogate_advance: boundary conditions differ from the network's");
    if (gate->judge && !(gate->l2_tol >= 0)) return sw_fail(SW_EINVAL, "surrogate_advance: l2_tol %g", gate->l2_tol);
    hipStream_t s = (hipStream_t)stream;
    const int B = bi.n;
    if (gate->judge) {   // the plain solver's copy of U^n, and the books at the start
        if (n->shadow && !sw_batch_internal_compatible(n->shadow, solver)) drop_shadow(n);
        if (!n->shadow && (st = (sw_status)sw_batch_internal_clone(solver, &n->shadow, &n->shadow_arena)) != SW_OK)
            return st;
        if ((st = (sw_status)sw_batch_internal_copy_state(n->shadow, solver, s)) != SW_OK) return st;
        SHIP(sw_sur_judge_begin(bi.d_sc, B, n->judge, s));
        if ((st = enqueue_rollout(n, solver, bi, nsteps, gate, fallbacks, s)) != SW_OK) return st;
        // the plain solver over the same span, then the verdict per grid
        if ((st = sw_batch_step(n->shadow, nsteps, stream)) != SW_OK) return st;
        SwBatchInfo si;
        if ((st = (sw_status)sw_batch_internal_info(n->shadow, &si)) != SW_OK) return st;
        SwBatchInfo now;
        if ((st = (sw_status)sw_batch_internal_info(solver, &now)) != SW_OK) return st;
        SHIP(sw_sur_judge(bi.d_grids, now.cur, si.d_grids, si.cur, B, n->H, n->W, n->judge, bi.d_sc, si.d_sc,
                          gate->l2_tol, nsteps / n->cfg.jump, n->reject, fallbacks, l2, s));
        return SW_OK;
    }
    if (!n->use_graph || nsteps == 0) return enqueue_rollout(n, solver, bi, nsteps, gate, fallbacks, s);
    // graph replay: everything the launches bake in is part of the key
    if ((st = (sw_status)sw_batch_internal_prepare(solver)) != SW_OK) return st;
    if ((st = (sw_status)sw_batch_internal_info(solver, &bi)) != SW_OK) return st;
    hipGraphExec_t exec = nullptr;
    for (auto &g : n->graphs)
        if (g.solver == solver && g.gen == bi.gen && g.cur == bi.cur && g.nsteps == nsteps && g.fallbacks == fallbacks &&
            g.gate.mass_rel_tol == gate->mass_rel_tol && g.gate.hmin == gate->hmin &&
            (g.gate.project_mass != 0) == (gate->project_mass != 0))
            exec = g.exec;
    if (exec) {
        const int njumps = nsteps / n->cfg.jump;
        if ((st = (sw_status)sw_batch_internal_set_cur(solver, bi.cur ^ (njumps & 1))) != SW_OK) return st;
    } else {
        if (n->graphs.size() >= 8) drop_graphs(n);
        if (!n->cap) SHIP(hipStreamCreateWithFlags(&n->cap, hipStreamNonBlocking));
        SHIP(hipStreamBeginCapture(n->cap, hipStreamCaptureModeThreadLocal));
        st = enqueue_rollout(n, solver, bi, nsteps, gate, fallbacks, n->cap);   // leaves the batch's final buffer current
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(n->cap, &graph);
        if (st != SW_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)sw_batch_internal_set_cur(solver, bi.cur);
            return st;
        }
        if (e != hipSuccess) {
            (void)sw_batch_internal_set_cur(solver, bi.cur);
            return sw_fail(SW_EHIP, "surrogate_advance: capture: %s", hipGetErrorString(e));
        }
        e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            (void)sw_batch_internal_set_cur(solver, bi.cur);
            return sw_fail(SW_EHIP, "surrogate_advance: instantiate: %s", hipGetErrorString(e));
        }
        sw_net::Graph g{solver, bi.gen, bi.cur, nsteps, *gate, fallbacks, exec};
        n->graphs.push_back(g);
    }
    SHIP(hipGraphLaunch(exec, s));
    return SW_OK;
}

}  // extern "C"
