"""CPU FP64 oracle of the learned surrogate (forward, loss, gradients).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline); shares
nothing with the HIP path.  Written from the definition of the network:

* input: ``x_c = (u_c - offset_c) / scale_c`` for ``u = (h, hu, hv)``, with a
  one-cell halo holding the boundary ghosts (reflective: mirror with the
  wall-normal momentum negated; periodic: wrap), arranged NHWC;
* ``A_1 = relu(Z_1)``, then four residual blocks ``A_l = A_{l-1} + relu(Z_l)``
  (l = 2..5), then ``delta = Z_6`` (3 channels), where
  ``Z_l = conv3x3(A_{l-1}, W_l) + b_l`` with zero padding (``A_0`` is the input);
* ``conv3x3(x, W)[p, co] = sum_{tap, ci} x[p + (tap // 3 - 1, tap % 3 - 1), ci] W[co, tap, ci]``
  (cross-correlation; tap = 3 * ky + kx);
* loss: mean over pixels and the three channels of ``(delta - target)^2``,
  ``target = (u8 - u) / out_scale``;
* gradients by the chain rule: ``dZ_6 = 2 (delta - target) / N``,
  ``dW_l[co, tap, ci] = sum_p dZ_l[p, co] A_{l-1}[p + tap, ci]``,
  ``db_l = sum_p dZ_l``, ``G_{l-1}[q, ci] = sum_{tap, co} dZ_l[q - tap, co] W_l[co, tap, ci]``
  plus ``G_l`` when layer l is a residual block (``G_l = dL/dA_l``),
  ``dZ_{l-1} = G_{l-1} * (Z_{l-1} > 0)``;
* the training update: Adam (Kingma and Ba 2015, Algorithm 1) on the FP64
  parameter vector, with the moment decays 0.9 / 0.999 and eps = 1e-8 the
  network's trainer uses.

``bf16=True`` rounds the tensors the GPU stores in BF16 (input, weights,
hidden activations, gradient seeds and hidden-layer gradients ``G``, ``dZ``)
to BF16 after computing them, so the oracle sees the same quantised values;
accumulation is FP64 throughout.
"""
from __future__ import annotations

import numpy as np

LAYERS = [(3, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3)]


def residual(l: int) -> bool:
    """Layer l (0-based) adds its input to its output: the 32 -> 32 blocks."""
    return 1 <= l <= len(LAYERS) - 2


def nparams() -> int:
    return sum(co * 9 * ci + co for ci, co in LAYERS)


def unpack(params):
    """Flat master vector -> [(W[co][9][ci], b[co])] per layer."""
    p = np.asarray(params, dtype=np.float64)
    out, off = [], 0
    for ci, co in LAYERS:
        w = p[off:off + co * 9 * ci].reshape(co, 9, ci)
        off += co * 9 * ci
        b = p[off:off + co]
        off += co
        out.append((w, b))
    return out


def bf16(a):
    """Round to bfloat16 (nearest, ties to even) via FP32, as the GPU converts."""
    f = np.asarray(a, dtype=np.float32)
    bits = f.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    r = ((bits + 0x7FFF + lsb) >> 16) << 16
    return (r.astype(np.uint32)).view(np.float32).astype(np.float64)


def input_tensor(u, offset, scale, bc_x=0, bc_y=0, quant=True):
    """[B][3][H][W] state -> normalised NHWC input with halo [B][H+2][W+2][3]."""
    u = np.asarray(u, dtype=np.float32)
    B, _, H, W = u.shape
    ys = np.array([H - 1 if bc_y else 0] + list(range(H)) + [0 if bc_y else H - 1])
    xs = np.array([W - 1 if bc_x else 0] + list(range(W)) + [0 if bc_x else W - 1])
    fy = np.ones(H + 2, dtype=np.float32)
    fx = np.ones(W + 2, dtype=np.float32)
    if not bc_y:
        fy[0] = fy[-1] = -1
    if not bc_x:
        fx[0] = fx[-1] = -1
    g = u[:, :, ys][:, :, :, xs]                      # [B][3][H+2][W+2]
    g = g.copy()
    g[:, 1] *= fx[None, None, :]
    g[:, 2] *= fy[None, :, None]
    x = np.empty((B, H + 2, W + 2, 3), dtype=np.float32)
    for c in range(3):
        x[..., c] = (g[:, c] - np.float32(offset[c])) / np.float32(scale[c])
    return bf16(x) if quant else x.astype(np.float64)


def pad(a):
    B, H, W, C = a.shape
    out = np.zeros((B, H + 2, W + 2, C))
    out[:, 1:-1, 1:-1] = a
    return out


def conv3x3(xh, w, b=None):
    """xh: [B][H+2][W+2][ci] (halo), w: [co][9][ci] -> [B][H][W][co]."""
    B, Hp, Wp, _ = xh.shape
    H, W = Hp - 2, Wp - 2
    out = np.zeros((B, H, W, w.shape[0]))
    for tap in range(9):
        dy, dx = tap // 3, tap % 3
        out += np.tensordot(xh[:, dy:dy + H, dx:dx + W, :], w[:, tap, :], axes=([3], [1]))
    if b is not None:
        out += b
    return out


def forward(params, u, offset, scale, bc_x=0, bc_y=0, bf16_mode=True, masks=None):
    """Returns (activations with halo [x0, A1..A5], delta [B][H][W][3]);
    appends ``Z_l > 0`` of the hidden layers to ``masks`` if given."""
    q = bf16 if bf16_mode else (lambda a: np.asarray(a, dtype=np.float64))
    layers = [(q(w), b) for w, b in unpack(params)]
    x = input_tensor(u, offset, scale, bc_x, bc_y, quant=bf16_mode)
    acts = [x]
    a = x
    for l, (w, b) in enumerate(layers):
        z = conv3x3(a, w, b)
        if l == len(layers) - 1:
            return acts, z
        if masks is not None:
            masks.append(z > 0.0)
        r = np.maximum(z, 0.0)
        a = pad(q(a[:, 1:-1, 1:-1, :] + r if residual(l) else r))
        acts.append(a)


def target_of(u, u8, out_scale):
    """Normalised 8-step increment ``(u8 - u) / out_scale`` as [B][H][W][3]."""
    u = np.asarray(u, dtype=np.float32)
    u8 = np.asarray(u8, dtype=np.float32)
    return np.stack([(u8[:, c] - u[:, c]) / np.float32(out_scale[c]) for c in range(3)], axis=-1).astype(np.float64)


def weight_grad(dz, a_in):
    """dW[co, tap, ci] = sum_p dZ[p, co] A[p + tap, ci] and db[co] = sum_p dZ[p, co]
    (dz: [B][H][W][co], a_in: the layer input with halo)."""
    H, W = dz.shape[1], dz.shape[2]
    gw = np.zeros((dz.shape[3], 9, a_in.shape[3]))
    for tap in range(9):
        dy, dx = tap // 3, tap % 3
        gw[:, tap, :] = np.tensordot(dz, a_in[:, dy:dy + H, dx:dx + W, :], axes=([0, 1, 2], [0, 1, 2]))
    return gw, dz.sum(axis=(0, 1, 2))


def input_grad(dz, w):
    """dL/dA_in[q, ci] = sum_{tap, co} dZ[q - off(tap), co] W[co, tap, ci]: the
    correlation of the zero-padded dZ with the flipped, transposed kernel."""
    wflip = w[:, ::-1, :].transpose(2, 1, 0)          # [ci][tap'][co], tap' = 8 - tap
    return conv3x3(pad(dz), wflip)


def backward(params, acts, masks, delta, tgt, bf16_mode=True, abs_sums=False):
    """Loss and flat gradient from a forward pass's activations (with halo,
    ``acts[l]`` = input of layer l), the hidden layers' masks ``Z_l > 0``, the
    output ``delta`` and the target.  With ``abs_sums`` also returns, per
    gradient entry, the sum of the absolute values of the terms it adds up
    (``sum_p |dZ| |A|`` for a weight, ``sum_p |dZ|`` for a bias): the scale a
    rounding bound for that sum is stated against."""
    q = bf16 if bf16_mode else (lambda a: np.asarray(a, dtype=np.float64))
    layers = [(q(w), b) for w, b in unpack(params)]
    n = delta.shape[0] * delta.shape[1] * delta.shape[2] * 3
    d = delta - tgt
    loss = float(np.sum(d * d) / n)
    dz = q(2.0 * d / n)
    g_out = None                     # dL/d(output of layer l), needed where layer l is residual
    grads, sums = [None] * len(layers), [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        grads[l] = weight_grad(dz, acts[l])
        if abs_sums:
            sums[l] = weight_grad(np.abs(dz), np.abs(acts[l]))
        if l == 0:
            break
        g = input_grad(dz, layers[l][0])
        if residual(l):
            g = g + g_out
        g = q(g)
        dz = g * masks[l - 1]
        g_out = g
    flat = np.concatenate([np.concatenate([gw.ravel(), gb]) for gw, gb in grads])
    if not abs_sums:
        return loss, flat
    return loss, flat, np.concatenate([np.concatenate([sw.ravel(), sb]) for sw, sb in sums])


def loss_and_grad(params, u, u8, offset, scale, out_scale, bc_x=0, bc_y=0, bf16_mode=True, abs_sums=False):
    """MSE loss and the gradient (flat, master layout) of one pair."""
    masks = []
    acts, delta = forward(params, u, offset, scale, bc_x, bc_y, bf16_mode, masks)
    return backward(params, acts, masks, delta, target_of(u, u8, out_scale), bf16_mode, abs_sums)


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, "Adam: a method for stochastic
    optimization", Algorithm 1) of step number ``t`` (1-based): exponential
    moving averages of the gradient and of its square, each divided by its
    bias correction ``1 - beta^t``, and the step ``lr * m_hat / (sqrt(v_hat) + eps)``
    against the gradient.  Returns the new ``(theta, m, v)`` in FP64."""
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    theta = np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps)
    return theta, m, v


def init_params(seed: int, out_gain: float = 0.1):
    """He-normal test weights (fan-in 9 * cin), small random biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for l, (ci, co) in enumerate(LAYERS):
        sd = np.sqrt(2.0 / (9 * ci)) * (out_gain if l == len(LAYERS) - 1 else 1.0)
        parts.append(rng.standard_normal(co * 9 * ci) * sd)
        parts.append(rng.standard_normal(co) * 0.05)
    return np.concatenate(parts)
