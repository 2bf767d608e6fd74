"""Pins of the surrogate's CPU FP64 oracle: the 3x3 convolution against
scipy's 2-D correlation, the analytic gradient against central finite
differences, the input ghosts against the solver oracle's boundary rule, and
the BF16 rounding against torch's conversion."""
import numpy as np
import pytest
import scipy.signal
import torch

import oracle
from oracle import net_oracle as no
from paper_1107_2157_amd import ics

OFF = (1.0, 0.0, 0.0)
SCALE = (0.25, 0.25 * 9.8 ** 0.5, 0.25 * 9.8 ** 0.5)


def test_conv3x3_is_2d_correlation():
    rng = np.random.default_rng(0)
    xh = rng.standard_normal((2, 9, 11, 5))
    w = rng.standard_normal((4, 9, 5))
    b = rng.standard_normal(4)
    got = no.conv3x3(xh, w, b)
    for bb in range(2):
        for co in range(4):
            want = sum(scipy.signal.correlate2d(xh[bb, :, :, ci], w[co, :, ci].reshape(3, 3), mode="valid")
                       for ci in range(5)) + b[co]
            np.testing.assert_allclose(got[bb, :, :, co], want, rtol=1e-12, atol=1e-12)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.00390625, 1.0078125, 1.01171875, 3.0e38, -2.5]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(no.bf16(x), want)


@pytest.mark.parametrize("bcx,bcy", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_input_ghosts_follow_the_boundary_rule(bcx, bcy):
    h, hu, hv = (a.numpy() for a in ics.random_state(7, 5, seed=2))
    u = np.stack([h, hu, hv])[None].astype(np.float32)
    x = no.input_tensor(u, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), bcx, bcy, quant=False)
    H, U, V = (oracle.with_halo(a.astype(np.float32).astype(np.float64)) for a in (h, hu, hv))
    oracle.fill_halo(H, U, V, bcx, bcy)
    for c, ref in enumerate((H, U, V)):
        np.testing.assert_array_equal(x[0, :, :, c], ref)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    h, hu, hv = (a.numpy() for a in ics.random_state(7, 6, seed=4, amp_h=0.4, amp_m=0.1))
    u = np.stack([h, hu, hv])[None]
    u8 = u + 0.01 * rng.standard_normal(u.shape)
    p = no.init_params(5, out_gain=1.0)
    out_scale = (0.01, 0.02, 0.02)
    loss, g = no.loss_and_grad(p, u, u8, OFF, SCALE, out_scale, bf16_mode=False)
    idx = np.concatenate([rng.choice(no.nparams(), 80, replace=False),
                          np.cumsum([co * 9 * ci + co for ci, co in no.LAYERS]) - 1])   # include last biases
    eps = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        lp, _ = no.loss_and_grad(pp, u, u8, OFF, SCALE, out_scale, bf16_mode=False)
        lm, _ = no.loss_and_grad(pm, u, u8, OFF, SCALE, out_scale, bf16_mode=False)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) * max(1.0, loss), (i, fd, g[i])


@pytest.mark.parametrize("c", [0.0, 0.375])
def test_residual_blocks_add_relu_of_bias(c):
    """With zero hidden weights and biases c >= 0 every residual block adds
    relu(c) = c to its input, so A_l = A_1 + (l - 1) c in the interior and
    the output layer sees A_5 = A_1 + 4c."""
    p = no.init_params(9, out_gain=1.0)
    layers = no.unpack(p)
    for l in range(1, 5):
        layers[l][0][:] = 0.0
        layers[l][1][:] = c
    flat = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in layers])
    h, hu, hv = (a.numpy() for a in ics.random_state(8, 6, seed=3))
    u = np.stack([h, hu, hv])[None]
    acts, delta = no.forward(flat, u, OFF, SCALE, bf16_mode=False)
    a1 = acts[1][:, 1:-1, 1:-1]
    for l in range(2, 6):
        np.testing.assert_allclose(acts[l][:, 1:-1, 1:-1], a1 + (l - 1) * c, rtol=0, atol=1e-14)
        assert not np.any(acts[l][:, 0]) and not np.any(acts[l][:, :, -1])      # zero padding stays zero
    w6, b6 = layers[5]
    want = no.conv3x3(no.pad(a1 + 4 * c), w6, b6)
    np.testing.assert_allclose(delta, want, rtol=1e-13, atol=1e-13)


def test_loss_of_the_zero_network_is_the_mean_squared_target():
    """With every parameter zero the prediction is zero, so the loss is the
    mean over pixels and the three channels of ((u8 - u) / out_scale)^2 and
    its bias gradient of the output layer is -2 * mean target per channel."""
    rng = np.random.default_rng(6)
    h, hu, hv = (a.numpy() for a in ics.random_state(9, 5, seed=6))
    u = np.stack([h, hu, hv])[None]
    u8 = u + 0.02 * rng.standard_normal(u.shape)
    out_scale = (0.01, 0.03, 0.05)
    loss, g = no.loss_and_grad(np.zeros(no.nparams()), u, u8, OFF, SCALE, out_scale, bf16_mode=False)
    t = [(u8[0, c].astype(np.float32) - u[0, c].astype(np.float32)) / np.float32(out_scale[c]) for c in range(3)]
    want = sum(float(np.sum(np.square(tc, dtype=np.float64))) for tc in t) / (3 * 9 * 5)
    assert abs(loss - want) <= 1e-12 * want
    np.testing.assert_allclose(g[-3:], [-2.0 * float(np.mean(tc, dtype=np.float64)) / 3 for tc in t], rtol=1e-12)


def test_param_count():
    assert no.nparams() == 38755


# ---- the Adam update (Kingma and Ba 2015, Algorithm 1) ----------------------
# Closed forms of the two moment recurrences m_t = b1 m_{t-1} + (1 - b1) g_t,
# v_t = b2 v_{t-1} + (1 - b2) g_t^2 from m_0 = v_0 = 0, pinned below without
# running the recurrence:
#  * first step: m_1 / (1 - b1) = g and v_1 / (1 - b2) = g^2, so the update
#    is -lr g / (|g| + eps) whatever b1, b2 are;
#  * a constant g for t steps: m_t = g (1 - b1^t), v_t = g^2 (1 - b2^t), so
#    every bias-corrected step is again -lr g / (|g| + eps);
#  * g_k = (-1)^k g: m_t = (1 - b1) g (-1)^t (1 - (-b1)^t) / (1 + b1) (a
#    geometric sum) while v_t = g^2 (1 - b2^t), which separates b1 from b2
#    and pins the bias correction of the first moment;
#  * g, then 0: the second step is -lr (b1 / (1 + b1)) g / (|g| sqrt(b2 / (1 + b2)) + eps).
B1, B2, EPS = 0.9, 0.999, 1e-8


def _adam_run(grads, lr, theta0):
    th = np.array(theta0, dtype=np.float64)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    out = []
    for t, g in enumerate(grads, start=1):
        th, m, v = no.adam_step(th, m, v, g, t, lr)
        out.append(th.copy())
    return out, m, v


def _grads():
    rng = np.random.default_rng(21)
    return np.concatenate([rng.standard_normal(200) * 10.0 ** rng.integers(-6, 3, 200),
                           [1e-8, -3e-9, 2.5e-8, 0.0]])      # |g| near eps pins where eps enters


def test_adam_first_step_closed_form():
    g = _grads()
    theta0 = np.linspace(-1.0, 1.0, g.size)
    (th,), m, v = _adam_run([g], 1e-3, theta0)
    np.testing.assert_allclose(th - theta0, -1e-3 * g / (np.abs(g) + EPS), rtol=1e-12, atol=1e-19)
    np.testing.assert_allclose(m, (1 - B1) * g, rtol=1e-15)
    np.testing.assert_allclose(v, (1 - B2) * g * g, rtol=1e-15)


def test_adam_constant_gradient_closed_form():
    g = _grads()
    theta0 = np.zeros(g.size)
    ths, m, v = _adam_run([g] * 25, 2e-3, theta0)
    for t, th in enumerate(ths, start=1):
        np.testing.assert_allclose(th, -t * 2e-3 * g / (np.abs(g) + EPS), rtol=1e-11, atol=1e-18)
    np.testing.assert_allclose(m, g * (1 - B1 ** 25), rtol=1e-12)
    np.testing.assert_allclose(v, g * g * (1 - B2 ** 25), rtol=1e-12)


def test_adam_alternating_gradient_closed_form():
    g = np.array([0.7, -1.3e-3, 4.0e2, 2.0e-7])
    lr = 1e-2
    T = 12
    ths, _, _ = _adam_run([(-1.0) ** k * g for k in range(1, T + 1)], lr, np.zeros(g.size))
    prev = np.zeros(g.size)
    for t, th in enumerate(ths, start=1):
        m_t = (1 - B1) * g * (-1.0) ** t * (1 - (-B1) ** t) / (1 + B1)
        v_t = g * g * (1 - B2 ** t)
        step = -lr * (m_t / (1 - B1 ** t)) / (np.sqrt(v_t / (1 - B2 ** t)) + EPS)
        np.testing.assert_allclose(th - prev, step, rtol=1e-10, atol=1e-18)
        prev = th


def test_adam_decay_after_a_zero_gradient_closed_form():
    g = _grads()
    ths, _, _ = _adam_run([g, np.zeros(g.size)], 1e-3, np.zeros(g.size))
    want = -1e-3 * (B1 / (1 + B1)) * g / (np.abs(g) * np.sqrt(B2 / (1 + B2)) + EPS)
    np.testing.assert_allclose(ths[1] - ths[0], want, rtol=1e-10, atol=1e-19)


def test_abs_sums_bound_the_gradient_and_equal_it_for_positive_terms():
    """The per-entry sum of |terms| is >= |gradient| everywhere, and equals it
    where every term is non-negative (all inputs and weights made positive,
    periodic ghosts, target below the prediction, hidden masks all on)."""
    rng = np.random.default_rng(8)
    h, hu, hv = (a.numpy() for a in ics.random_state(8, 6, seed=11, amp_h=0.3, amp_m=0.1))
    u = np.stack([h, hu, hv])[None]
    u8 = u + 0.01 * rng.standard_normal(u.shape)
    p = no.init_params(4, out_gain=1.0)
    _, g, s = no.loss_and_grad(p, u, u8, OFF, SCALE, (0.02, 0.02, 0.02), bf16_mode=False, abs_sums=True)
    assert np.all(s >= np.abs(g) * (1 - 1e-12))
    pos = np.abs(p)
    u_pos = np.stack([h * 0 + 2.0, np.abs(hu) + 0.1, np.abs(hv) + 0.1])[None]
    _, g, s = no.loss_and_grad(pos, u_pos, u_pos - 1.0, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (1.0, 1.0, 1.0),
                               bc_x=1, bc_y=1, bf16_mode=False, abs_sums=True)
    np.testing.assert_allclose(np.abs(g), s, rtol=1e-12)
