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
