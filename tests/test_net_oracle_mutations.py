"""Strength of the surrogate oracle's pins: plant plausible mistakes in a
copy of oracle/net_oracle.py (on the CPU), load the copy as its own module,
and check that a quick battery of the same pins (2-D correlation, BF16
rounding, input ghosts, central differences, the residual closed form, the
zero network's loss) rejects every one, while accepting the unmodified
oracle."""
import os
import types

import numpy as np
import pytest
import scipy.signal
import torch

import oracle
from paper_1107_2157_amd import ics

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "net_oracle.py")
OFF = (1.0, 0.0, 0.0)
SCALE = (0.25, 0.25 * 9.8 ** 0.5, 0.25 * 9.8 ** 0.5)

# (name, text to find, replacement): the first occurrence is replaced
MUTATIONS = [
    ("conv taps transposed", "dy, dx = tap // 3, tap % 3\n        out +=", "dy, dx = tap % 3, tap // 3\n        out +="),
    ("conv bias dropped", "        out += b\n", "        out += 0.0 * b\n"),
    ("skip dropped in forward", "a = pad(q(a[:, 1:-1, 1:-1, :] + r if residual(l) else r))", "a = pad(q(r))"),
    ("skip gradient dropped", "g = g + g_out", "g = g"),
    ("mask of the wrong layer", "dz = g * masks[l - 1]", "dz = g * masks[l - 2]"),
    ("no ReLU mask", "masks.append(z > 0.0)", "masks.append(z > -1e300)"),
    ("input-gradient kernel not flipped", "wflip = w[:, ::-1, :].transpose(2, 1, 0)", "wflip = w.transpose(2, 1, 0)"),
    ("bf16 ties away from zero", "r = ((bits + 0x7FFF + lsb) >> 16) << 16", "r = ((bits + 0x8000) >> 16) << 16"),
    ("wall momentum not negated", "fx[0] = fx[-1] = -1", "fx[0] = fx[-1] = 1"),
    ("loss over pixels only", "n = delta.shape[0] * delta.shape[1] * delta.shape[2] * 3",
     "n = delta.shape[0] * delta.shape[1] * delta.shape[2]"),
    ("target sign", "(u8[:, c] - u[:, c])", "(u[:, c] - u8[:, c])"),
    ("weight gradient of the wrong tap", "gw[:, tap, :] = np.tensordot", "gw[:, 8 - tap, :] = np.tensordot"),
    ("Adam: first moment not bias-corrected", "m_hat = m / (1.0 - beta1 ** t)", "m_hat = m"),
    ("Adam: second moment not bias-corrected", "v_hat = v / (1.0 - beta2 ** t)", "v_hat = v"),
    ("Adam: decays swapped", "m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g",
     "m = beta2 * np.asarray(m, dtype=np.float64) + (1.0 - beta2) * g"),
    ("Adam: eps inside the root", "(np.sqrt(v_hat) + eps)", "np.sqrt(v_hat + eps)"),
    ("Adam: step along the gradient", "theta = np.asarray(theta, dtype=np.float64) - lr", "theta = np.asarray(theta, dtype=np.float64) + lr"),
    ("Adam: gradient not squared", "(1.0 - beta2) * g * g", "(1.0 - beta2) * np.abs(g)"),
]


def load(src: str) -> types.ModuleType:
    m = types.ModuleType("net_oracle_variant")
    exec(compile(src, SRC, "exec"), m.__dict__)
    return m


def battery(no) -> list[str]:
    bad = []

    def check(name, fn):
        try:
            ok = bool(fn())
        except Exception:
            ok = False
        if not ok:
            bad.append(name)

    rng = np.random.default_rng(0)

    def conv():
        xh = rng.standard_normal((1, 7, 8, 3))
        w = rng.standard_normal((2, 9, 3))
        b = rng.standard_normal(2)
        got = no.conv3x3(xh, w, b)
        want = np.stack([sum(scipy.signal.correlate2d(xh[0, :, :, ci], w[co, :, ci].reshape(3, 3), mode="valid")
                             for ci in range(3)) + b[co] for co in range(2)], axis=-1)
        return np.allclose(got[0], want, rtol=1e-12, atol=1e-12)

    def rounding():
        x = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-5, 5, 2000), [1.00390625, 1.01171875]])
        return np.array_equal(no.bf16(x), torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy())

    def ghosts():
        h, hu, hv = (a.numpy() for a in ics.random_state(6, 5, seed=2))
        u = np.stack([h, hu, hv])[None].astype(np.float32)
        x = no.input_tensor(u, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0), 0, 0, quant=False)
        H, U, V = (oracle.with_halo(a.astype(np.float32).astype(np.float64)) for a in (h, hu, hv))
        oracle.fill_halo(H, U, V, 0, 0)
        return all(np.array_equal(x[0, :, :, c], r) for c, r in enumerate((H, U, V)))

    h, hu, hv = (a.numpy() for a in ics.random_state(6, 5, seed=4, amp_h=0.4, amp_m=0.1))
    u = np.stack([h, hu, hv])[None]
    u8 = u + 0.01 * rng.standard_normal(u.shape)
    osc = (0.01, 0.02, 0.02)

    def fd():
        p = no.init_params(5, out_gain=1.0)
        loss, g = no.loss_and_grad(p, u, u8, OFF, SCALE, osc, bf16_mode=False)
        idx = np.concatenate([rng.choice(no.nparams(), 30, replace=False),
                              np.cumsum([co * 9 * ci + co for ci, co in no.LAYERS]) - 1])
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += 1e-6
            pm[i] -= 1e-6
            fdv = (no.loss_and_grad(pp, u, u8, OFF, SCALE, osc, bf16_mode=False)[0] -
                   no.loss_and_grad(pm, u, u8, OFF, SCALE, osc, bf16_mode=False)[0]) / 2e-6
            if abs(fdv - g[i]) > 1e-6 * max(1.0, abs(g[i])) * max(1.0, loss):
                return False
        return True

    def residual_form():
        c = 0.375
        layers = no.unpack(no.init_params(9, out_gain=1.0))
        for l in range(1, 5):
            layers[l][0][:] = 0.0
            layers[l][1][:] = c
        flat = np.concatenate([np.concatenate([w.ravel(), b]) for w, b in layers])
        acts, _ = no.forward(flat, u, OFF, SCALE, bf16_mode=False)
        return np.allclose(acts[5][:, 1:-1, 1:-1], acts[1][:, 1:-1, 1:-1] + 4 * c, rtol=0, atol=1e-14)

    def zero_net():
        loss, g = no.loss_and_grad(np.zeros(no.nparams()), u, u8, OFF, SCALE, osc, bf16_mode=False)
        t = [(u8[0, c].astype(np.float32) - u[0, c].astype(np.float32)) / np.float32(osc[c]) for c in range(3)]
        want = sum(float(np.sum(np.square(tc, dtype=np.float64))) for tc in t) / (3 * u.shape[2] * u.shape[3])
        return abs(loss - want) <= 1e-12 * want and np.allclose(
            g[-3:], [-2.0 * float(np.mean(tc, dtype=np.float64)) / 3 for tc in t], rtol=1e-12)

    def adam():
        # first step, then a zero gradient, then a constant one (closed forms
        # of the moment recurrences; see test_net_oracle.py)
        b1, b2, eps, lr = 0.9, 0.999, 1e-8, 1e-3
        g = np.concatenate([rng.standard_normal(50) * 10.0 ** rng.integers(-6, 3, 50), [1e-8, -2e-8]])
        th, m, v = no.adam_step(np.zeros(g.size), np.zeros(g.size), np.zeros(g.size), g, 1, lr)
        ok = np.allclose(th, -lr * g / (np.abs(g) + eps), rtol=1e-12, atol=1e-19)
        th2, _, _ = no.adam_step(th, m, v, np.zeros(g.size), 2, lr)
        want = -lr * (b1 / (1 + b1)) * g / (np.abs(g) * np.sqrt(b2 / (1 + b2)) + eps)
        ok = ok and np.allclose(th2 - th, want, rtol=1e-10, atol=1e-19)
        th, m, v = np.zeros(g.size), np.zeros(g.size), np.zeros(g.size)
        for t in range(1, 6):
            th, m, v = no.adam_step(th, m, v, g, t, lr)
        return ok and np.allclose(th, -5 * lr * g / (np.abs(g) + eps), rtol=1e-11, atol=1e-18)

    for name, fn in (("conv", conv), ("bf16", rounding), ("ghosts", ghosts), ("central differences", fd),
                     ("residual closed form", residual_form), ("zero network", zero_net), ("adam", adam)):
        check(name, fn)
    return bad


def test_unmodified_oracle_passes_the_battery():
    assert battery(load(open(SRC).read())) == []


@pytest.mark.parametrize("name,find,repl", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_battery_rejects_planted_mistake(name, find, repl):
    src = open(SRC).read()
    assert find in src, f"mutation site of '{name}' not found"
    bad = battery(load(src.replace(find, repl, 1)))
    assert bad, f"no pin rejects '{name}'"
