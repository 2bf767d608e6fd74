"""The learned surrogate on the GPU (through the C ABI): forward activations
and gradients against the CPU FP64 oracle fed the same BF16-quantised
tensors, training, the forced fallback, and what the trained network gains
over the method without it."""
import numpy as np
import pytest
import torch

from oracle import net_oracle as no
from paper_1107_2157_amd import ics, surrogate, sw
from swtest import announce

pytestmark = pytest.mark.gpu

OFF, SCALE = surrogate.IN_OFFSET, surrogate.IN_SCALE


def states(n, H, W, seed):
    u = surrogate.initial_states(n, H, W, seed)
    g = torch.Generator().manual_seed(seed)
    u[:, 1:] += 0.05 * (torch.rand((n, 2, H, W), generator=g) - 0.5).cuda()
    return u


def make_net(H, W, B, params, out_scale):
    net = sw.Surrogate(H, W, B, jump=8, seed=1)
    net.set_params(torch.tensor(params, dtype=torch.float32))
    net.set_norm(OFF, SCALE, out_scale)
    return net


U32 = 2.0 ** -24          # FP32 unit roundoff


def gamma(n):
    """Bound on the relative error of an n-term FP32 sum, |err| <= gamma(n) *
    sum |terms| (Higham, Accuracy and Stability of Numerical Algorithms, 3.1)."""
    return n * U32 / (1.0 - n * U32)


def ulp_bf16(x):
    """Spacing of BF16 numbers (8 significant bits) at |x|; 0 at 0."""
    _, e = np.frexp(np.abs(x))
    return np.where(x == 0, 0.0, np.ldexp(1.0, e - 8))


def gpu_acts(net, B):
    """The GPU's last forward pass: layer inputs with halo (FP64 copies of the
    BF16 values; the network input's 3 used channels) and delta."""
    acts = [net.activation(0, B).float().cpu().numpy().astype(np.float64)[..., :3]]
    acts += [net.activation(l, B).float().cpu().numpy().astype(np.float64) for l in range(1, 6)]
    return acts, net.activation(6, B).cpu().numpy().astype(np.float64)[..., :3]


@pytest.mark.parametrize("B,H,W,cap", [(2, 48, 64, 0), (3, 22, 128, 0), (2, 48, 64, 3)])
def test_forward_layers_match_oracle(B, H, W, cap):
    """Every layer against the oracle fed the GPU's own BF16 input of that
    layer: a BF16 output within 1 BF16 ulp of the oracle's rounded value,
    plus the FP32 accumulation bound gamma(9 cin + 1) * sum|terms| where that
    exceeds it; the FP32 output layer within that accumulation bound and
    within 1e-5 of its largest value.  H = 22 leaves a partial tile of output
    rows; a cap of 3 blocks makes every conv block walk several tiles."""
    p = no.init_params(11, out_gain=1.0)
    layers = no.unpack(p)
    out_scale = (0.05, 0.05, 0.05)
    u = states(B, H, W, 21)
    announce(f"surrogate forward parity B={B} {H}x{W} cap={cap}")
    net = make_net(H, W, B, p, out_scale)
    net.set_block_cap(cap)
    net.forward(u)
    acts, delta = gpu_acts(net, B)
    ref0 = no.input_tensor(u.cpu().numpy(), OFF, SCALE)
    x0 = net.activation(0, B).float().cpu().numpy()
    assert np.array_equal(x0[..., :3], ref0) and not np.any(x0[..., 3:])
    for l in range(6):
        w, b = no.bf16(layers[l][0]), layers[l][1]
        a_in = acts[l]
        z = no.conv3x3(a_in, w, b)
        S = no.conv3x3(np.abs(a_in), np.abs(w), np.abs(b))
        acc = gamma(9 * w.shape[2] + 1) * S
        if l == 5:
            err = np.abs(delta - z)
            print(f"output layer: max err {err.max() / np.abs(z).max():.2e} of max|z|, "
                  f"{np.max(err / acc):.2e} of the accumulation bound")
            assert np.all(err <= acc)
            assert err.max() <= 1e-5 * np.abs(z).max()
            continue
        y = np.maximum(z, 0.0)
        if no.residual(l):
            y = y + a_in[:, 1:-1, 1:-1]
        ref = no.bf16(y)
        got = acts[l + 1][:, 1:-1, 1:-1]
        err = np.abs(got - ref)
        ulp = ulp_bf16(np.maximum(np.abs(got), np.abs(ref)))
        beyond_1ulp = int(np.sum(err > ulp))
        print(f"layer {l + 1}: differ {np.mean(err > 0):.2e}, beyond 1 ulp {beyond_1ulp}, "
              f"max err/(ulp + bound) {np.max(err / (ulp + acc + U32 * np.abs(y))):.2e}")
        assert np.all(err <= ulp + acc + U32 * np.abs(y)), l
        halo = acts[l + 1].copy()
        halo[:, 1:-1, 1:-1] = 0.0
        assert not np.any(halo)                   # zero padding of the hidden layers
    # the oracle's own forward pass from the input (BF16 differences compound
    # through the layers): within 1e-2 of the output scale, 1e-4 on average
    _, chained = no.forward(p, u.cpu().numpy(), OFF, SCALE, bf16_mode=True)
    scale = np.max(np.abs(chained))
    err = np.abs(delta - chained)
    print(f"chained delta: max {err.max() / scale:.2e}, mean {err.mean() / scale:.2e}")
    assert err.max() <= 1e-2 * scale and err.mean() <= 1e-4 * scale


def grad_case(B, H, W, seed):
    p = no.init_params(seed, out_gain=1.0)
    out_scale = (0.02, 0.03, 0.03)
    u = states(B, H, W, 31 + seed)
    u8 = u + 0.01 * torch.randn(u.shape, generator=torch.Generator().manual_seed(seed)).cuda()
    return p, out_scale, u, u8


def oracle_grad_from_gpu_forward(net, p, B, u, u8, out_scale):
    """The oracle's backward pass fed the GPU's forward pass (activations,
    delta) and masks Z > 0 recomputed in FP64 from the GPU's layer inputs."""
    layers = no.unpack(p)
    acts, delta = gpu_acts(net, B)
    masks = [no.conv3x3(acts[l], no.bf16(layers[l][0]), layers[l][1]) > 0.0 for l in range(5)]
    tgt = no.target_of(u.cpu().numpy(), u8.cpu().numpy(), out_scale)
    return no.backward(p, acts, masks, delta, tgt, bf16_mode=True, abs_sums=True)


# Element-wise bound of a gradient entry: |gpu - oracle| <= KAPPA * S, with S
# the entry's sum of |terms| (sum_p |dZ| |A|).  The operands are the same BF16
# values on both sides up to single-ulp rounding differences of the stored
# intermediate gradients (FP32 vs FP64 sums rounded to BF16), so each term of
# the sum is off by at most one BF16 ulp (2^-8 relative) and only for the few
# operands whose sums straddle a rounding boundary; 2^-9 S is the error if
# every term were off by half an ulp, and the FP32 accumulation adds
# gamma(pixels) S.
KAPPA_FROM_GPU_FORWARD = 2.0 ** -9
# The oracle's own chain (forward included) also takes every ReLU decision
# itself: where a pre-activation lies within rounding of zero the two sides
# may keep or drop a whole term of a later sum, which no per-term rounding
# bound covers.  Its comparison is therefore held to the same bound on 99 %
# of the entries and to 1e-2 normwise per layer; the element-wise gate is
# the comparison above, fed the GPU's own forward pass.
KAPPA_CHAINED = 2.0 ** -8


def check_grad_chained(g, ref, S, npix):
    bound = (KAPPA_CHAINED + gamma(npix)) * S
    err = np.abs(g - ref)
    within = np.mean(err <= bound)
    print(f"chained: {within:.4f} of the entries within (2^-8 + gamma) S")
    assert within >= 0.99
    off = 0
    for l, (ci, co) in enumerate(no.LAYERS):
        n = co * 9 * ci + co
        a, r = g[off:off + n], ref[off:off + n]
        rel = np.linalg.norm(a - r) / np.linalg.norm(r)
        print(f"chained layer {l + 1}: normwise {rel:.2e}")
        assert rel <= 1e-2, (l, rel)
        off += n


def check_grad(g, ref, S, kappa, npix, what):
    bound = (kappa + gamma(npix)) * S
    err = np.abs(g - ref)
    r = err / np.maximum(S, 1e-300)
    print(f"{what}: max err/S {np.max(r):.2e}, "
          f"max err/bound {np.max(err / np.maximum(bound, 1e-300)):.2e}, "
          f"normwise {np.linalg.norm(err) / np.linalg.norm(ref):.2e}, "
          f"err/S quantiles 50/90/99/99.9 % {np.quantile(r, [0.5, 0.9, 0.99, 0.999])}")
    bad = np.flatnonzero(err > bound)
    if bad.size:
        order = bad[np.argsort(-r[bad])][:12]
        print(f"{what}: {bad.size} entries beyond the bound; worst: idx {order.tolist()}\n gpu {g[order]}\n "
              f"ref {ref[order]}\n S {S[order]}")
    assert bad.size == 0, (what, bad[:10], g[bad[:10]], ref[bad[:10]], S[bad[:10]])
    assert np.linalg.norm(err) <= 1e-2 * np.linalg.norm(ref)


@pytest.mark.parametrize("B,H,W,cap", [(2, 40, 64, 0), (2, 40, 64, 1), (2, 40, 64, 3), (3, 22, 128, 2)])
def test_gradient_matches_oracle_elementwise(B, H, W, cap):
    """Every entry of the loss gradient against the oracle: (a) element by
    element, the oracle's backward pass fed the GPU's forward pass (the same
    BF16 operands); (b) the oracle's whole chain from the input, on 99 % of
    the entries and normwise per layer.  Caps of 1-3 blocks make each
    weight-gradient and input-gradient block walk 7-20 tiles (the persistent,
    double-buffered multi-tile loop that runs at full size); H = 22 leaves a
    partial tile."""
    p, out_scale, u, u8 = grad_case(B, H, W, 12)
    announce(f"surrogate gradient parity B={B} {H}x{W} cap={cap}")
    net = make_net(H, W, B, p, out_scale)
    net.set_block_cap(cap)
    g, loss = net.grad(u, u8)
    g = g.cpu().numpy().astype(np.float64)
    loss = float(loss[0])
    la, ra, Sa = oracle_grad_from_gpu_forward(net, p, B, u, u8, out_scale)
    assert abs(loss - la) <= 1e-5 * la
    check_grad(g, ra, Sa, KAPPA_FROM_GPU_FORWARD, B * H * W, "from the GPU forward")
    lb, rb, Sb = no.loss_and_grad(p, u.cpu().numpy(), u8.cpu().numpy(), OFF, SCALE, out_scale,
                                  bf16_mode=True, abs_sums=True)
    assert abs(loss - lb) <= 1e-4 * lb
    check_grad_chained(g, rb, Sb, B * H * W)


def test_block_cap_keeps_forward_bits():
    """The cap only changes which block walks which tiles: every activation
    and the output are bitwise those of the uncapped launch."""
    B, H, W = 2, 48, 128
    p = no.init_params(13, out_gain=1.0)
    u = states(B, H, W, 23)
    net = make_net(H, W, B, p, (0.05, 0.05, 0.05))
    outs = []
    for cap in (0, 1, 5):
        net.set_block_cap(cap)
        d = net.forward(u).clone()
        outs.append([d] + [net.activation(l, B).clone() for l in range(6)])
    for other in outs[1:]:
        assert all(torch.equal(a, b) for a, b in zip(outs[0], other))
    with pytest.raises(sw.SwError):
        net.set_block_cap(-1)
    with pytest.raises(sw.SwError):
        net.set_block_cap(1025)


def test_adam_steps_match_oracle():
    """Three sw_surrogate_train_step calls against the oracle's FP64 Adam
    (Kingma and Ba 2015) applied to the same gradients (the GPU's own,
    taken by sw_surrogate_grad at the same parameters just before each
    step; the gradient is deterministic): the FP32 master weights after each
    step within the FP32 rounding of the update (2^-22 of the weight plus
    1e-5 of the learning rate)."""
    B, H, W = 2, 40, 64
    p, out_scale, u, u8 = grad_case(B, H, W, 14)
    announce("surrogate Adam steps")
    net = make_net(H, W, B, p, out_scale)
    lr = 3e-3
    theta = net.get_params().cpu().numpy().astype(np.float64)
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    for t in range(1, 4):
        ut = u + 0.002 * t
        g, _ = net.grad(ut, u8)
        g = g.cpu().numpy().astype(np.float64)
        g_again, _ = net.grad(ut, u8)
        assert np.array_equal(g, g_again.cpu().numpy())
        net.train_step(ut, u8, lr)
        got = net.get_params().cpu().numpy().astype(np.float64)
        theta, m, v = no.adam_step(theta, m, v, g, t, lr)
        err = np.abs(got - theta)
        bound = 2.0 ** -22 * np.abs(theta) + 1e-5 * lr
        print(f"Adam step {t}: max err/bound {np.max(err / bound):.2e}")
        assert np.all(err <= bound), (t, np.flatnonzero(err > bound)[:10])
        theta = got
    # the forward pass now runs on the updated weights (BF16 copies refreshed)
    net.forward(u)
    acts, _ = gpu_acts(net, B)
    w1, b1 = no.unpack(theta)[0]
    w1 = no.bf16(w1)
    z1 = no.conv3x3(acts[0], w1, b1)
    bound = gamma(28) * no.conv3x3(np.abs(acts[0]), np.abs(w1), np.abs(b1)) + U32 * np.abs(z1)
    ref = no.bf16(np.maximum(z1, 0.0))
    got = acts[1][:, 1:-1, 1:-1]
    assert np.all(np.abs(got - ref) <= ulp_bf16(np.maximum(np.abs(got), np.abs(ref))) + bound)


def test_train_step_matches_oracle_chain():
    """One whole training step (forward, loss, backward, Adam, BF16 weight
    copies) against the oracle's gradient followed by the oracle's Adam step.
    The first Adam step moves each weight by -lr g / (|g| + eps), so a
    gradient entry known to within e moves the weight to within
    lr min(2, 2 e / (|g| + eps)) (2 where the sign of a gradient entry that
    small is not determined); e is the chained gradient bound."""
    B, H, W = 2, 40, 64
    p, out_scale, u, u8 = grad_case(B, H, W, 15)
    announce("surrogate train step vs oracle chain")
    net = make_net(H, W, B, p, out_scale)
    p32 = net.get_params().cpu().numpy().astype(np.float64)
    lr = 1e-3
    net.train_step(u, u8, lr)
    got = net.get_params().cpu().numpy().astype(np.float64)
    _, g_ref, S = no.loss_and_grad(p32, u.cpu().numpy(), u8.cpu().numpy(), OFF, SCALE, out_scale,
                                   bf16_mode=True, abs_sums=True)
    want, _, _ = no.adam_step(p32, np.zeros_like(p32), np.zeros_like(p32), g_ref, 1, lr)
    e = (KAPPA_CHAINED + gamma(B * H * W)) * S
    bound = lr * np.minimum(2.0, 2.0 * e / (np.abs(g_ref) + 1e-8)) + 2.0 ** -22 * np.abs(want) + 1e-5 * lr
    err = np.abs(got - want)
    determined = np.abs(g_ref) > 4 * e
    print(f"train step: max err/bound {np.max(err / bound):.2e}; {np.mean(determined):.3f} of the entries "
          f"have a determined sign, max err there {np.max(err[determined]) / lr:.2e} lr")
    assert np.all(err <= bound)
    assert np.mean(determined) > 0.5


def test_export_import_roundtrip():
    u = states(3, 40, 64, 5)
    b = sw.Batch([(64, 40)] * 3, dtype="f32")
    b.load(u)
    assert torch.equal(b.export(), u)
    for k in range(3):
        h, hu, hv = b.get_state(k)
        assert torch.equal(h, u[k, 0].cpu().double())


@pytest.mark.parametrize("fault", ["nan_hv", "mass_drift", "dry_cell"])
def test_forced_fallback_equals_solver(fault):
    """A network that fails every gate leaves the plain solver's result,
    bitwise, and every jump is counted as a fallback.  Each case trips one
    check: a NaN hv output (the last bias of the output layer; a NaN in a
    hidden layer would not do, since ReLU maps it to zero) only the
    non-finite check sees; a constant dh with the mass projection off only
    the mass-drift check; a large negative dh with the projection on (mass
    kept) only the positivity check."""
    n, H, W = 4, 64, 64
    u0 = states(n, H, W, 41)
    net = sw.Surrogate(H, W, n, jump=8, seed=3)
    p = net.get_params()
    gate = {}
    if fault == "nan_hv":
        p[-1] = float("nan")
    elif fault == "mass_drift":
        p[-3] += 1.0
        gate = dict(project_mass=False)
    else:
        # dh swings far beyond the depth; the projection removes its mean,
        # so the mass is kept and only negative depths are left to reject
        w6 = p[-3 - 3 * 9 * 32:-3].view(3, 9, 32)
        w6[0] *= 1.0e4
        gate = dict(project_mass=True, mass_rel_tol=1.0)
    net.set_params(p)
    got, fb, _ = surrogate.rollout(net, u0, 24, gate)
    ref, _ = surrogate.solver_run(u0, 24)
    assert torch.equal(got, ref)
    assert fb.tolist() == [3] * n


def test_judge_rejects_to_the_solver():
    """Judge mode with a bound no rollout meets: every grid ends with the plain
    solver's state (bitwise), step count, unstable flag (clear, although the
    untrained network's states may have tripped a fallback step) and a full
    fallback count; the reported L2 is the rollout's error before the
    replacement."""
    n, H, W, nsteps = 3, 64, 64, 24
    u0 = states(n, H, W, 51)
    net = sw.Surrogate(H, W, n, jump=8, seed=4)
    l2 = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    b = sw.Batch([(W, H)] * n, dtype="f32")
    got, fb, _ = surrogate.rollout(net, u0, nsteps, dict(judge=True, l2_tol=1e-9), l2=l2, batch=b)
    ref, _ = surrogate.solver_run(u0, nsteps)
    assert torch.equal(got, ref)
    assert fb.tolist() == [nsteps // 8] * n
    assert bool((l2 > 1e-9).all()) and bool(torch.isfinite(l2).all())
    _, steps, _ = b.sync_status()
    assert list(steps) == [nsteps] * n


def test_judge_keeps_accepted_rollouts():
    """A loose bound changes nothing: the judged rollout equals the unjudged
    one bitwise, and the reported L2 equals ||h - h_solver|| / ||h_solver||."""
    n, H, W, nsteps = 3, 64, 64, 16
    u0 = states(n, H, W, 61)
    net = sw.Surrogate(H, W, n, jump=8, seed=4)
    plain, fb0, _ = surrogate.rollout(net, u0, nsteps)
    l2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    judged, fb1, _ = surrogate.rollout(net, u0, nsteps, dict(judge=True, l2_tol=10.0), l2=l2)
    assert torch.equal(plain, judged) and torch.equal(fb0, fb1)
    ref, _ = surrogate.solver_run(u0, nsteps)
    d = (plain[:, 0].double() - ref[:, 0].double()).flatten(1).norm(dim=1)
    want = d / ref[:, 0].double().flatten(1).norm(dim=1)
    torch.testing.assert_close(l2, want, rtol=1e-9, atol=0)
    with pytest.raises(RuntimeError):
        net.advance(sw.Batch([(W, H)] * n, dtype="f32"), 8, judge=True, l2_tol=-1.0)


def test_training_gains_over_untrained_and_persistence():
    """Train on solver trajectories (64 x 64 grids), then roll out 64 steps
    on held-out initial states: the trained network is several times closer
    to the plain solver than the untrained one and than persistence
    (U^{n+8} := U^n), with relative L2(h) <= 1e-2 on average."""
    H = W = 64
    jump, frames = 8, 64
    announce("surrogate training")
    data = surrogate.trajectories(64, H, W, frames, seed0=70000)
    out_scale = surrogate.fit_out_scale(data, jump)
    net = sw.Surrogate(H, W, 64, jump=jump, seed=5)
    net.set_norm(OFF, SCALE, out_scale)
    untrained = net.get_params().clone()
    losses = surrogate.train(net, data, steps=6000, B=64, lr=1e-3, jump=jump, seed=1, lr_final=5e-5)
    first, last = float(losses[:20].mean()), float(losses[-20:].mean())
    print(f"loss {first:.3e} -> {last:.3e}")
    assert last < 0.3 * first
    u0 = surrogate.initial_states(16, H, W, 90000)
    ref, _ = surrogate.solver_run(u0, 64)
    gate = dict(mass_rel_tol=1e-4, project_mass=True)
    trained, fb_t, _ = surrogate.rollout(net, u0, 64, gate)
    e_trained = surrogate.rel_l2_h(trained[:, 0], ref[:, 0])
    net.set_params(untrained)
    untr, fb_u, _ = surrogate.rollout(net, u0, 64, gate)
    e_untr = surrogate.rel_l2_h(untr[:, 0], ref[:, 0])
    e_pers = surrogate.rel_l2_h(u0[:, 0], ref[:, 0])
    print(f"rel L2(h): trained {e_trained[0].mean():.2e} (fallbacks {int(fb_t.sum())}), "
          f"untrained {e_untr[0].mean():.2e} (fallbacks {int(fb_u.sum())}), persistence {e_pers[0].mean():.2e}; "
          f"strict: trained {e_trained[1].mean():.2e}, persistence {e_pers[1].mean():.2e}")
    assert e_trained[0].mean() < 0.25 * e_pers[0].mean() and e_trained[0].mean() < 0.25 * e_untr[0].mean()
    assert e_trained[1].mean() < 0.25 * e_pers[1].mean()
    assert e_trained[0].mean() <= 1e-2 and float(e_trained[0].max()) <= 2e-2


def test_committed_weights_gain_at_256():
    """The committed 256 x 256 network on 16 held-out states (seeds disjoint
    from its training trajectories): 64 gated steps land within relative
    L2(h) 1e-2 of the plain solver on average and several times closer than
    persistence; in judge mode with bound 1e-2 every grid ends within the
    bound (rejected grids carry the solver's state)."""
    announce("committed surrogate weights, 16 held-out 256x256 grids")
    n, size = 16, 256
    net, meta = surrogate.load_weights(surrogate.WEIGHTS_256, n)
    assert meta["recipe"]["H"] == size and meta["recipe"]["jump"] == 8
    u0 = surrogate.initial_states(n, size, size, ics.SEED_SURR_EVAL0 + 1000)
    ref, _ = surrogate.solver_run(u0, 64)
    got, fb, _ = surrogate.rollout(net, u0, 64, dict(mass_rel_tol=1e-4, project_mass=True))
    e, _ = surrogate.rel_l2_h(got[:, 0], ref[:, 0])
    p, _ = surrogate.rel_l2_h(u0[:, 0], ref[:, 0])
    print(f"rel L2(h): mean {e.mean():.2e} max {e.max():.2e}, persistence {p.mean():.2e}, fallbacks {int(fb.sum())}")
    assert e.mean() <= 1e-2 and e.mean() < 0.25 * p.mean()
    l2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    judged, _, _ = surrogate.rollout(net, u0, 64, dict(mass_rel_tol=1e-4, project_mass=True, judge=True, l2_tol=1e-2),
                                     l2=l2)
    ej, _ = surrogate.rel_l2_h(judged[:, 0], ref[:, 0])
    assert bool((ej <= 1e-2).all())
    torch.testing.assert_close(l2.cpu(), e.cpu(), rtol=1e-6, atol=1e-12)


def test_binding_rejects_mismatched_tensors():
    """Wrong shapes, host tensors and oversize batches are refused before any
    kernel runs (a kernel would read or write past the tensor's end)."""
    net = sw.Surrogate(64, 64, 2, jump=8, seed=1)
    with pytest.raises(ValueError):
        net.forward(torch.zeros(2, 3, 64, 48, device="cuda"))
    with pytest.raises(ValueError):
        net.forward(torch.zeros(3, 3, 64, 64))
    with pytest.raises(ValueError):
        net.train_step(torch.zeros(2, 3, 64, 64, device="cuda"), torch.zeros(2, 3, 32, 64, device="cuda"), 1e-3)
    with pytest.raises(ValueError):
        net.activation(1, 3)
    b = sw.Batch([(64, 40)] * 2, dtype="f32")
    with pytest.raises(ValueError):
        b.export(torch.zeros(2, 3, 40, 63, device="cuda"))
    with pytest.raises(ValueError):
        b.load(torch.zeros(2, 3, 40, 64))
    with pytest.raises(ValueError):
        b.load(torch.zeros(1, 3, 40, 64, device="cuda"))


def _rollout_runs(net, b, u0, nsteps, gate, graph, reps):
    """reps rollouts from u0 (time and step counters cleared) through one
    fallbacks array: (state, fallbacks, solver steps taken, simulated time)
    of each, with eager work (a forward pass, copies) and synchronisations
    between the calls."""
    net.set_graph(graph)
    fb = torch.zeros(b.n, dtype=torch.int32, device="cuda")
    out = []
    for _ in range(reps):
        b.load(u0)
        b.reset_time()
        fb.zero_()
        net.advance(b, nsteps, fallbacks=fb, **gate)
        state = b.export()
        t, steps, _ = b.sync_status()
        out.append((state, fb.clone(), list(steps), list(t)))
        net.forward(u0)
        torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("case", ["accepted", "rejected"])
def test_graph_replays_equal_eager_rollouts(case):
    """Unjudged rollouts are captured into a hipGraph on the first call and
    replayed afterwards; every replay gives bitwise the eager rollout's
    state, fallback counts, solver step counts and time, both when the
    network's jumps are accepted (trained weights) and when every jump is
    rejected (a forced mass drift), so that the masked solver steps run
    inside the graph."""
    if case == "accepted":
        n, nsteps = 2, 32
        net, _ = surrogate.load_weights(surrogate.WEIGHTS_256, n)
        u0 = surrogate.initial_states(n, 256, 256, ics.SEED_SURR_EVAL0)
        gate = dict(mass_rel_tol=1e-4, project_mass=True)
    else:
        n, nsteps = 3, 24
        u0 = states(n, 64, 64, 71)
        net = sw.Surrogate(64, 64, n, jump=8, seed=3)
        p = net.get_params()
        p[-3] += 1.0
        net.set_params(p)
        gate = dict(project_mass=False)
    H, W = u0.shape[2], u0.shape[3]
    announce(f"surrogate graph replays {case}")
    b = sw.Batch([(W, H)] * n, dtype="f32")
    (ref, fb_ref, steps_ref, t_ref), = _rollout_runs(net, b, u0, nsteps, gate, graph=False, reps=1)
    assert fb_ref.tolist() == ([0] * n if case == "accepted" else [nsteps // 8] * n)
    assert steps_ref == ([0] * n if case == "accepted" else [nsteps] * n)
    for state, fb, steps, t in _rollout_runs(net, b, u0, nsteps, gate, graph=True, reps=4):
        assert torch.equal(state, ref)
        assert torch.equal(fb, fb_ref) and steps == steps_ref and t == t_ref


def test_set_norm_drops_captured_rollouts():
    """The normalisation is baked into a captured rollout by value: after
    set_norm the next rollout is captured anew and equals the eager rollout
    under the new normalisation."""
    n, H, W, nsteps = 2, 64, 64, 16
    u0 = states(n, H, W, 81)
    net = sw.Surrogate(H, W, n, jump=8, seed=2)
    b = sw.Batch([(W, H)] * n, dtype="f32")
    gate = dict(mass_rel_tol=10.0, project_mass=True)
    net.set_norm(OFF, SCALE, (0.01, 0.01, 0.01))
    (a_graph, *_), = _rollout_runs(net, b, u0, nsteps, gate, graph=True, reps=1)
    net.set_norm(OFF, SCALE, (0.03, 0.02, 0.02))
    (b_graph, *_), = _rollout_runs(net, b, u0, nsteps, gate, graph=True, reps=1)
    (b_eager, *_), = _rollout_runs(net, b, u0, nsteps, gate, graph=False, reps=1)
    assert torch.equal(b_graph, b_eager)
    assert not torch.equal(a_graph, b_graph)


def _advance_both(net, u0, nsteps, gate):
    """The same rollout with the fused network launch and with the per-layer
    kernels: (state, fallbacks, last delta) of each."""
    out = []
    for fused in (True, False):
        net.set_fused(fused)
        state, fb, _ = surrogate.rollout(net, u0, nsteps, gate)
        out.append((state, fb, net.activation(6, u0.shape[0]).clone()))
    net.set_fused(surrogate.DEFAULT_FORM)
    return out


@pytest.mark.parametrize("n,H,W,cap", [(3, 40, 64, 0), (2, 37, 128, 0), (4, 256, 256, 0), (3, 40, 64, 2)])
def test_fused_rollout_equals_per_layer(n, H, W, cap):
    """The rollout's fused network launch (all six layers per tile in LDS,
    the border recomputed) against the per-layer kernels: the prediction of
    the last jump and, with the mass projection off, every grid's state
    after two jumps are bitwise equal; with the projection on, the mean dh is
    summed per tile instead of per row segment, so hu and hv stay bitwise
    and h agrees to float rounding.  Shapes cover ragged bottom tiles (37 and
    40 rows), both tile widths (16 x 32 where a batch has two such tiles per
    CU: 4 grids of 256^2) and a capped persistent grid (each workgroup walks
    several tiles)."""
    announce(f"fused rollout n={n} {H}x{W} cap={cap}")
    u0 = states(n, H, W, 61)
    net = sw.Surrogate(H, W, n, jump=8, seed=4)
    net.set_norm(OFF, SCALE, (0.02, 0.02, 0.02))
    if cap:
        net.set_block_cap(cap)
    accept = dict(mass_rel_tol=10.0, hmin=-1.0e30)
    (a, fa, da), (b, fb, db) = _advance_both(net, u0, 16, dict(accept, project_mass=False))
    assert fa.tolist() == fb.tolist() == [0] * n
    assert torch.equal(da, db)
    assert torch.equal(a, b)
    (a, fa, da), (b, fb, db) = _advance_both(net, u0, 16, dict(accept, project_mass=True))
    assert torch.equal(da, db)
    assert torch.equal(a[:, 1:], b[:, 1:])
    assert torch.max(torch.abs(a[:, 0] - b[:, 0])).item() <= 4 * 2.0 ** -23 * torch.max(torch.abs(b[:, 0])).item()


def test_fused_rollout_mixed_verdicts_equal_per_layer():
    """A batch where the gate rejects some grids and accepts the others (a
    depth threshold between the grids' depths): the fused path (gate verdict
    and the rejected grids' solver steps in one launch) leaves bitwise the
    per-layer path's states and fallback counts, and the rejected grids hold
    the plain solver's result."""
    n, H, W = 4, 48, 64
    u0 = states(n, H, W, 67)
    for k in (1, 3):                  # grids 1 and 3 sit below the threshold: depth at most 0.5
        u0[k] *= 0.5 / u0[k, 0].max()
    announce("fused rollout, mixed verdicts")
    net = sw.Surrogate(H, W, n, jump=8, seed=5)
    net.set_norm(OFF, SCALE, (0.02, 0.02, 0.02))
    gate = dict(mass_rel_tol=10.0, hmin=0.75, project_mass=True)
    (a, fa, _), (b, fb, _) = _advance_both(net, u0, 16, gate)
    assert fa.tolist() == fb.tolist() == [0, 2, 0, 2]
    assert torch.equal(a, b)
    ref, _ = surrogate.solver_run(u0, 16, tune_cache=None)
    assert torch.equal(a[1], ref[1]) and torch.equal(a[3], ref[3])
