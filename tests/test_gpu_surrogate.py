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


@pytest.mark.parametrize("B,H,W", [(2, 48, 64), (3, 22, 128)])
def test_forward_matches_oracle(B, H, W):
    """H = 22 leaves a partial tile of output rows."""
    p = no.init_params(11, out_gain=1.0)
    out_scale = (0.05, 0.05, 0.05)
    u = states(B, H, W, 21)
    announce("surrogate forward parity")
    net = make_net(H, W, B, p, out_scale)
    delta = net.forward(u).cpu().numpy()
    acts, ref_delta = no.forward(p, u.cpu().numpy(), OFF, SCALE, bf16_mode=True)
    x0 = net.activation(0, B).float().cpu().numpy()
    assert np.array_equal(x0[..., :3], acts[0]) and not np.any(x0[..., 3:])
    for l in range(1, 6):
        got = net.activation(l, B).float().cpu().numpy()
        ref = acts[l]
        mism = np.mean(got != ref)
        rel = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"layer {l}: mismatch fraction {mism:.2e}, max rel {rel:.2e}")
        assert mism < 2e-3 and rel < 2e-2
    scale = np.max(np.abs(ref_delta))
    err = np.abs(delta[..., :3] - ref_delta)
    print(f"delta: max {err.max() / scale:.2e}, mean {err.mean() / scale:.2e}")
    assert err.max() <= 1e-2 * scale and err.mean() <= 1e-4 * scale
    assert not np.any(delta[..., 3])


def test_gradient_matches_oracle():
    B, H, W = 2, 40, 64
    p = no.init_params(12, out_gain=1.0)
    out_scale = (0.02, 0.03, 0.03)
    u = states(B, H, W, 31)
    u8 = u + 0.01 * torch.randn_like(u)
    announce("surrogate gradient parity")
    net = make_net(H, W, B, p, out_scale)
    g, loss = net.grad(u, u8)
    g = g.cpu().numpy().astype(np.float64)
    ref_loss, ref = no.loss_and_grad(p, u.cpu().numpy(), u8.cpu().numpy(), OFF, SCALE, out_scale, bf16_mode=True)
    assert abs(float(loss[0]) - ref_loss) <= 1e-4 * ref_loss
    off = 0
    for l, (ci, co) in enumerate(no.LAYERS):
        for name, cnt in (("W", co * 9 * ci), ("b", co)):
            a, r = g[off:off + cnt], ref[off:off + cnt]
            rel = np.linalg.norm(a - r) / np.linalg.norm(r)
            print(f"layer {l + 1} {name}: rel {rel:.2e}")
            assert rel <= 2e-2, (l, name, rel)
            off += cnt


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
