"""Train the learned surrogate on trajectories of the library's own solver.

    python -m paper_1107_2157_amd.train_surrogate [--steps N] [--out PATH]

Default recipe (the 256 x 256 surrogate workload): 2000 trajectories of 64
frames (states after 0..63 solver steps) from seeded Gaussian-bump states
(seeds ``ics.SEED_TRAJ0 + k``, 1-8 bumps, reflective walls, FP32, CFL 0.5),
held on the GPU (about 100 GB); training pairs (U^t, U^{t+8}); Adam with
batch 256 and a cosine learning rate 1e-3 -> 5e-5; evaluation: 64-step gated
rollouts (mass tolerance 1e-4 with projection) of 256 held-out states (seeds
``ics.SEED_SURR_EVAL0 + k``) against the plain solver, relative L2 of h.
Writes the FP32 master parameters, the normalisation and the recipe with its
results to an .npz.
"""
from __future__ import annotations

import argparse
import time

import torch

from . import ics, surrogate, sw


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--grids", type=int, default=2000)
    ap.add_argument("--frames", type=int, default=64)
    ap.add_argument("--size", type=int, default=256, help="H = W")
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--steps", type=int, default=6000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--lr-final", type=float, default=5e-5)
    ap.add_argument("--jump", type=int, default=8)
    ap.add_argument("--seed", type=int, default=5, help="weight initialisation")
    ap.add_argument("--eval", type=int, default=256, help="held-out grids")
    ap.add_argument("--out", default=surrogate.WEIGHTS_256)
    args = ap.parse_args(argv)
    H = W = args.size
    t0 = time.perf_counter()
    data = surrogate.trajectories(args.grids, H, W, args.frames)
    out_scale = surrogate.fit_out_scale(data, args.jump)
    print(f"[train_surrogate] {args.grids} trajectories x {args.frames} frames of {H}x{W} "
          f"({data.numel() * 4 / 1e9:.1f} GB) in {time.perf_counter() - t0:.1f} s; out_scale {out_scale}", flush=True)
    net = sw.Surrogate(H, W, args.batch, jump=args.jump, seed=args.seed)
    net.set_norm(surrogate.IN_OFFSET, surrogate.IN_SCALE, out_scale)
    t1 = time.perf_counter()
    losses = surrogate.train(net, data, steps=args.steps, B=args.batch, lr=args.lr, jump=args.jump, seed=1,
                             lr_final=args.lr_final, log_every=max(args.steps // 40, 1))
    train_s = time.perf_counter() - t1
    del data
    torch.cuda.empty_cache()
    # held-out evaluation with the deployed gate
    u0 = surrogate.initial_states(args.eval, H, W, ics.SEED_SURR_EVAL0)
    ref, _ = surrogate.solver_run(u0, 64)
    evalnet = sw.Surrogate(H, W, args.eval, jump=args.jump, seed=0)
    evalnet.set_params(net.get_params())
    evalnet.set_norm(surrogate.IN_OFFSET, surrogate.IN_SCALE, out_scale)
    got, fb, _ = surrogate.rollout(evalnet, u0, 64, dict(mass_rel_tol=1e-4, project_mass=True))
    e, e_strict = surrogate.rel_l2_h(got[:, 0], ref[:, 0])
    p, p_strict = surrogate.rel_l2_h(u0[:, 0], ref[:, 0])
    meta = dict(recipe=dict(grids=args.grids, frames=args.frames, H=H, W=W, batch=args.batch, steps=args.steps,
                            lr=args.lr, lr_final=args.lr_final, jump=args.jump, init_seed=args.seed,
                            traj_seed0=ics.SEED_TRAJ0, bc="reflect", dtype="f32", cfl=0.5),
                loss_first=float(losses[:50].mean()), loss_last=float(losses[-50:].mean()),
                train_seconds=round(train_s, 1), train_steps_per_s=round(args.steps / train_s, 2),
                eval=dict(grids=args.eval, seed0=ics.SEED_SURR_EVAL0, steps=64,
                          rel_l2_h_mean=float(e.mean()), rel_l2_h_max=float(e.max()),
                          rel_l2_h_strict_mean=float(e_strict.mean()), persistence_mean=float(p.mean()),
                          fallbacks=int(fb.sum())))
    surrogate.save_weights(args.out, net, surrogate.IN_OFFSET, surrogate.IN_SCALE, out_scale, meta)
    print(f"[train_surrogate] loss {meta['loss_first']:.3e} -> {meta['loss_last']:.3e} in {train_s:.0f} s "
          f"({meta['train_steps_per_s']} steps/s); held-out rel L2(h) at step 64: mean {e.mean():.2e} "
          f"max {e.max():.2e} (persistence {p.mean():.2e}), fallbacks {int(fb.sum())}; wrote {args.out}", flush=True)


if __name__ == "__main__":
    main()
