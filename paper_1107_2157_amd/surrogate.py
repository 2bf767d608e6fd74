"""Training data, training loop and evaluation of the learned surrogate.

Orchestration only: trajectories come from the library's batched solver,
training steps and rollouts are library calls (``sw.Surrogate``); torch is
used to hold tensors and to pick random training pairs.

Workload (the surrogate configuration): H x W grids with reflective walls,
initial states of 1-8 seeded Gaussian bumps (seeds ``ics.SEED_TRAJ0 + k``),
trajectories of ``frames`` states (after 0 .. frames-1 solver steps), training
pairs ``(U^t, U^{t+jump})`` for every ``t <= frames - 1 - jump``.
"""
from __future__ import annotations

import json
import math
import os
import time

import numpy as np
import torch

from . import ics, sw

IN_OFFSET = (1.0, 0.0, 0.0)
IN_SCALE = (0.25, 0.25 * math.sqrt(9.8), 0.25 * math.sqrt(9.8))


def initial_states(n: int, H: int, W: int, seed0: int, periodic: bool = False, device="cuda") -> torch.Tensor:
    """Dense [n][3][H][W] FP32 bump states."""
    out = torch.empty((n, 3, H, W), dtype=torch.float32, device=device)
    for k in range(n):
        h, hu, hv = ics.bumps_state(W, H, seed=seed0 + k, periodic=periodic, device=device)
        out[k, 0], out[k, 1], out[k, 2] = h, hu, hv
    return out


def trajectories(n: int, H: int, W: int, frames: int, seed0: int = ics.SEED_TRAJ0, chunk: int = 256,
                 bc: int = sw.REFLECT) -> torch.Tensor:
    """Solver trajectories as a dense [frames][n][3][H][W] FP32 device tensor."""
    out = torch.empty((frames, n, 3, H, W), dtype=torch.float32, device="cuda")
    for c0 in range(0, n, chunk):
        m = min(chunk, n - c0)
        b = sw.Batch([(W, H)] * m, dtype="f32", bc_x=bc, bc_y=bc)
        b.load(initial_states(m, H, W, seed0 + c0, periodic=bc == sw.PERIODIC))
        b.export(out[0, c0:c0 + m])
        for t in range(1, frames):
            b.step(1)
            b.export(out[t, c0:c0 + m])
        b.sync_status()
        del b
    torch.cuda.synchronize()
    return out


def fit_out_scale(data: torch.Tensor, jump: int) -> tuple:
    """RMS of U^{t+jump} - U^t per channel over the trajectories."""
    d = data[jump:] - data[:-jump]
    return tuple(max(float(d[:, :, c].pow(2).mean().sqrt()), 1e-6) for c in range(3))


def sample_pairs(data: torch.Tensor, B: int, jump: int, gen: torch.Generator):
    frames, n = data.shape[0], data.shape[1]
    ti = torch.randint(0, frames - jump, (B,), generator=gen).to(data.device)
    ni = torch.randint(0, n, (B,), generator=gen).to(data.device)
    return data[ti, ni].contiguous(), data[ti + jump, ni].contiguous()


def train(net: "sw.Surrogate", data: torch.Tensor, steps: int, B: int, lr: float, jump: int, seed: int = 0,
          lr_final: float | None = None, log_every: int = 0):
    """Adam steps on random pairs; cosine decay from lr to lr_final.
    Returns the per-step losses."""
    gen = torch.Generator().manual_seed(seed)
    losses = torch.empty(steps, dtype=torch.float32, device="cuda")
    lr_final = lr if lr_final is None else lr_final
    t0 = time.perf_counter()
    for k in range(steps):
        u, u8 = sample_pairs(data, B, jump, gen)
        lr_k = lr_final + 0.5 * (lr - lr_final) * (1 + math.cos(math.pi * k / max(steps - 1, 1)))
        loss = net.train_step(u, u8, lr_k)
        losses[k] = loss[0]
        if log_every and (k + 1) % log_every == 0:
            print(f"[train] step {k + 1}/{steps} loss {float(losses[k]):.4e} "
                  f"({time.perf_counter() - t0:.1f} s)", flush=True)
    torch.cuda.synchronize()
    return losses.cpu()


def rel_l2_h(h, h_ref):
    """||h - h_ref||_2 / ||h_ref||_2 per grid, and the stricter
    ||h - h_ref||_2 / ||h_ref - mean(h_ref)||_2."""
    d = (h - h_ref).flatten(1).double()
    r = h_ref.flatten(1).double()
    return (d.norm(dim=1) / r.norm(dim=1)), (d.norm(dim=1) / (r - r.mean(dim=1, keepdim=True)).norm(dim=1))


def rollout(net, u0: torch.Tensor, nsteps: int, gate: dict | None = None, l2: torch.Tensor | None = None,
            batch: "sw.Batch | None" = None, fallbacks: torch.Tensor | None = None):
    """Surrogate rollout of a dense [n][3][H][W] state: returns (final state,
    fallbacks per grid, seconds).  gate: keyword arguments of
    ``Surrogate.advance`` (judge mode writes ``l2``); ``batch`` reuses a batch
    of the right shape and ``fallbacks`` an int32 counter array (zeroed here):
    with both reused, repeated calls replay the rollout's captured graph."""
    n, _, H, W = u0.shape
    b = batch if batch is not None else sw.Batch([(W, H)] * n, dtype="f32")
    b.load(u0)
    fb = fallbacks if fallbacks is not None else torch.zeros(n, dtype=torch.int32, device="cuda")
    fb.zero_()
    gate = gate or {}
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net.advance(b, nsteps, fallbacks=fb, l2=l2, **gate)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    return b.export(), fb.cpu(), sec


TUNE_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_cache_gfx950.txt")


def solver_run(u0: torch.Tensor, nsteps: int, tune_cache: str | None = TUNE_CACHE):
    """Plain batched solver from the same state, in its tuned launch shape
    (from the cache; timed and stored there if missing): (final state, seconds)."""
    n, _, H, W = u0.shape
    b = sw.Batch([(W, H)] * n, dtype="f32")
    b.load(u0)
    if tune_cache:
        b.autotune(steps_per_trial=3, cache_path=tune_cache)   # leaves the state as it was
    b.step(nsteps)          # capture
    b.load(u0)
    b.reset_time()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(nsteps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    b.sync_status()
    return b.export(), sec


DEFAULT_FORM = 2   # sw_surrogate_set_fused: the library picks the rollout network's form per batch size
WEIGHTS_256 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "surrogate_256x256_j8.npz")


def save_weights(path: str, net: "sw.Surrogate", in_offset, in_scale, out_scale, meta: dict):
    """FP32 master parameters, normalisation and a JSON description in an
    .npz of plain arrays (loadable without pickle)."""
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    np.savez(path, params=net.get_params().cpu().numpy(), in_offset=np.asarray(in_offset, np.float32),
             in_scale=np.asarray(in_scale, np.float32), out_scale=np.asarray(out_scale, np.float32),
             jump=np.int32(net.jump), H=np.int32(net.H), W=np.int32(net.W), meta=np.array(json.dumps(meta)))


def load_weights(path: str, max_batch: int, seed: int = 0) -> tuple:
    """(network with the stored weights and normalisation, meta dict)."""
    with np.load(path, allow_pickle=False) as z:
        net = sw.Surrogate(int(z["H"]), int(z["W"]), max_batch, jump=int(z["jump"]), seed=seed)
        net.set_params(torch.from_numpy(z["params"]))
        net.set_norm(tuple(z["in_offset"]), tuple(z["in_scale"]), tuple(z["out_scale"]))
        return net, json.loads(str(z["meta"]))
