"""Benchmark of the shallow-water step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

A "step" is one time step of the whole path: CFL dt from the device-side max
signal speed, the two-step Lax-Wendroff update of h, hu, hv, and the boundary
ghosts of the new state (all inside the step kernel).  The timed region is
one sw_step(K) call on the current stream, bracketed by device
synchronisation; inputs are resident in HBM before it starts.  Prints one
JSON line.

Default workload: 16384 x 16384 FP32, periodic, eight seeded Gaussian bumps,
CFL 0.5, 200 steps (the bandwidth-roofline configuration).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gcell-updates/s and % HBM roofline; surrogate speedup at L2(h)≤1e-2"
HBM_PEAK_GBS = 8000.0
FUSED_SRC = [os.path.join(ROOT, "paper_1107_2157_amd", "csrc", f) for f in ("sw_fused.hip", "sw_tile.h", "sw_common.h")]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_fused_swe16384_f32.json")

WORKLOADS = {
    # name: (n, dtype, bc, seed, steps, description)
    "swe16384-f32-periodic": (16384, "f32", "periodic", 3, 200,
                              "16384x16384 FP32, periodic, 8 Gaussian bumps (seed 3), CFL 0.5"),
    "swe4096-f32-reflect": (4096, "f32", "reflect", 2, 1000,
                            "4096x4096 FP32, reflective walls, 8 Gaussian bumps (seed 2), CFL 0.5"),
    "swe4096-f64-reflect": (4096, "f64", "reflect", 2, 1000,
                            "4096x4096 FP64, reflective walls, 8 Gaussian bumps (seed 2), CFL 0.5"),
    "dam128-f64": (128, "f64", "reflect", None, 100,
                   "128x128 FP64 dam break, reflective walls, CFL 0.5"),
    "swe4096-f32-reflect-transverse": (4096, "f32", "reflect", 2, 1000,
                                       "4096x4096 FP32, reflective walls, 8 Gaussian bumps (seed 2), CFL 0.5, "
                                       "transverse scheme"),
    "swe4096-f64-reflect-transverse": (4096, "f64", "reflect", 2, 1000,
                                       "4096x4096 FP64, reflective walls, 8 Gaussian bumps (seed 2), CFL 0.5, "
                                       "transverse scheme"),
}
GOLDEN_4096 = os.path.join(ROOT, "tests", "golden", "swe4096_1000steps.json")
# where the synthetic initial states are generated ("cpu" with --host-inputs:
# they are then copied in, and the GPU runs only the library's kernels and
# copies, which is how the committed profiles are taken)
INPUT_DEVICE = "cuda"


def scheme_of(name):
    return "transverse" if name.endswith("-transverse") else "paper"


def source_hash(paths) -> str:
    h = hashlib.sha256()
    for p in paths:
        with open(p, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def make_solver(name, sw, ics, torch):
    n, dtype, bc, seed, _, _ = WORKLOADS[name]
    bcv = sw.PERIODIC if bc == "periodic" else sw.REFLECT
    scheme = sw.SCHEME_TRANSVERSE if scheme_of(name) == "transverse" else sw.SCHEME_PAPER
    s = sw.Solver(n, n, dtype=dtype, bc_x=bcv, bc_y=bcv, scheme=scheme)
    if seed is None:
        st = ics.dam_break_state(n, device=INPUT_DEVICE)
    else:
        st = ics.bumps_state(n, n, seed=seed, periodic=bc == "periodic", count=8, device=INPUT_DEVICE)
    s.set_state(*st)
    del st
    torch.cuda.synchronize()
    return s


def timed(torch, fn):
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    fn()
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3


def run_workload(name, steps, warmup, sw, ics, torch, tune_cache, fixed=None):
    n, dtype, bc, seed, _, desc = WORKLOADS[name]
    s = make_solver(name, sw, ics, torch)
    ic = tuple(s.interior(k).clone() for k in range(3))
    if fixed:
        s.set_tuning(*fixed)
        tuning = s.get_tuning()
    else:
        tuning = s.autotune(steps_per_trial=3 if n >= 8192 else 10, cache_path=tune_cache)
    if warmup > 0:
        s.step(warmup)

    def restart():                                   # the initial state in buffer 0, time zero
        s.state.cur = 0
        s.set_state(*ic)
        s.reset_time()

    # untimed calibration call: with the timed call it separates the per-call
    # prologue (halo fill + first CFL reduction) from the per-step kernel time.
    # Both calls start from the initial state; their graphs (keyed by steps
    # and current buffer) are captured beforehand, outside the timed calls.
    k_cal = max(1, steps // 4)
    for k in (k_cal, steps):
        restart()
        s.step(k)
    restart()
    t_cal = timed(torch, lambda: s.step(k_cal))
    restart()
    torch.cuda.synchronize()
    t = timed(torch, lambda: s.step(steps))          # the timed region: exactly `steps` steps from the initial state
    finite = True
    try:
        s.sync_status()
    except sw.Unstable:
        finite = False
    per_step = (t - t_cal) / (steps - k_cal) if steps > k_cal else t / steps
    cells = n * n
    elem = 4 if dtype == "f32" else 8
    out = {
        "workload": name, "description": desc, "nx": n, "ny": n, "steps": steps, "dtype": dtype,
        "scheme": scheme_of(name), "seconds": t, "gcells_per_s": cells * steps / t / 1e9,
        "ms_per_step": 1e3 * t / steps, "kernel_us": per_step * 1e6, "alg_bytes_per_launch": 6 * elem * cells,
        "tuning": tuning, "finite": finite,
    }
    vs = versus_oracle_1000(name, s, steps, torch)
    if vs is not None:
        out["vs_oracle_1000"] = vs
    del s
    torch.cuda.empty_cache()
    return out


def versus_oracle_1000(name, s, steps, torch):
    """The GPU state after the timed run (`steps` steps from the initial
    state) against the CPU oracle's stored 1000-step state of the same
    4096^2 workload (tests/golden, written by a script that calls only the
    oracle): reported, not gated.  Differences at a 16 x 16 lattice of cells,
    relative to the max-norm scales of h and of the momenta, and relative
    differences of the per-field sums and 2-norms; FP32 runs are compared
    with the oracle run started from the FP32-rounded state."""
    import math
    import numpy as np
    n, dtype = WORKLOADS[name][0], WORKLOADS[name][1]
    if n != 4096 or steps != 1000 or not os.path.exists(GOLDEN_4096):
        return None
    with open(GOLDEN_4096) as f:
        gold = json.load(f)
    run = [r for r in gold["runs"] if r["scheme"] == scheme_of(name) and r["start"] == dtype]
    if not run:
        return None
    run = run[0]
    lat = gold["lattice"]
    t_gpu, _, _ = s.sync_status() if run["finite"] else (float("nan"), 0, 0)
    got = {k: s.interior(i).to("cpu", dtype=torch.float64).numpy() for i, k in enumerate(("h", "hu", "hv"))}
    sh = run["fields"]["h"]["max_abs"]
    sm = sh * math.sqrt(9.8 * sh)
    out = {"scheme": run["scheme"], "oracle_finite": run["finite"], "t_gpu": t_gpu, "t_oracle": run["t"]}
    for k in ("h", "hu", "hv"):
        g = got[k]
        ref = np.array(run["fields"][k]["lattice"])
        samp = g[np.ix_(lat, lat)]
        scale = sh if k == "h" else sm
        out[f"{k}_lattice_rel_max"] = float(np.max(np.abs(samp - ref)) / scale)
        out[f"{k}_sum_rel"] = float(abs(math.fsum(g.ravel()) - run["fields"][k]["sum"]) / max(abs(run["fields"][k]["sum"]), scale))
        out[f"{k}_l2_rel"] = float(abs(float(np.sqrt(np.sum(g * g))) - run["fields"][k]["l2"]) / run["fields"][k]["l2"])
    return out


def run_fixed_dt(steps, fused_tuning, sw, ics, torch, tune_cache):
    """Fixed-dt mode (dt = 0.5 dx / the initial state's max signal speed) on
    the headline grid: the fused single-step kernel in the headline's tuned
    shape against the autotuner's fixed-dt choice, which may be temporal
    blocking (K steps of a tile per launch, staged in LDS).  `steps` is a
    multiple of every K, so no single-step remainder runs.  Both runs start
    from the same state; their final states must be bitwise equal."""
    n, dtype, _, seed, _, _ = WORKLOADS["swe16384-f32-periodic"]
    st = ics.bumps_state(n, n, seed=seed, periodic=True, count=8, device=INPUT_DEVICE)
    h, hu, hv = st
    dt = 0.5 / float((torch.maximum(hu.abs(), hv.abs()) / h + torch.sqrt(9.8 * h)).max())
    s = sw.Solver(n, n, dtype=dtype, bc_x=sw.PERIODIC, bc_y=sw.PERIODIC, cfl=0.0, dt_fixed=dt)

    def restart():
        s.state.cur = 0
        s.set_state(*st)
        s.reset_time()

    out = {"workload": "swe16384-f32-periodic-fixed-dt", "dtype": dtype, "steps": steps, "dt": dt}
    finals = []
    for label in ("fused", "tuned"):
        restart()
        if label == "fused":
            s.set_tuning(**fused_tuning)
            tuning = s.get_tuning()
        else:
            tuning = s.autotune(steps_per_trial=3, cache_path=tune_cache)
        restart()
        s.step(steps)                                # graph capture + warm-up
        restart()
        t = timed(torch, lambda: s.step(steps))
        s.sync_status()
        finals.append([s.interior(k).clone() for k in range(3)])
        g = n * n * steps / t / 1e9
        out[label] = {"tuning": tuning, "gcells_per_s": g, "ms_per_step": 1e3 * t / steps,
                      # bandwidth a single-step kernel would need for this rate (24 B per cell-update)
                      "single_step_equiv_hbm_frac": g * 24 / HBM_PEAK_GBS}
    out["speedup"] = out["tuned"]["gcells_per_s"] / out["fused"]["gcells_per_s"]
    out["bitwise_equal"] = all(torch.equal(a, b) for a, b in zip(*finals))
    del s, st, finals
    torch.cuda.empty_cache()
    return out


def run_comparison(steps, fused_tuning, sw, ics, torch):
    """The paper's comparison designs (section "Performance Measurements") on
    the headline workload: the fused kernel in the headline's tuned shape,
    the unfused step (face states of the first half-step written to HBM and
    read back by a second kernel), the AoS step (one (h, hu, hv, 0) vector
    per cell; each call converts the state in and out) and the kernels
    generated from region expressions in both designs (row march in
    registers; the paper's LDS tiles with one thread per cell), halo filled
    by a separate launch.  Per-step times come from two calls of
    different length, so the per-call work (prologue, AoS conversions)
    cancels.  The fused, unfused and AoS final states must be bitwise equal;
    the generated kernel's differs by rounding."""
    name = "swe16384-f32-periodic"
    n = WORKLOADS[name][0]
    s = make_solver(name, sw, ics, torch)
    ic = tuple(s.interior(k).clone() for k in range(3))

    def restart():
        s.state.cur = 0
        s.set_state(*ic)
        s.reset_time()

    out = {"workload": name + "-paper-comparison", "dtype": "f32", "steps": steps}
    finals = []
    k_cal = steps // 5
    for label, tuning in (("fused", fused_tuning), ("unfused", {"variant": 4}), ("aos", {"variant": 5}),
                          ("generated", {"variant": 6, "vec": 2}), ("generated_lds", {"variant": 6, "vec": 1})):
        s.set_tuning(**tuning)
        for k in (k_cal, steps):                   # graph capture (and workspace) outside the timed calls
            restart()
            s.step(k)
        restart()
        t_cal = timed(torch, lambda: s.step(k_cal))
        restart()
        t = timed(torch, lambda: s.step(steps))
        s.sync_status()
        finals.append([s.interior(k).clone() for k in range(3)])
        per_step = (t - t_cal) / (steps - k_cal)
        out[label] = {"tuning": s.get_tuning(), "gcells_per_s": n * n / per_step / 1e9,
                      "ms_per_step": 1e3 * per_step, "ms_per_call": 1e3 * t}
    for label in ("unfused", "aos", "generated", "generated_lds"):
        out[label]["ratio_to_fused"] = out[label]["gcells_per_s"] / out["fused"]["gcells_per_s"]
    out["unfused_to_aos"] = out["unfused"]["gcells_per_s"] / out["aos"]["gcells_per_s"]
    out["generated_to_aos"] = out["generated"]["gcells_per_s"] / out["aos"]["gcells_per_s"]
    out["bitwise_equal"] = all(torch.equal(a, b) and torch.equal(a, c) for a, b, c, _, _ in zip(*finals))
    # the generated kernels evaluate the program's own expressions: equal to rounding
    for label, k in (("generated", 3), ("generated_lds", 4)):
        out[label]["max_rel_diff_to_fused"] = max(
            float((g.double() - f.double()).abs().max() / f.double().abs().max()) for f, g in zip(finals[0], finals[k]))
    del s, ic, finals
    torch.cuda.empty_cache()
    return out


# Table 1 of the paper: ms per time step of its generated OpenCL kernel (work-group 16 x 8) on a
# Tesla C2050, FP32, mean over 100 iterations of the time loop.  Context only (other hardware).
TABLE1 = os.path.join(ROOT, "tests", "golden", "table1_times.csv")


def paper_table1_gpu_ms():
    """width -> the paper's GPU ms per step (Table 1), from the stored copy of the table."""
    out = {}
    with open(TABLE1) as f:
        for line in f:
            if line.startswith("#") or line.startswith("width"):
                continue
            w, _, gpu_ms, _ = line.strip().split(",")
            out[int(w)] = float(gpu_ms)
    return out


def run_batch_uniform(n_grids, side, steps, sw, ics, torch, tune_cache):
    """A batch of equal grids: n_grids of side^2 cells (the surrogate's
    solver workload at 256 grids of 256^2), each with its own 1-8 Gaussian
    bumps (seed 4000 + k), FP32, reflective walls, one graph launch per
    call in the autotuner's launch shape."""
    b = sw.Batch([side] * n_grids, dtype="f32")
    for k in range(n_grids):
        b.set_state(k, *ics.bumps_state(side, side, seed=ics.SEED_BATCH_GRID0 + k, periodic=False,
                                        device=INPUT_DEVICE))
    torch.cuda.synchronize()
    tuning = b.autotune(steps_per_trial=3, cache_path=tune_cache)
    b.step(2)
    b.step(steps)
    t = timed(torch, lambda: b.step(steps))
    finite = True
    try:
        b.sync_status()
    except sw.Unstable:
        finite = False
    del b
    torch.cuda.empty_cache()
    cells = n_grids * side * side
    rate = cells * steps / t / 1e9
    return {"workload": f"batch{n_grids}x{side}-f32-reflect", "grids": n_grids, "cells_per_step": cells,
            "steps": steps, "seconds": t, "gcells_per_s": rate, "ms_per_step": 1e3 * t / steps, "tuning": tuning,
            "finite": finite, "hbm_frac": rate * 24 / HBM_PEAK_GBS}


def run_table1(sw, ics, torch, tune_cache, steps=100):
    """The widths of the paper's Table 1, FP32, reflective walls, CFL 0.5,
    8 Gaussian bumps (the paper does not state its initial state): one
    sw_step(100) call (one graph launch) per width, timed whole, as the
    paper averaged 100 iterations of its time loop; the fused kernel in the
    autotuner's launch shape for the width (`ms_per_step`) and in its default
    shape (`default_ms_per_step`)."""
    rows = []
    for n, paper_ms in paper_table1_gpu_ms().items():
        s = sw.Solver(n, n, dtype="f32")
        st = ics.bumps_state(n, n, seed=ics.SEED_BUMPS_4096, periodic=False, count=8, device=INPUT_DEVICE)

        def call_ms():
            for _ in range(2):                     # graph capture for both buffers, warm
                s.state.cur = 0
                s.set_state(*st)
                s.step(steps)
            s.state.cur = 0
            s.set_state(*st)
            s.reset_time()
            t = timed(torch, lambda: s.step(steps))
            s.sync_status()
            return 1e3 * t / steps

        default_ms = call_ms()
        tuning = s.autotune(steps_per_trial=10, cache_path=tune_cache)
        ms = call_ms()
        rows.append({"width": n, "ms_per_step": ms, "gcells_per_s": n * n / (ms * 1e-3) / 1e9,
                     "paper_c2050_ms": paper_ms, "ratio_to_paper": paper_ms / ms, "tuning": tuning,
                     "default_ms_per_step": default_ms})
        del s, st
    torch.cuda.empty_cache()
    return {"workload": "table1-widths-f32-reflect", "steps_per_call": steps, "rows": rows}


def run_batch(steps, sw, ics, torch, tune_cache, per_grid_steps):
    """Batched workload: 512 grids, sides 64*(1 + floor(16u)) (seed 4), each
    with its own 1-8 Gaussian bumps (seed 4000 + k), FP32, reflective walls.
    One hipGraph launch per call covering every grid, against per-grid
    launches (one sw_step call per grid on the same stream)."""
    sides = ics.batch_sides(512)
    cells = sum(s * s for s in sides)
    b = sw.Batch(sides, dtype="f32")
    for k, n in enumerate(sides):
        b.set_state(k, *ics.bumps_state(n, n, seed=ics.SEED_BATCH_GRID0 + k, periodic=False, device=INPUT_DEVICE))
    torch.cuda.synchronize()
    tuning = b.autotune(steps_per_trial=3, cache_path=tune_cache)
    b.step(2)                                          # warm: captures the graph for this call shape
    b.step(steps)                                      # (captures the graph for `steps`)
    t = timed(torch, lambda: b.step(steps))
    finite = True
    try:
        b.sync_status()
    except sw.Unstable:
        finite = False
    del b
    torch.cuda.empty_cache()
    rate = cells * steps / t / 1e9
    if per_grid_steps <= 0:
        return {"workload": "batch512-f32-reflect", "grids": 512, "cells_per_step": cells, "steps": steps,
                "seconds": t, "gcells_per_s": rate, "ms_per_step": 1e3 * t / steps, "tuning": tuning,
                "finite": finite, "hbm_frac": rate * 24 / HBM_PEAK_GBS}
    # per-grid launches: every grid its own context and planes, `per_grid_steps` steps
    solvers = []
    for k, n in enumerate(sides):
        s = sw.Solver(n, n, dtype="f32")
        s.set_state(*ics.bumps_state(n, n, seed=ics.SEED_BATCH_GRID0 + k, periodic=False, device=INPUT_DEVICE))
        solvers.append(s)
    for s in solvers:
        s.step(1)
    t_pg = timed(torch, lambda: [s.step(per_grid_steps) for s in solvers])
    del solvers
    torch.cuda.empty_cache()
    per_grid_rate = cells * per_grid_steps / t_pg / 1e9
    rate = cells * steps / t / 1e9
    return {"workload": "batch512-f32-reflect", "grids": 512, "cells_per_step": cells, "steps": steps,
            "seconds": t, "gcells_per_s": rate, "ms_per_step": 1e3 * t / steps, "tuning": tuning,
            "finite": finite, "per_grid_launches": {"steps": per_grid_steps, "seconds": t_pg,
                                                     "gcells_per_s": per_grid_rate,
                                                     "launches": 512 * (per_grid_steps + 2)},
            "speedup_vs_per_grid": rate / per_grid_rate,
            "hbm_frac": rate * 24 / HBM_PEAK_GBS}


SUR_FLOP_PER_PIXEL_FWD = 2 * 9 * (3 * 32 + 4 * 32 * 32 + 32 * 3)          # 77 184 per pixel per jump
SUR_FLOP_PER_PIXEL_TRAIN = SUR_FLOP_PER_PIXEL_FWD * 2 + 2 * 9 * (4 * 32 * 32 + 32 * 3)   # + wgrad + dgrad
BF16_PEAK_TFLOPS = 2500.0


def run_surrogate(sw, ics, torch, n=256, size=256, nsteps=64, kernels=True):
    """Surrogate workload: n held-out size x size grids (seeds SEED_SURR_EVAL0 + k,
    1-8 bumps, reflective walls, FP32), advanced nsteps = nsteps / 8 jumps of the
    trained network (committed weights) under the gate (mass drift 1e-4 with
    projection, h > 0, finite), against the plain batched solver (one graph
    launch) from the same states.  The rollout is timed in the library's
    default form (the network as one fused launch or as per-layer launches,
    whichever the batch size favours) and in both forms; the judged rollout
    (the solver's state replaces any grid above relative L2(h) 1e-2) is timed
    too, and its final L2 checked.  With kernels, also the per-layer forward
    pass alone and one training step at batch n."""
    from paper_1107_2157_amd import surrogate
    name = f"surrogate{size}-b{n}-{nsteps}steps"
    if os.path.exists(surrogate.WEIGHTS_256):
        net, meta = surrogate.load_weights(surrogate.WEIGHTS_256, n)
    else:   # timings only: accuracy figures of an untrained network mean nothing
        net, meta = sw.Surrogate(size, size, n, jump=8, seed=1), {"untrained": True}
    u0 = surrogate.initial_states(n, size, size, ics.SEED_SURR_EVAL0, device=INPUT_DEVICE).cuda()
    ref, t_solver = surrogate.solver_run(u0, nsteps)
    gate = dict(mass_rel_tol=1e-4, project_mass=True)
    b = sw.Batch([(size, size)] * n, dtype="f32")
    fbs = torch.zeros(n, dtype=torch.int32, device="cuda")

    def best_rollout(g, **kw):
        surrogate.rollout(net, u0, nsteps, g, batch=b, fallbacks=fbs, **kw)       # warm: captures the graph
        runs = [surrogate.rollout(net, u0, nsteps, g, batch=b, fallbacks=fbs, **kw) for _ in range(3)]
        return min(runs, key=lambda r: r[2])

    forms = {}
    for form, mode in (("fused", 1), ("per_layer", 0), ("default", None)):
        net.set_fused(surrogate.DEFAULT_FORM if mode is None else mode)
        got, fb, t_sur = best_rollout(gate)
        forms[form] = {"seconds": t_sur, "speedup_vs_solver": t_solver / t_sur}
    e, e_strict = surrogate.rel_l2_h(got[:, 0], ref[:, 0])
    p, _ = surrogate.rel_l2_h(u0[:, 0], ref[:, 0])
    l2 = torch.zeros(n, dtype=torch.float64, device="cuda")
    jg = dict(gate, judge=True, l2_tol=1e-2)
    judged, fbj, t_judge = best_rollout(jg, l2=l2)
    ej, _ = surrogate.rel_l2_h(judged[:, 0], ref[:, 0])
    judged_out = int((l2 > 1e-2).sum())
    del b
    out = {"workload": name, "grids": n, "size": size, "steps": nsteps, "jump": 8,
           "solver_seconds": t_solver, "rollout_seconds": forms["default"]["seconds"],
           "speedup_vs_solver": forms["default"]["speedup_vs_solver"], "forms": forms,
           "rel_l2_h_mean": float(e.mean()), "rel_l2_h_max": float(e.max()),
           "rel_l2_h_strict_mean": float(e_strict.mean()), "persistence_rel_l2_h_mean": float(p.mean()),
           "fallback_jumps": int(fb.sum()), "jumps": n * nsteps // 8,
           "judged": {"seconds": t_judge, "speedup_vs_solver": t_solver / t_judge, "rejected_grids": judged_out,
                      "rel_l2_h_max": float(ej.max()), "within_1e-2": bool(ej.max() <= 1e-2)},
           "weights": "untrained" if meta.get("untrained") else "trained",
           "weights_recipe": meta.get("recipe"), "weights_eval": meta.get("eval")}
    if kernels:
        net.forward(u0)
        t_fwd = timed(torch, lambda: net.forward(u0))
        pixels = n * size * size
        fwd_tflops = SUR_FLOP_PER_PIXEL_FWD * pixels / t_fwd / 1e12
        # one Adam step on (U^0, U^8) pairs of the same grids, on a separate network
        bt = sw.Batch([(size, size)] * n, dtype="f32")
        bt.load(u0)
        bt.step(8)
        u8 = bt.export()
        del bt
        tnet = sw.Surrogate(size, size, n, jump=8, seed=1)
        tnet.train_step(u0, u8, 1e-5)
        t_train = timed(torch, lambda: tnet.train_step(u0, u8, 1e-5))
        del tnet
        out.update({"forward_ms": 1e3 * t_fwd, "forward_tflops": fwd_tflops,
                    "forward_frac_bf16_peak": fwd_tflops / BF16_PEAK_TFLOPS, "train_step_ms": 1e3 * t_train,
                    "train_tflops": SUR_FLOP_PER_PIXEL_TRAIN * pixels / t_train / 1e12})
    del net
    torch.cuda.empty_cache()
    return out


def surrogate_kernels(sw, ics, torch, n=256, size=256, reps=3):
    """The surrogate's kernels alone, reps times each, on n seeded bump states
    (and their states 8 solver steps later): the per-layer forward pass, the
    Adam step, and one rollout jump with the fused network launch and with
    the per-layer kernels (eager launches, gate wide open, so that every
    jump is the network's)."""
    from paper_1107_2157_amd import surrogate
    u0 = surrogate.initial_states(n, size, size, ics.SEED_SURR_EVAL0, device=INPUT_DEVICE).cuda()
    b = sw.Batch([(size, size)] * n, dtype="f32")
    b.load(u0)
    b.step(8)
    u8 = b.export()
    net = sw.Surrogate(size, size, n, jump=8, seed=1)
    t_fwd = [timed(torch, lambda: net.forward(u0)) for _ in range(reps)]
    t_train = [timed(torch, lambda: net.train_step(u0, u8, 1e-5)) for _ in range(reps)]
    net.set_graph(False)
    jumps = {}
    for fused in (True, False):
        net.set_fused(fused)
        b.load(u0)
        ts = [timed(torch, lambda: net.advance(b, 8, mass_rel_tol=10.0, hmin=-1e30)) for _ in range(reps)]
        jumps["fused" if fused else "per_layer"] = [1e3 * t for t in ts]
    del b
    pixels = n * size * size
    return {"workload": f"surrogate{size}-b{n}-kernels", "forward_ms": [1e3 * t for t in t_fwd],
            "train_step_ms": [1e3 * t for t in t_train], "rollout_jump_ms": jumps,
            "forward_tflops": SUR_FLOP_PER_PIXEL_FWD * pixels / min(t_fwd) / 1e12,
            "train_tflops": SUR_FLOP_PER_PIXEL_TRAIN * pixels / min(t_train) / 1e12}


def copy_bandwidth(torch, nbytes):
    """Device copy of nbytes (read + write) with torch: attainable streaming BW."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    ts = [timed(torch, lambda: b.copy_(a)) for _ in range(5)]
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / min(ts) / 1e9


def cpu_baseline(name, ics):
    """The oracle on a bounded sample of the same workload: a 256-row band of
    the full-width grid (same bumps), periodic, ~10 s of single-thread CPU."""
    import oracle
    n, dtype, bc, seed, _, _ = WORKLOADS[name]
    rows = min(n, 256)
    if seed is None:
        h, hu, hv = (a.numpy() for a in ics.dam_break_state(n))
    else:
        h, hu, hv = (a.numpy() for a in ics.bumps_band(n, n, 0, rows, seed, bc == "periodic", count=8))
    nrows = h.shape[0]
    t0 = time.perf_counter()
    oracle.run(h, hu, hv, 1, bcx=oracle.PERIODIC, bcy=oracle.PERIODIC)
    one = time.perf_counter() - t0
    k = max(1, min(200, int(10.0 / max(one, 1e-6))))
    t0 = time.perf_counter()
    oracle.run(h, hu, hv, k, bcx=oracle.PERIODIC, bcy=oracle.PERIODIC)
    sec = time.perf_counter() - t0
    return {"value": n * nrows * k / sec / 1e9, "unit": "Gcell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{n}x{nrows} band of the same initial state, periodic, FP64, {k} steps, {sec:.1f} s, "
                      f"single thread",
            "all_cores": cpu_all_cores(h, hu, hv, k)}


def cpu_all_cores(h, hu, hv, k):
    """The same oracle, unchanged and single-threaded, in one child process
    per host core (at most the 16-core share of one GPU), each stepping its
    own copy of the band k steps at once: aggregate cell-updates / wall time.
    The children import only numpy and the oracle."""
    import subprocess
    import tempfile
    import numpy as np
    procs = min(16, len(os.sched_getaffinity(0)), int(os.environ.get("OMP_NUM_THREADS", "16")))
    code = ("import sys, numpy as np; sys.path.insert(0, sys.argv[1]); import oracle; "
            "h, hu, hv = (np.load(sys.argv[2] + f'/{c}.npy') for c in 'huv'); "
            "oracle.run(h, hu, hv, int(sys.argv[3]), bcx=oracle.PERIODIC, bcy=oracle.PERIODIC)")
    with tempfile.TemporaryDirectory() as d:
        for c, a in zip("huv", (h, hu, hv)):
            np.save(os.path.join(d, f"{c}.npy"), np.ascontiguousarray(a))
        t0 = time.perf_counter()
        ps = [subprocess.Popen([sys.executable, "-c", code, ROOT, d, str(k)]) for _ in range(procs)]
        rcs = [p.wait() for p in ps]
        sec = time.perf_counter() - t0
    if any(rcs):
        return None
    cells = h.shape[0] * h.shape[1]
    return {"value": procs * cells * k / sec / 1e9, "unit": "Gcell-updates/s", "cores": procs, "kind": "oracle",
            "sample": f"{procs} processes, each the {h.shape[1]}x{h.shape[0]} band for {k} steps, {sec:.1f} s wall "
                      f"(process start included)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="swe16384-f32-periodic", choices=sorted(WORKLOADS))
    ap.add_argument("--no-also", action="store_true", help="skip the secondary 4096^2 FP32/FP64 runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched 512-grid run")
    ap.add_argument("--no-surrogate", action="store_true", help="skip the learned-surrogate run")
    ap.add_argument("--comparison-only", action="store_true",
                    help="run only the paper-comparison record (fused against unfused and AoS steps)")
    ap.add_argument("--fixed-dt-only", action="store_true",
                    help="run only the fixed-dt comparison (fused single step against temporal blocking)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the learned-surrogate workload and print its record")
    ap.add_argument("--batch-only", action="store_true",
                    help="run only the batched 512-grid workload and print its record")
    ap.add_argument("--no-per-grid", action="store_true",
                    help="with --batch-only: skip the per-grid-launch comparison (for counter profiles)")
    ap.add_argument("--surrogate-kernels", action="store_true",
                    help="run only the surrogate's forward pass and training step at 256 grids of 256^2 (three "
                         "each, for kernel profiles) and print their times")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1107_2157_amd", "tune_cache_gfx950.txt"),
                    help="autotuner cache (launch shapes found by sw_autotune on MI355X; missing keys are tuned "
                         "and appended)")
    ap.add_argument("--host-inputs", action="store_true",
                    help="generate the initial states on the host and copy them in (for profiled runs)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 3 GiB device-to-device copy (counter calibration) and exit")
    ap.add_argument("--tuning", default=None,
                    help="fixed launch shape 'variant,rows,vec,occupancy' instead of the autotuner")
    args = ap.parse_args()
    global INPUT_DEVICE
    if args.host_inputs:
        INPUT_DEVICE = "cpu"
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the library has no "
              "domain-decomposed path", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.calibrate_copy:
        # a plain copy of known size: 3 GiB read + 3 GiB written per dispatch
        a = torch.ones(3 * 2 ** 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(6):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes_read": a.numel() * 4, "bytes_written": b.numel() * 4}))
        return
    from paper_1107_2157_amd import ics, sw
    sw.lib()    # fails loudly if the HIP library is not built
    if args.surrogate_only:
        print(json.dumps(run_surrogate(sw, ics, torch)), flush=True)
        return
    if args.surrogate_kernels:
        print(json.dumps(surrogate_kernels(sw, ics, torch)), flush=True)
        return
    if args.batch_only:
        print(json.dumps(run_batch(args.steps or 500, sw, ics, torch, args.tune_cache,
                                   per_grid_steps=0 if args.no_per_grid else 50)), flush=True)
        return

    if args.comparison_only:
        probe = make_solver("swe16384-f32-periodic", sw, ics, torch)
        fused = probe.autotune(steps_per_trial=3, cache_path=args.tune_cache)   # the headline's shape
        del probe
        torch.cuda.empty_cache()
        print(json.dumps(run_comparison(50, fused, sw, ics, torch)), flush=True)
        return

    if args.fixed_dt_only:
        probe = make_solver("swe16384-f32-periodic", sw, ics, torch)
        fused = probe.autotune(steps_per_trial=3, cache_path=args.tune_cache)   # the headline's shape
        del probe
        torch.cuda.empty_cache()
        print(json.dumps(run_fixed_dt(210, fused, sw, ics, torch, args.tune_cache)), flush=True)
        return

    steps = args.steps or WORKLOADS[args.workload][4]
    fixed = tuple(int(x) for x in args.tuning.split(",")) if args.tuning else None
    main_run = run_workload(args.workload, steps, args.warmup, sw, ics, torch, args.tune_cache, fixed)
    value = main_run["gcells_per_s"]
    achieved = main_run["alg_bytes_per_launch"] / (main_run["kernel_us"] * 1e-6) / 1e9
    copy_bw = copy_bandwidth(torch, main_run["alg_bytes_per_launch"] // 2)

    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("source_sha256_16") == source_hash(FUSED_SRC) and tr.get("tuning") == main_run["tuning"]:
            traffic = tr.get("bytes_per_launch")

    also = []
    if not args.no_also and args.workload == "swe16384-f32-periodic":
        for name in ("swe4096-f32-reflect", "swe4096-f64-reflect", "swe4096-f32-reflect-transverse",
                     "swe4096-f64-reflect-transverse", "dam128-f64"):
            r = run_workload(name, WORKLOADS[name][4], args.warmup, sw, ics, torch, args.tune_cache)
            also.append({k: r[k] for k in ("workload", "dtype", "scheme", "steps", "gcells_per_s", "ms_per_step",
                                            "kernel_us", "finite", "tuning") + (("vs_oracle_1000",) if "vs_oracle_1000" in r else ())} |
                        {"hbm_frac": r["alg_bytes_per_launch"] / (r["kernel_us"] * 1e-6) / 1e9 / HBM_PEAK_GBS})

    if not args.no_also and args.workload == "swe16384-f32-periodic":
        also.append(run_comparison(50, main_run["tuning"], sw, ics, torch))

    if not args.no_also and args.workload == "swe16384-f32-periodic":
        also.append(run_fixed_dt(210, main_run["tuning"], sw, ics, torch, args.tune_cache))

    if not args.no_also and not args.no_batch and args.workload == "swe16384-f32-periodic":
        also.append(run_batch(500, sw, ics, torch, args.tune_cache, per_grid_steps=50))
        also.append(run_batch_uniform(256, 256, 200, sw, ics, torch, args.tune_cache))

    if not args.no_also and args.workload == "swe16384-f32-periodic":
        also.append(run_table1(sw, ics, torch, args.tune_cache))

    if not args.no_also and not args.no_surrogate and args.workload == "swe16384-f32-periodic":
        also.append(run_surrogate(sw, ics, torch))
        also.append(run_surrogate(sw, ics, torch, n=16, kernels=False))
        also.append(run_surrogate(sw, ics, torch, n=1, kernels=False))      # batch 1: the launch-bound end

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "Gcell-updates/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": main_run["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": main_run["dtype"],
        "data": "synthetic",
        "config": {"workload": main_run["workload"], "description": main_run["description"],
                   "nx": main_run["nx"], "ny": main_run["ny"], "scheme": "paper", "cfl": 0.5,
                   "tuning": main_run["tuning"], "finite": main_run["finite"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "k_step_fused", "kernel_us": main_run["kernel_us"],
                     "alg_bytes_per_launch": main_run["alg_bytes_per_launch"],
                     "torch_copy_gbs": copy_bw},
        "also": also,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(args.workload, ics)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
