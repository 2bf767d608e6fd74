"""Parity at the benchmark workloads' full sizes, in the launch shapes
bench.py times (tuned shapes from the committed cache).

The oracle cannot afford 268 M cells, so it checks sampled outputs.  With a
fixed time step a cell after k steps depends only on the initial state within
k cells of it (every step reads a one-cell neighbourhood), so the oracle
advances a patch of radius k + 2 around each sampled cell (wrapped on
periodic axes, clipped at reflective walls, where the patch's own boundary
rule is the wall's) and its centre is exact.  The CFL time step is checked
at full size against the oracle's global maximum signal speed, the full
200-step CFL run by properties that hold at any size, batched grids against
whole-grid oracle runs (each grid of a batch is independent), and the
network's output at sampled pixels against the network oracle on a patch
that contains the pixel's receptive field.
"""
import math
import os

import numpy as np
import pytest
import torch

import oracle
from oracle import net_oracle as no
from paper_1107_2157_amd import ics, surrogate, sw
from swtest import G, announce

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
CACHE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1107_2157_amd",
                     "tune_cache_gfx950.txt")


def sample_cells(nx, ny, rng, count=24, tile_rows=8, tile_cols=256, bumps=()):
    """Corners, edge midpoints, cells on tile seams, cells at each bump's
    centre and about one sigma out (where the state moves: far from the bumps
    the water is still), and random cells."""
    pts = {(0, 0), (nx - 1, 0), (0, ny - 1), (nx - 1, ny - 1), (nx // 2, 0), (0, ny // 2), (nx - 1, ny // 2),
           (nx // 2, ny - 1)}
    for bp in bumps:
        a = rng.uniform(0, 2 * math.pi)
        for r in (0.0, bp.sigma):
            pts.add((int(bp.cx + r * math.cos(a)) % nx, int(bp.cy + r * math.sin(a)) % ny))
    for _ in range(4):
        pts.add((int(rng.integers(1, max(nx // tile_cols, 1) + 1)) * tile_cols % nx, int(rng.integers(0, ny))))
        pts.add((int(rng.integers(0, nx)), int(rng.integers(1, max(ny // tile_rows, 1) + 1)) * tile_rows % ny))
    while len(pts) < count:
        pts.add((int(rng.integers(0, nx)), int(rng.integers(0, ny))))
    return sorted(pts)


def patch_reference(state, x, y, k, dt, periodic, dx=1.0, dy=1.0):
    """Oracle value of cell (x, y) after k fixed-dt steps, from a patch."""
    h = state[0]
    ny, nx = h.shape
    R = k + 2

    def axis(c, n):
        if periodic:
            assert n > 2 * R + 1
            return np.arange(c - R, c + R + 1) % n, R
        lo, hi = max(0, c - R), min(n, c + R + 1)
        return np.arange(lo, hi), c - lo

    ix, cx = axis(x, nx)
    iy, cy = axis(y, ny)
    p = [np.ascontiguousarray(a[np.ix_(iy, ix)]) for a in state]
    H, U, V, _ = oracle.run(*p, k, g=G, dx=dx, dy=dy, dt_fixed=dt, bcx=oracle.REFLECT, bcy=oracle.REFLECT)
    return H[1 + cy, 1 + cx], U[1 + cy, 1 + cx], V[1 + cy, 1 + cx]


def gpu_cells(s, cells):
    xs = torch.tensor([c[0] for c in cells], device="cuda")
    ys = torch.tensor([c[1] for c in cells], device="cuda")
    return [s.interior(k)[ys, xs].double().cpu().numpy() for k in range(3)]


def compare(got, ref, dtype):
    sh = max(np.max(np.abs(ref[0])), 1e-300)
    sm = sh * math.sqrt(G * sh)
    err = max(np.max(np.abs(got[0] - ref[0])) / sh, np.max(np.abs(got[1] - ref[1])) / sm,
              np.max(np.abs(got[2] - ref[2])) / sm)
    assert err <= TOL[dtype], err
    return err


def rounded_state(st, dtype):
    """Interior state as FP64 numpy arrays, rounded through the run's dtype."""
    td = torch.float32 if dtype == "f32" else torch.float64
    return [a.to(td).double().cpu().numpy() for a in st]


def solver_at(n, dtype, bc, st, dt_fixed=0.0):
    s = sw.Solver(n, n, dtype=dtype, bc_x=bc, bc_y=bc, cfl=0.0 if dt_fixed > 0 else 0.5, dt_fixed=dt_fixed)
    s.set_state(*st)
    s.autotune(steps_per_trial=3, cache_path=CACHE)   # cache hit: bench.py's launch shape
    s.set_state(*st)
    s.reset_time()
    return s


@pytest.mark.parametrize("n,dtype,bc,seed", [(16384, "f32", sw.PERIODIC, ics.SEED_BUMPS_16384),
                                             (4096, "f32", sw.REFLECT, ics.SEED_BUMPS_4096),
                                             (4096, "f64", sw.REFLECT, ics.SEED_BUMPS_4096)])
def test_full_size_sampled_cells(n, dtype, bc, seed):
    """k fixed-dt steps at full size, sampled cells against oracle patches."""
    k = 12
    announce(f"full size {n}^2 {dtype} bc={bc}: {k} fixed-dt steps, sampled cells")
    st = ics.bumps_state(n, n, seed=seed, periodic=bc == sw.PERIODIC, count=8, device="cuda")
    hmax = float(st[0].max())
    dt = 0.5 / math.sqrt(G * hmax)
    s = solver_at(n, dtype, bc, st, dt_fixed=dt)
    s.step(k)
    cells = sample_cells(n, n, np.random.default_rng(seed), count=40, bumps=ics.draw_bumps(seed, n, n, count=8))
    got = gpu_cells(s, cells)
    ref0 = rounded_state(st, dtype)
    del s, st
    torch.cuda.empty_cache()
    refs = [patch_reference(ref0, x, y, k, dt, bc == sw.PERIODIC) for x, y in cells]
    ref = [np.array([r[f] for r in refs]) for f in range(3)]
    err = compare(got, ref, dtype)
    moved = int(np.sum(np.abs(got[1]) + np.abs(got[2]) > 0))
    print(f"{len(cells)} cells ({moved} with momentum), rel max-norm {err:.2e}")
    assert moved >= 8                      # at least the cells one sigma out from each bump


def test_full_size_cfl_step_and_200_step_run():
    """16384^2 FP32 periodic in CFL mode (the bandwidth-roofline workload):
    the first step's dt equals the oracle's from the global maximum signal
    speed, the cells after that step match oracle patches, and the 200-step
    run stays finite with its mass conserved to FP32 rounding."""
    n, k = 16384, 1
    announce("full size 16384^2 f32 periodic: CFL dt, one step, then 200 steps")
    st = ics.bumps_state(n, n, seed=ics.SEED_BUMPS_16384, periodic=True, count=8, device="cuda")
    s = solver_at(n, "f32", sw.PERIODIC, st)
    s.step(k)
    _, dt_gpu, steps = s.sync_status()
    cells = sample_cells(n, n, np.random.default_rng(7), count=32,
                         bumps=ics.draw_bumps(ics.SEED_BUMPS_16384, n, n, count=8))
    got = gpu_cells(s, cells)
    ref0 = rounded_state(st, "f32")
    H, U, V = (oracle.with_halo(a) for a in ref0)
    dt_ref = 0.5 / oracle.max_speed(H, U, V, G)
    del H, U, V
    assert steps == 1 and abs(dt_gpu - dt_ref) <= 1e-6 * dt_ref, (dt_gpu, dt_ref)
    refs = [patch_reference(ref0, x, y, k, dt_ref, True) for x, y in cells]
    compare(got, [np.array([r[f] for r in refs]) for f in range(3)], "f32")
    m0 = float(torch.from_numpy(ref0[0]).sum(dtype=torch.float64))
    del ref0
    s.state.cur = 0
    s.set_state(*st)
    s.reset_time()
    del st
    s.step(200)
    _, _, steps = s.sync_status()          # raises if the sticky flag is set
    m1 = float(s.interior(0).double().sum())
    assert steps == 200 and abs(m1 - m0) <= 1e-6 * m0, (m0, m1)


def test_batch_full_config_against_whole_grid_oracle():
    """The 512-grid batch (bench.py's configuration: CFL per grid, tuned tile
    table, one graph launch per call), 40 steps; the smallest, the largest and
    three random grids against whole-grid oracle runs in CFL mode."""
    k = 40
    sides = ics.batch_sides(512)
    announce(f"batch 512 grids full config, {k} steps, whole-grid oracle on 5 grids")
    b = sw.Batch(sides, dtype="f32")
    states = {}
    rng = np.random.default_rng(11)
    picks = {int(np.argmin(sides)), int(np.argmax(sides))} | {int(i) for i in rng.choice(512, 3, replace=False)}
    for i, n in enumerate(sides):
        st = ics.bumps_state(n, n, seed=ics.SEED_BATCH_GRID0 + i, periodic=False, device="cuda")
        b.set_state(i, *st)
        if i in picks:
            states[i] = rounded_state(st, "f32")
    b.autotune(steps_per_trial=3, cache_path=CACHE)
    b.step(k)
    t_gpu, steps, _ = b.sync_status()
    for i in sorted(picks):
        got = [a.cpu().numpy() for a in b.get_state(i)]
        H, U, V, t_ref = oracle.run(*states[i], k, g=G)
        err = compare(got, [H[1:-1, 1:-1], U[1:-1, 1:-1], V[1:-1, 1:-1]], "f32")
        assert steps[i] == k and abs(t_gpu[i] - t_ref) <= 1e-5 * t_ref
        print(f"grid {i} ({sides[i]}^2): rel max-norm {err:.2e}")


def test_surrogate_full_config_sampled_pixels():
    """The committed 256 x 256 network on a batch of 256 grids (the surrogate
    workload's batch), states after 8 solver steps: the normalised prediction
    at sampled pixels (corners, edges, random) against the network oracle on a
    15 x 15 patch around each (the receptive field is 13 x 13; patches are
    clipped at the grid edge, where the input ghosts follow the walls)."""
    n, size, R = 256, 256, 7
    announce("surrogate forward, 256 grids of 256^2, sampled pixels vs oracle patches")
    net, _ = surrogate.load_weights(surrogate.WEIGHTS_256, n)
    b = sw.Batch([(size, size)] * n, dtype="f32")
    b.load(surrogate.initial_states(n, size, size, ics.SEED_SURR_EVAL0 + 2000))
    b.step(8)
    u = b.export()
    delta = net.forward(u)
    params = net.get_params().cpu().numpy().astype(np.float64)
    off, scale = surrogate.IN_OFFSET, surrogate.IN_SCALE
    rng = np.random.default_rng(5)
    errs, scale_ref = [], 0.0
    for gi in rng.choice(n, 6, replace=False):
        ug = u[gi].cpu().numpy()
        for x, y in sample_cells(size, size, rng, count=8, tile_rows=4, tile_cols=64):
            x0, x1 = max(0, x - R), min(size, x + R + 1)
            y0, y1 = max(0, y - R), min(size, y + R + 1)
            _, d = no.forward(params, ug[None, :, y0:y1, x0:x1], off, scale, bf16_mode=True)
            want = d[0, y - y0, x - x0]
            got = delta[gi, y, x, :3].double().cpu().numpy()
            errs.append(np.max(np.abs(got - want)))
            scale_ref = max(scale_ref, float(np.max(np.abs(want))))
    print(f"{len(errs)} pixels: max abs err {max(errs):.2e} (scale {scale_ref:.2e})")
    assert max(errs) <= 1e-2 * scale_ref


def cached_tuning(key_tail):
    """The committed cache's launch shape for this GPU and `key_tail`."""
    p = torch.cuda.get_device_properties(0)
    key = f"{p.gcnArchName.split(':')[0]}:{p.multi_processor_count}:{key_tail}"
    best = None
    with open(CACHE) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] == key:
                best = dict(zip(("variant", "rows", "vec", "occupancy", "prefetch", "order"), map(int, parts[1:7])))
    return best


def test_full_size_blocked_and_comparison_variants():
    """The step variants bench.py times beside the headline, at 16384^2 FP32
    periodic with a fixed dt: the autotuner's fixed-dt choice (temporal
    blocking, K = 5), the fused kernel in the headline's tuned shape and the
    unfused and AoS steps give bitwise the same state after 12 steps (two
    blocked launches and two single steps); the kernels generated from region
    expressions (row march and LDS tiles) match oracle patches at sampled
    cells."""
    n, seed, k = 16384, ics.SEED_BUMPS_16384, 12
    announce(f"full size {n}^2 f32 periodic, fixed dt: blocked / fused / unfused / AoS / generated, {k} steps")
    st = ics.bumps_state(n, n, seed=seed, periodic=True, count=8, device="cuda")
    dt = 0.5 / math.sqrt(G * float(st[0].max()))
    s = solver_at(n, "f32", sw.PERIODIC, st, dt_fixed=dt)
    assert s.get_tuning()["variant"] == sw.VARIANT_TBLOCK
    s.step(k)
    first = [s.interior(i).clone() for i in range(3)]
    fused = cached_tuning(f"f32:0:{n}x{n}")
    assert fused and fused["variant"] == sw.VARIANT_FUSED
    for tun in (fused, {"variant": sw.VARIANT_UNFUSED}, {"variant": sw.VARIANT_AOS}):
        announce(f"full size variant {tun}")
        s.set_tuning(**tun)
        s.state.cur = 0
        s.set_state(*st)
        s.reset_time()
        s.step(k)
        assert all(torch.equal(s.interior(i), first[i]) for i in range(3)), tun
    del first
    cells = sample_cells(n, n, np.random.default_rng(seed + 1), count=32, tile_rows=8, tile_cols=62,
                         bumps=ics.draw_bumps(seed, n, n, count=8))
    got = {}
    for design in (2, 1):                      # the row march (default) and the paper's LDS tiles
        s.set_tuning(variant=sw.VARIANT_GENERATED, vec=design)
        s.state.cur = 0
        s.set_state(*st)
        s.reset_time()
        s.step(k)
        t, _, steps = s.sync_status()
        assert steps == k and abs(t - k * dt) <= 1e-12 * k * dt
        got[design] = gpu_cells(s, cells)
    ref0 = rounded_state(st, "f32")
    del s, st
    torch.cuda.empty_cache()
    refs = [patch_reference(ref0, x, y, k, dt, True) for x, y in cells]
    ref = [np.array([r[f] for r in refs]) for f in range(3)]
    for design, g in got.items():
        err = compare(g, ref, "f32")
        print(f"generated kernel, design {design}: {len(cells)} sampled cells, rel max-norm {err:.2e}")
