"""Temporal blocking (K steps per launch, fixed dt) on the GPU against the CPU
FP64 oracle: ragged grids spanning several tiles, both boundary rules and
their mix, step counts that leave a remainder for the single-step kernel,
grids narrower than the halo, mirror symmetry, and refusal in CFL mode.  The
blocked kernel repeats the fused kernel's arithmetic, so every blocked run
must also equal the same run through the fused single-step kernel bitwise."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1107_2157_amd import ics, sw
from swtest import G, announce, rel_maxnorm

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-5}
KS = {"f32": [3, 5, 7], "f64": [3, 5]}


def rounded(a, dtype):
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(torch.float32).to(torch.float64) if dtype == "f32" else t


def fixed_dt(h):
    return 0.5 / math.sqrt(G * float(torch.as_tensor(h).max())) * 0.9


def run_tb(state, nsteps, dtype, k, bc_x, bc_y, dt, variant=sw.VARIANT_TBLOCK, waves=0):
    h, hu, hv = (rounded(a, dtype) for a in state)
    ny, nx = h.shape
    announce(f"tblock {dtype} K={k} waves={waves} {nx}x{ny} steps={nsteps} bc=({bc_x},{bc_y}) variant={variant}")
    s = sw.Solver(nx, ny, g=G, dtype=dtype, bc_x=bc_x, bc_y=bc_y, cfl=0.0, dt_fixed=dt)
    if variant == sw.VARIANT_TBLOCK:
        s.set_tuning(variant=sw.VARIANT_TBLOCK, rows=k, vec=waves)
        assert s.get_tuning()["vec"] == (waves or (8 if dtype == "f64" else 16))
    else:
        s.set_variant(variant)
    s.set_state(h, hu, hv)
    s.step(nsteps)
    t, _, steps = s.sync_status()
    assert steps == nsteps and s.state.cur == nsteps & 1
    return s.get_state(), (h, hu, hv), t


def assert_bitwise_fused(got, state, nsteps, dtype, bc_x, bc_y, dt):
    fused, _, _ = run_tb(state, nsteps, dtype, 0, bc_x, bc_y, dt, variant=sw.VARIANT_FUSED)
    for a, b in zip(got, fused):
        assert torch.equal(a, b)


def oracle_run(state, nsteps, dt, bc_x, bc_y):
    H, U, V, t = oracle.run(*(a.numpy() for a in state), nsteps, g=G, dt_fixed=dt, bcx=bc_x, bcy=bc_y)
    return (H[1:-1, 1:-1], U[1:-1, 1:-1], V[1:-1, 1:-1]), t


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("bc", [(sw.REFLECT, sw.REFLECT), (sw.PERIODIC, sw.PERIODIC), (sw.REFLECT, sw.PERIODIC),
                                (sw.PERIODIC, sw.REFLECT)])
def test_blocked_matches_oracle(dtype, bc):
    nx, ny = 301, 203
    h, _, _ = ics.bumps_state(nx, ny, seed=7, periodic=False, count=4)
    _, hu, hv = ics.random_state(nx, ny, seed=9, amp_h=0.0, amp_m=0.02)
    dt = fixed_dt(h)
    for k in KS[dtype]:
        nsteps = 3 * k + 2                       # three blocked launches and two single steps
        got, start, t = run_tb((h, hu, hv), nsteps, dtype, k, bc[0], bc[1], dt)
        ref, t_ref = oracle_run(start, nsteps, dt, bc[0], bc[1])
        err = rel_maxnorm(got, ref)
        print(f"K={k} {dtype} bc={bc}: {err:.3e}")
        assert err <= TOL[dtype], (k, err)
        assert abs(t - t_ref) <= 1e-12 * t_ref
        assert_bitwise_fused(got, start, nsteps, dtype, bc[0], bc[1], dt)


@pytest.mark.parametrize("waves", [4, 8, 12, 16])
@pytest.mark.parametrize("dtype,k", [("f32", 5), ("f32", 7), ("f64", 3)])
def test_blocked_waves_per_tile(waves, dtype, k):
    """Every split of a tile's rows over 4, 8, 12 or 16 waves gives the same bits."""
    nx, ny = 333, 170
    h, _, _ = ics.bumps_state(nx, ny, seed=11, periodic=True, count=5)
    _, hu, hv = ics.random_state(nx, ny, seed=12, amp_h=0.0, amp_m=0.02)
    dt = fixed_dt(h)
    for bc in ((sw.PERIODIC, sw.REFLECT), (sw.REFLECT, sw.PERIODIC)):
        got, start, _ = run_tb((h, hu, hv), 2 * k + 1, dtype, k, bc[0], bc[1], dt, waves=waves)
        assert_bitwise_fused(got, start, 2 * k + 1, dtype, bc[0], bc[1], dt)


@pytest.mark.parametrize("dtype,k,waves", [("f32", 5, 16), ("f32", 3, 12), ("f64", 3, 8), ("f64", 5, 12)])
def test_blocked_walls_at_tile_and_chunk_edges(dtype, k, waves):
    """Grid sides one below, at and one above multiples of the tile's own
    width (64 - 2K) and height (staged rows - 2K), so reflective walls and
    their ghost cells fall on the first and last live lanes and on the rows
    where one wave's chunk meets the next."""
    tx = 64 - 2 * k
    ty = (98 if dtype == "f32" else 50) - 2 * k
    for nx, ny in ((2 * tx - 1, 2 * ty + 1), (2 * tx, 2 * ty), (2 * tx + 1, 2 * ty - 1), (tx + 3, ty - 3)):
        h, _, _ = ics.bumps_state(nx, ny, seed=nx + ny, periodic=False, count=3)
        _, hu, hv = ics.random_state(nx, ny, seed=nx * ny, amp_h=0.0, amp_m=0.02)
        dt = fixed_dt(h)
        for bc in ((sw.REFLECT, sw.REFLECT), (sw.PERIODIC, sw.REFLECT), (sw.REFLECT, sw.PERIODIC)):
            got, start, _ = run_tb((h, hu, hv), 2 * k + 1, dtype, k, bc[0], bc[1], dt, waves=waves)
            assert_bitwise_fused(got, start, 2 * k + 1, dtype, bc[0], bc[1], dt)
        ref, _ = oracle_run(start, 2 * k + 1, dt, sw.REFLECT, sw.PERIODIC)
        assert rel_maxnorm(got, ref) <= TOL[dtype], (nx, ny)


@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (2, 3), (5, 9), (64, 64), (65, 130), (257, 9)])
@pytest.mark.parametrize("bc", [sw.REFLECT, sw.PERIODIC])
def test_blocked_edge_shapes(shape, bc):
    nx, ny = shape
    st = ics.random_state(nx, ny, seed=nx * 131 + ny, amp_h=0.2, amp_m=0.05)
    dt = fixed_dt(st[0])
    for k in (3, 5):
        got, start, _ = run_tb(st, 2 * k + 1, "f64", k, bc, bc, dt)
        ref, _ = oracle_run(start, 2 * k + 1, dt, bc, bc)
        assert rel_maxnorm(got, ref) <= TOL["f64"], (shape, k)
        assert_bitwise_fused(got, start, 2 * k + 1, "f64", bc, bc, dt)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_blocked_mirror_symmetry_and_agreement_with_fused(dtype):
    """A centred dam break stays mirror-symmetric bitwise, and the blocked
    run equals the fused single-step run bitwise."""
    h, hu, hv = ics.dam_break_state(128)
    dt = fixed_dt(h)
    got, _, _ = run_tb((h, hu, hv), 25, dtype, 5, sw.REFLECT, sw.REFLECT, dt)
    H, U, V = (a.numpy() for a in got)
    assert np.array_equal(H, H[:, ::-1]) and np.array_equal(H, H[::-1, :])
    assert np.array_equal(U, -U[:, ::-1]) and np.array_equal(V, -V[::-1, :])
    assert_bitwise_fused(got, (h, hu, hv), 25, dtype, sw.REFLECT, sw.REFLECT, dt)


def test_blocked_refused_in_cfl_mode():
    s = sw.Solver(64, 64, dtype="f32")                       # CFL dt
    with pytest.raises(sw.SwError) as e:
        s.set_tuning(variant=sw.VARIANT_TBLOCK, rows=5)
    assert e.value.status == sw.ENOTSUP
    f = sw.Solver(64, 64, dtype="f32", cfl=0.0, dt_fixed=1e-3)
    for rows, waves in ((4, 8), (9, 8), (7, 8), (5, 2), (5, 32)):
        if rows == 7 and waves == 8:
            f.set_tuning(variant=sw.VARIANT_TBLOCK, rows=7, vec=8)   # K = 7 exists in FP32 only
            continue
        with pytest.raises(sw.SwError) as e:
            f.set_tuning(variant=sw.VARIANT_TBLOCK, rows=rows, vec=waves)
        assert e.value.status == sw.EINVAL, (rows, waves)
    d = sw.Solver(64, 64, dtype="f64", cfl=0.0, dt_fixed=1e-3)
    with pytest.raises(sw.SwError):
        d.set_tuning(variant=sw.VARIANT_TBLOCK, rows=7)
