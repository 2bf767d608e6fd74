"""The paper's comparison designs on the GPU (section "Performance
Measurements"): the unfused step (face states of the first half-step through
HBM, two kernels) and the AoS step (one (h, hu, hv, 0) vector per cell).
Both repeat the fused kernel's arithmetic, so every run must equal the same
run through the fused kernel bitwise (state with halo, time, dt, step count)
in CFL and fixed-dt mode, for both boundary rules and their mix, ragged and
degenerate grids; one case per dtype is also held against the CPU oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1107_2157_amd import ics, sw
from swtest import G, announce, rel_maxnorm

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-5}
VARIANTS = [sw.VARIANT_UNFUSED, sw.VARIANT_AOS]


def rounded(a, dtype):
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(torch.float32).to(torch.float64) if dtype == "f32" else t


def run(state, nsteps, dtype, bc, variant, dt_fixed=0.0, rows=0, solver=None):
    h, hu, hv = (rounded(a, dtype) for a in state)
    ny, nx = h.shape
    announce(f"compare variant={variant} {dtype} {nx}x{ny} steps={nsteps} bc={bc} dt_fixed={dt_fixed} rows={rows}")
    s = solver or sw.Solver(nx, ny, g=G, dtype=dtype, bc_x=bc[0], bc_y=bc[1],
                            cfl=0.0 if dt_fixed else 0.5, dt_fixed=dt_fixed)
    s.set_tuning(variant=variant, rows=rows)
    s.state.cur = 0
    s.set_state(h, hu, hv)
    s.reset_time()
    s.step(nsteps)
    status = s.sync_status()
    return [x.numpy() for x in s.get_state(halo=True)], status, s


def assert_same(a, b):
    (sa, ta), (sb, tb) = a[:2], b[:2]
    for x, y in zip(sa, sb):
        assert np.array_equal(x, y)
    assert ta == tb


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("bc", [(sw.REFLECT, sw.REFLECT), (sw.PERIODIC, sw.PERIODIC), (sw.PERIODIC, sw.REFLECT)])
@pytest.mark.parametrize("fixed", [False, True])
def test_bitwise_equal_to_fused(dtype, bc, fixed):
    nx, ny = 301, 203
    h, _, _ = ics.bumps_state(nx, ny, seed=17, periodic=False, count=4)
    _, hu, hv = ics.random_state(nx, ny, seed=19, amp_h=0.0, amp_m=0.02)
    dt = 0.5 / math.sqrt(G * float(h.max())) * 0.9 if fixed else 0.0
    fused = run((h, hu, hv), 13, dtype, bc, sw.VARIANT_FUSED, dt)
    for v in VARIANTS:
        assert_same(run((h, hu, hv), 13, dtype, bc, v, dt), fused)


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (63, 2), (64, 64), (65, 130), (130, 65)])
@pytest.mark.parametrize("bc", [sw.REFLECT, sw.PERIODIC])
def test_edge_shapes(shape, bc):
    nx, ny = shape
    st = ics.random_state(nx, ny, seed=nx * 7 + ny, amp_h=0.2, amp_m=0.05)
    fused = run(st, 5, "f64", (bc, bc), sw.VARIANT_FUSED)
    for v in VARIANTS:
        assert_same(run(st, 5, "f64", (bc, bc), v), fused)
    for rows in (1, 3):
        assert_same(run(st, 5, "f64", (bc, bc), sw.VARIANT_AOS, rows=rows), fused)


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_against_oracle(dtype):
    nx, ny = 130, 97
    h, _, _ = ics.bumps_state(nx, ny, seed=23, periodic=False, count=3)
    _, hu, hv = ics.random_state(nx, ny, seed=29, amp_h=0.0, amp_m=0.02)
    start = tuple(rounded(a, dtype) for a in (h, hu, hv))
    H, U, V, t_ref = oracle.run(*(a.numpy() for a in start), 40, g=G, cfl=0.5, bcx=sw.REFLECT, bcy=sw.PERIODIC)
    ref = (H[1:-1, 1:-1], U[1:-1, 1:-1], V[1:-1, 1:-1])
    for v in VARIANTS:
        got, (t, _, steps), _ = run(start, 40, dtype, (sw.REFLECT, sw.PERIODIC), v)
        assert steps == 40
        assert rel_maxnorm([x[1:-1, 1:-1] for x in got], ref) <= TOL[dtype]
        assert abs(t - t_ref) <= (1e-12 if dtype == "f64" else 1e-5) * t_ref


def test_workspace_grows_and_other_variants_stay_exact():
    """One context runs the unfused step (face planes), then AoS (a larger
    workspace, reallocated), then the fused kernel again: all agree."""
    n = 200
    st = ics.bumps_state(n, n, seed=31, periodic=True, count=2)
    first = run(st, 7, "f32", (sw.PERIODIC, sw.PERIODIC), sw.VARIANT_FUSED)
    s = first[2]
    for v in (sw.VARIANT_UNFUSED, sw.VARIANT_AOS, sw.VARIANT_UNFUSED, sw.VARIANT_FUSED):
        assert_same(run(st, 7, "f32", (sw.PERIODIC, sw.PERIODIC), v, solver=s), first)
    s.set_graph(False)                                   # eager launches: the same bits
    assert_same(run(st, 7, "f32", (sw.PERIODIC, sw.PERIODIC), sw.VARIANT_AOS, solver=s), first)


def test_refusals():
    s = sw.Solver(32, 16, dtype="f32", scheme=sw.SCHEME_TRANSVERSE)
    for v in VARIANTS:
        with pytest.raises(sw.SwError) as e:
            s.set_tuning(variant=v)
        assert e.value.status == sw.ENOTSUP
    f = sw.Solver(32, 16, dtype="f32")
    with pytest.raises(sw.SwError) as e:
        f.set_tuning(variant=sw.VARIANT_AOS, rows=-1)
    assert e.value.status == sw.EINVAL
    with pytest.raises(sw.SwError) as e:
        f.set_tuning(variant=7)
    assert e.value.status == sw.EINVAL
