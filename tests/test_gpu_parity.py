"""Parity of the HIP path (through the C ABI) with the CPU FP64 oracle.

Bars: GPU FP64 within 1e-12 relative max-norm of the oracle, GPU FP32 within
1e-5, after 100 steps, on the same seeded inputs.  FP32 runs start from the
FP32-rounded initial state, which the oracle then advances in FP64.
"""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1107_2157_amd import ics, sw
from swtest import G, announce, rel_maxnorm

pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
VARIANTS = [sw.VARIANT_CELL, sw.VARIANT_FUSED]
BCS = [sw.REFLECT, sw.PERIODIC]
SCHEMES = [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE]


def rounded(a, dtype):
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(torch.float32).to(torch.float64) if dtype == "f32" else t


def run_both(state, nsteps, dtype, variant, bc_x=sw.REFLECT, bc_y=sw.REFLECT, scheme=sw.SCHEME_PAPER,
             dx=1.0, dy=1.0, cfl=0.5, dt_fixed=0.0):
    h, hu, hv = (rounded(a, dtype) for a in state)
    ny, nx = h.shape
    announce(f"{dtype} variant={variant} {nx}x{ny} steps={nsteps} bc=({bc_x},{bc_y}) scheme={scheme}")
    s = sw.Solver(nx, ny, g=G, dx=dx, dy=dy, dtype=dtype, bc_x=bc_x, bc_y=bc_y, scheme=scheme,
                  cfl=cfl, dt_fixed=dt_fixed, variant=variant)
    s.set_state(h, hu, hv)
    s.step(nsteps)
    t_gpu, _, steps = s.sync_status()
    got = s.get_state()
    H, U, V, t_ref = oracle.run(h.numpy(), hu.numpy(), hv.numpy(), nsteps, g=G, dx=dx, dy=dy, cfl=cfl,
                                dt_fixed=dt_fixed, scheme=scheme, bcx=bc_x, bcy=bc_y)
    ref = (H[1:-1, 1:-1], U[1:-1, 1:-1], V[1:-1, 1:-1])
    assert steps == nsteps
    return got, ref, t_gpu, t_ref, s


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_dam_break_128(variant, dtype):
    """FP64 dam break: 128^2, reflective walls, CFL 0.5, 100 steps."""
    got, ref, t_gpu, t_ref, _ = run_both(ics.dam_break_state(128), 100, dtype, variant)
    err = rel_maxnorm(got, ref)
    print(f"dam break {dtype} variant {variant}: rel max-norm {err:.3e}")
    assert err <= TOL[dtype]
    assert abs(t_gpu - t_ref) / t_ref <= (1e-13 if dtype == "f64" else 1e-5)


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("bc", BCS)
@pytest.mark.parametrize("scheme", SCHEMES)
def test_bumps_ragged(variant, dtype, bc, scheme):
    """Gaussian bumps plus moving water on a ragged grid spanning several
    tiles in both directions, both schemes."""
    nx, ny = 301, 203
    h, _, _ = ics.bumps_state(nx, ny, seed=7, periodic=bc == sw.PERIODIC, count=4)
    _, hu, hv = ics.random_state(nx, ny, seed=9, amp_h=0.0, amp_m=0.02)
    got, ref, _, _, _ = run_both((h, hu, hv), 100, dtype, variant, bc_x=bc, bc_y=bc, scheme=scheme)
    err = rel_maxnorm(got, ref)
    print(f"bumps {dtype} v{variant} bc{bc} s{scheme}: {err:.3e}")
    assert err <= TOL[dtype]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("shape", [(1, 1), (1, 37), (37, 1), (2, 3), (63, 5), (64, 64), (65, 130), (257, 9)])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("scheme", SCHEMES)
def test_edge_shapes(variant, shape, dtype, scheme):
    """Degenerate and ragged grids (single rows/columns, one cell, exact and
    off-by-one tile multiples), mixed boundary conditions (the transverse
    scheme reads the corner ghosts), random moving state."""
    nx, ny = shape
    st = ics.random_state(nx, ny, seed=nx * 1000 + ny, amp_h=0.2, amp_m=0.05)
    for bc_x, bc_y in ((sw.REFLECT, sw.PERIODIC), (sw.PERIODIC, sw.REFLECT), (sw.REFLECT, sw.REFLECT),
                       (sw.PERIODIC, sw.PERIODIC)):
        got, ref, _, _, _ = run_both(st, 40, dtype, variant, bc_x=bc_x, bc_y=bc_y, dx=1.0, dy=0.7, scheme=scheme)
        assert rel_maxnorm(got, ref) <= TOL[dtype], (shape, bc_x, bc_y)


@pytest.mark.parametrize("variant", VARIANTS)
def test_fixed_dt_mode(variant):
    st = ics.random_state(50, 40, seed=3, amp_h=0.2, amp_m=0.05)
    got, ref, t_gpu, t_ref, _ = run_both(st, 30, "f64", variant, dt_fixed=0.01, cfl=0.0)
    assert rel_maxnorm(got, ref) <= 1e-12
    assert t_gpu == pytest.approx(0.3, rel=1e-14)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_fill_halo_matches_oracle(dtype):
    nx, ny = 37, 23
    st = [rounded(a, dtype) for a in ics.random_state(nx, ny, seed=4)]
    for bc_x in BCS:
        for bc_y in BCS:
            announce(f"fill_halo {dtype} bc=({bc_x},{bc_y})")
            s = sw.Solver(nx, ny, dtype=dtype, bc_x=bc_x, bc_y=bc_y)
            s.set_state(*st)
            s.fill_halo()
            got = s.get_state(halo=True)
            H, U, V = (oracle.with_halo(a.numpy()) for a in st)
            oracle.fill_halo(H, U, V, bc_x, bc_y)
            for g_, r_ in zip(got, (H, U, V)):
                assert np.array_equal(g_.numpy(), r_)


@pytest.mark.parametrize("variant", VARIANTS)
def test_halo_after_step_is_filled(variant):
    """After sw_step the halo of buf[cur] holds the boundary values of the new
    interior (the kernel writes them as it produces the edge cells)."""
    nx, ny = 70, 33
    st = ics.random_state(nx, ny, seed=6)
    for bc_x, bc_y in ((sw.REFLECT, sw.REFLECT), (sw.PERIODIC, sw.REFLECT), (sw.PERIODIC, sw.PERIODIC)):
        s = sw.Solver(nx, ny, dtype="f64", bc_x=bc_x, bc_y=bc_y, variant=variant)
        s.set_state(*st)
        s.step(3)
        got = [a.numpy().copy() for a in s.get_state(halo=True)]
        H, U, V = (a.copy() for a in got)
        oracle.fill_halo(H, U, V, bc_x, bc_y)
        for g_, r_ in zip(got, (H, U, V)):
            assert np.array_equal(g_, r_)


def test_variants_agree_to_rounding():
    st = ics.bumps_state(513, 257, seed=12, periodic=False, count=6)
    outs = []
    for v in VARIANTS:
        s = sw.Solver(513, 257, dtype="f64", variant=v)
        s.set_state(*st)
        s.step(50)
        outs.append(s.get_state())
    assert rel_maxnorm(outs[0], outs[1]) <= 1e-13
