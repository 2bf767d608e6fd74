"""sw_diagnostics on the GPU: the conserved sums, the max signal speed, the
min depth and the non-finite count of buf[cur], against numpy / the oracle
on the same state; bitwise repeatable; and mass conservation over a
periodic run measured through the library itself."""
import math

import numpy as np
import pytest
import torch

import oracle
from paper_1107_2157_amd import ics, sw
from swtest import G, announce

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("shape", [(1, 1), (300, 7), (1031, 517)])
def test_diagnostics_match_numpy(dtype, shape):
    nx, ny = shape
    announce(f"diagnostics {dtype} {nx}x{ny}")
    h, hu, hv = ics.random_state(nx, ny, seed=nx + 3 * ny, amp_h=0.3, amp_m=0.1)
    s = sw.Solver(nx, ny, g=G, dtype=dtype)
    s.set_state(h, hu, hv)
    d = s.diagnostics()
    H, U, V = (x.numpy() for x in s.get_state())            # the state as stored (rounded in FP32)
    n = H.size
    for key, ref in (("mass", H.sum()), ("sum_hu", U.sum()), ("sum_hv", V.sum())):
        scale = np.abs({"mass": H, "sum_hu": U, "sum_hv": V}[key]).sum()
        assert abs(d[key] - ref) <= 1e-13 * scale + 1e-300, key
    assert d["min_h"] == H.min()
    assert d["nonfinite"] == 0
    Hh, Uh, Vh = (oracle.with_halo(a) for a in (H, U, V))
    smax = oracle.max_speed(Hh, Uh, Vh, G)
    assert abs(d["max_speed"] - smax) <= (1e-6 if dtype == "f32" else 1e-14) * smax
    assert s.diagnostics() == d                               # bitwise repeatable
    assert n == nx * ny


def test_diagnostics_count_nonfinite_and_negative_depth():
    nx, ny = 64, 40
    h, hu, hv = ics.random_state(nx, ny, seed=5, amp_h=0.2, amp_m=0.05)
    s = sw.Solver(nx, ny, g=G, dtype="f64")
    s.set_state(h, hu, hv)
    s.interior(0)[3, 7] = float("nan")
    s.interior(2)[10, 11] = float("inf")
    s.interior(0)[20, 30] = -0.5
    d = s.diagnostics()
    assert d["nonfinite"] == 2 and d["min_h"] == -0.5
    assert math.isnan(d["mass"])


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-6)])
def test_mass_conserved_through_the_library(dtype, tol):
    """Periodic walls: the sum of h is conserved by the flux form (to
    rounding); reflective walls also conserve it (no flux through a wall)."""
    n = 257
    for bc in (sw.PERIODIC, sw.REFLECT):
        st = ics.bumps_state(n, n, seed=9, periodic=bc == sw.PERIODIC, count=4)
        s = sw.Solver(n, n, g=G, dtype=dtype, bc_x=bc, bc_y=bc)
        s.set_state(*st)
        m0 = s.diagnostics()["mass"]
        s.step(200)
        s.sync_status()
        m1 = s.diagnostics()["mass"]
        assert abs(m1 - m0) <= tol * m0, (bc, m0, m1)
