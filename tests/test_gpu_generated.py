"""The step kernel generated from region expressions (sw_step variant 6) on
the GPU against the CPU FP64 oracle: ragged grids spanning several 64 x 8
tiles, both boundary rules and their mix, CFL and fixed dt, degenerate
shapes; and against the fused kernel, to rounding."""
import math

import pytest
import torch

import oracle
from paper_1107_2157_amd import ics, sw
from swtest import G, announce, rel_maxnorm

pytestmark = pytest.mark.gpu
TOL = {"f64": 1e-12, "f32": 1e-5}


def rounded(a, dtype):
    t = torch.as_tensor(a, dtype=torch.float64)
    return t.to(torch.float32).to(torch.float64) if dtype == "f32" else t


def run(state, nsteps, dtype, bc, variant, dt_fixed=0.0, design=0):
    h, hu, hv = (rounded(a, dtype) for a in state)
    ny, nx = h.shape
    announce(f"generated variant={variant} design={design} {dtype} {nx}x{ny} steps={nsteps} bc={bc} "
             f"dt_fixed={dt_fixed}")
    s = sw.Solver(nx, ny, g=G, dtype=dtype, bc_x=bc[0], bc_y=bc[1], cfl=0.0 if dt_fixed else 0.5,
                  dt_fixed=dt_fixed, variant=variant)
    if design:
        s.set_tuning(variant=variant, vec=design)
    s.set_state(h, hu, hv)
    s.step(nsteps)
    t, _, steps = s.sync_status()
    assert steps == nsteps
    return s.get_state(halo=True), (h, hu, hv), t


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("bc", [(sw.REFLECT, sw.REFLECT), (sw.PERIODIC, sw.PERIODIC), (sw.REFLECT, sw.PERIODIC),
                                (sw.PERIODIC, sw.REFLECT)])
@pytest.mark.parametrize("fixed", [False, True])
@pytest.mark.parametrize("design", [1, 2])
def test_generated_matches_oracle(dtype, bc, fixed, design):
    nx, ny = 301, 203
    h, _, _ = ics.bumps_state(nx, ny, seed=41, periodic=False, count=4)
    _, hu, hv = ics.random_state(nx, ny, seed=43, amp_h=0.0, amp_m=0.02)
    dt = 0.5 / math.sqrt(G * float(h.max())) * 0.9 if fixed else 0.0
    got, start, t = run((h, hu, hv), 100, dtype, bc, sw.VARIANT_GENERATED, dt, design)
    H, U, V, t_ref = oracle.run(*(a.numpy() for a in start), 100, g=G, cfl=0.0 if fixed else 0.5, dt_fixed=dt,
                                bcx=bc[0], bcy=bc[1])
    err = rel_maxnorm([x[1:-1, 1:-1] for x in got], (H[1:-1, 1:-1], U[1:-1, 1:-1], V[1:-1, 1:-1]))
    print(f"{dtype} bc={bc} fixed={fixed}: {err:.3e}")
    assert err <= TOL[dtype]
    assert abs(t - t_ref) <= (1e-12 if dtype == "f64" else 1e-5) * t_ref
    # the halo of the result holds the boundary values of the new state
    herr = rel_maxnorm(got, (H, U, V))
    assert herr <= TOL[dtype]
    fused, _, _ = run((h, hu, hv), 100, dtype, bc, sw.VARIANT_FUSED, dt)
    assert rel_maxnorm(got, fused) <= TOL[dtype]


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (61, 7), (62, 8), (63, 7), (64, 8), (65, 9), (124, 33),
                                   (130, 17)])
@pytest.mark.parametrize("bc", [sw.REFLECT, sw.PERIODIC])
@pytest.mark.parametrize("design", [1, 2])
def test_generated_edge_shapes(shape, bc, design):
    nx, ny = shape
    st = ics.random_state(nx, ny, seed=nx * 13 + ny, amp_h=0.2, amp_m=0.05)
    got, start, _ = run(st, 9, "f64", (bc, bc), sw.VARIANT_GENERATED, design=design)
    H, U, V, _ = oracle.run(*(a.numpy() for a in start), 9, g=G, cfl=0.5, bcx=bc, bcy=bc)
    assert rel_maxnorm(got, (H, U, V)) <= TOL["f64"], shape


@pytest.mark.parametrize("design,rows,prefetch", [(1, 4, 0), (1, 16, 0), (2, 4, 2), (2, 8, 3), (2, 16, 1),
                                                 (2, 32, 3)])
def test_generated_tile_heights(design, rows, prefetch):
    """Every instantiated tile height (LDS design) or march length and
    input prefetch depth (row march) gives the same bits as the default
    shape of its design."""
    nx, ny = 150, 70
    st = ics.random_state(nx, ny, seed=71, amp_h=0.2, amp_m=0.04)
    ref, _, _ = run(st, 9, "f32", (sw.PERIODIC, sw.REFLECT), sw.VARIANT_GENERATED, design=design)
    h, hu, hv = (rounded(a, "f32") for a in st)
    s = sw.Solver(nx, ny, g=G, dtype="f32", bc_x=sw.PERIODIC, bc_y=sw.REFLECT)
    s.set_tuning(variant=sw.VARIANT_GENERATED, rows=rows, vec=design, prefetch=prefetch)
    assert s.get_tuning()["prefetch"] == (prefetch or 0)
    s.set_state(h, hu, hv)
    s.step(9)
    for a, b in zip(s.get_state(halo=True), ref):
        assert torch.equal(a, b)
    for bad in (dict(rows=5), dict(prefetch=4 if design == 2 else 1)):
        with pytest.raises(sw.SwError) as e:
            s.set_tuning(variant=sw.VARIANT_GENERATED, vec=design, **bad)
        assert e.value.status == sw.EINVAL


def test_generated_refused_for_the_transverse_scheme():
    s = sw.Solver(32, 16, dtype="f32", scheme=sw.SCHEME_TRANSVERSE)
    with pytest.raises(sw.SwError) as e:
        s.set_tuning(variant=sw.VARIANT_GENERATED)
    assert e.value.status == sw.ENOTSUP


def test_tall_grids_refused_by_tiled_variants():
    """More than 65535 rows of tiles: the generated kernel (4-row tiles) and
    the blocked kernel (FP64, K = 5: 40-row tiles) refuse with SW_ENOTSUP
    when the shape is chosen, instead of failing at launch."""
    s = sw.Solver(1, 65535 * 4 + 1, g=G, dtype="f32")
    with pytest.raises(sw.SwError) as e:
        s.set_tuning(variant=sw.VARIANT_GENERATED, rows=4, vec=1)
    assert e.value.status == sw.ENOTSUP
    s.set_tuning(variant=sw.VARIANT_GENERATED, rows=4, vec=2)   # the row march has no such limit
    s.set_tuning(variant=sw.VARIANT_GENERATED, rows=8, vec=1)   # 32768 rows of tiles: fine
    del s
    b = sw.Solver(1, 65535 * 40 + 1, g=G, dtype="f64", cfl=0.0, dt_fixed=1e-3)
    with pytest.raises(sw.SwError) as e:
        b.set_tuning(variant=sw.VARIANT_TBLOCK, rows=5)
    assert e.value.status == sw.ENOTSUP
    b.set_tuning(variant=sw.VARIANT_TBLOCK, rows=3)             # 44-row tiles: 59580 rows of tiles
