"""Invariants of the scheme checked on the GPU path (through the C ABI):
lake at rest (bitwise), mass conservation, mirror symmetry of a centred dam
break (bitwise), determinism, the sticky instability flag, and the linear
gravity-wave speed sqrt(g H) through the fused, blocked and generated
kernels."""
import math

import numpy as np
import pytest
import torch

from paper_1107_2157_amd import ics, sw
from swtest import G, announce

pytestmark = pytest.mark.gpu
VARIANTS = [sw.VARIANT_CELL, sw.VARIANT_FUSED]


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_lake_at_rest_bitwise(variant, dtype, scheme):
    for bc in (sw.REFLECT, sw.PERIODIC):
        announce(f"lake at rest {dtype} v{variant} s{scheme} bc{bc}")
        s = sw.Solver(129, 65, dtype=dtype, bc_x=bc, bc_y=bc, scheme=scheme, variant=variant)
        h = torch.full((65, 129), 1.37, dtype=torch.float64)
        s.set_state(h, torch.zeros_like(h), torch.zeros_like(h))
        s.step(50)
        H, U, V = s.get_state()
        want = torch.tensor(1.37, dtype=s.torch_dtype).item()
        assert bool((H == want).all()) and bool((U == 0).all()) and bool((V == 0).all())


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_mirror_symmetry_bitwise(variant, dtype, scheme):
    """Both transverse terms are odd or even under each mirror exactly as the
    fluxes they correct, and every fma is written so that negating its
    operands negates it, so the fused transverse step keeps the dam break's
    mirror symmetry bit for bit as the paper scheme does."""
    announce(f"mirror {dtype} v{variant} s{scheme}")
    s = sw.Solver(128, 128, dtype=dtype, variant=variant, scheme=scheme)
    s.set_state(*ics.dam_break_state(128))
    s.step(100)
    H, U, V = (a.numpy() for a in s.get_state())
    assert np.array_equal(H, H[:, ::-1]) and np.array_equal(U, -U[:, ::-1]) and np.array_equal(V, V[:, ::-1])
    assert np.array_equal(H, H[::-1, :]) and np.array_equal(U, U[::-1, :]) and np.array_equal(V, -V[::-1, :])


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-6)])
@pytest.mark.parametrize("bc", [sw.REFLECT, sw.PERIODIC])
@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_mass_conservation(variant, dtype, tol, bc, scheme):
    announce(f"mass {dtype} v{variant} bc{bc} s{scheme}")
    n = 512
    st = ics.bumps_state(n, n, seed=21, periodic=bc == sw.PERIODIC, count=8)
    s = sw.Solver(n, n, dtype=dtype, bc_x=bc, bc_y=bc, variant=variant, scheme=scheme)
    s.set_state(*st)
    m0 = math.fsum(s.get_state()[0].numpy().ravel())
    s.step(100)
    m1 = math.fsum(s.get_state()[0].numpy().ravel())
    assert abs(m1 - m0) / m0 <= tol


@pytest.mark.parametrize("variant", VARIANTS)
def test_deterministic_bitwise(variant):
    st = ics.bumps_state(700, 300, seed=5, periodic=True, count=8)
    outs = []
    for _ in range(2):
        s = sw.Solver(700, 300, dtype="f32", bc_x=sw.PERIODIC, bc_y=sw.PERIODIC, variant=variant)
        s.set_state(*st)
        s.step(60)
        outs.append([a.numpy() for a in s.get_state(halo=True)] + [s.sync_status()])
    for a, b in zip(outs[0][:3], outs[1][:3]):
        assert np.array_equal(a, b)
    assert outs[0][3] == outs[1][3]


@pytest.mark.parametrize("variant", VARIANTS)
def test_negative_depth_sets_sticky_flag(variant):
    s = sw.Solver(40, 30, dtype="f32", variant=variant, dt_fixed=0.01, cfl=0.0)
    h = torch.ones((30, 40), dtype=torch.float64)
    h[10, 20] = -1.0
    s.set_state(h, torch.zeros_like(h), torch.zeros_like(h))
    s.step(2)
    with pytest.raises(sw.Unstable):
        s.sync_status()
    s.reset_time()
    s.set_state(torch.ones_like(h), torch.zeros_like(h), torch.zeros_like(h))
    s.step(2)
    t, dt, n = s.sync_status()
    assert n == 2 and t == pytest.approx(0.02)


def test_step_zero_and_cur_flip():
    s = sw.Solver(16, 16, dtype="f64")
    s.set_state(*ics.dam_break_state(16))
    s.step(0)
    assert s.state.cur == 0
    s.step(3)
    assert s.state.cur == 1
    s.step(1)
    assert s.state.cur == 0


@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_fused_tunings_bitwise_identical(scheme):
    """Every fused launch shape (cells per lane, rows per tile, register
    budget, prefetch depth, tile order) computes each cell with the same arithmetic: results are bitwise equal,
    including the halo and the simulated time."""
    nx, ny = 531, 190
    for dtype, vecs in (("f32", (2, 4)), ("f64", (1, 2))):
        st = ics.bumps_state(nx, ny, seed=31, periodic=False, count=5)
        ref = None
        ran = 0
        for vec in vecs:
            for occ in (0, 3, 4):
                for pd in (1, 2, 3):
                    for rows, order in ((7, 0), (16, 1), (64, 2), (5, 1), (3, 0), (2, 2)):
                        s = sw.Solver(nx, ny, dtype=dtype, scheme=scheme)
                        try:
                            s.set_tuning(variant=sw.VARIANT_FUSED, rows=rows, vec=vec, occupancy=occ, prefetch=pd, order=order)
                        except sw.SwError as e:
                            assert e.status == sw.EINVAL
                            continue
                        announce(f"tuning {dtype} s{scheme} vec={vec} occ={occ} pd={pd} rows={rows} order={order}")
                        s.set_state(*st)
                        s.step(25)
                        out = [a.numpy() for a in s.get_state(halo=True)] + [s.sync_status()]
                        ran += 1
                        if ref is None:
                            ref = out
                        else:
                            for x, y in zip(ref[:3], out[:3]):
                                assert np.array_equal(x, y), (dtype, vec, occ, pd, rows)
                            assert ref[3] == out[3]
        assert ran >= (40 if scheme == sw.SCHEME_PAPER else 20)


def test_fused_tile_span_limit():
    """The fused kernel reaches a tile's rows through 32-bit buffer offsets.
    On the widest grid (nx = 2^21, FP64: 50 MB from one row of a plane to the
    next, three planes interleaved) 40 rows per tile fit below 2 GiB and 41
    are refused when the shape is chosen."""
    s = sw.Solver(2 ** 21, 1, dtype="f64")
    assert s.layout.pitch * 8 * 42 <= 2 ** 31 - 1 < s.layout.pitch * 8 * 43
    s.set_tuning(variant=sw.VARIANT_FUSED, rows=40)
    with pytest.raises(sw.SwError) as e:
        s.set_tuning(variant=sw.VARIANT_FUSED, rows=41)
    assert e.value.status == sw.EINVAL


@pytest.mark.parametrize("variant", [sw.VARIANT_FUSED, sw.VARIANT_TBLOCK, sw.VARIANT_UNFUSED, sw.VARIANT_AOS,
                                     sw.VARIANT_GENERATED])
def test_separate_plane_allocations_step_like_interleaved(variant):
    """The library's layout interleaves the rows of h, hu and hv in one
    allocation per buffer; planes placed in six separate allocations of
    plane_elems elements each are stepped to bitwise the same state."""
    nx, ny = 300, 77
    st = ics.bumps_state(nx, ny, seed=33, periodic=False, count=4)
    dt = 0.1 if variant == sw.VARIANT_TBLOCK else 0.0
    kw = dict(dtype="f32", bc_x=sw.PERIODIC, bc_y=sw.REFLECT, cfl=0.0 if dt else 0.5, dt_fixed=dt)
    announce(f"separate planes variant={variant}")
    a = sw.Solver(nx, ny, variant=variant, **kw)
    b = sw.Solver(nx, ny, variant=variant, **kw)
    L = b.layout
    planes = [[torch.zeros(L.plane_elems, dtype=torch.float32, device="cuda") for _ in range(3)] for _ in range(2)]
    for buf in range(2):
        for k in range(3):
            b.state.plane[buf][k] = planes[buf][k].data_ptr()

    def halo_view(k, buf=None):
        p = planes[b.state.cur if buf is None else buf][k]
        return torch.as_strided(p, (ny + 2, nx + 2), (L.pitch, 1), L.origin - L.pitch - 1)
    b.halo_view = halo_view
    for s in (a, b):
        s.set_state(*st)
        s.step(11)
    for x, y in zip(a.get_state(halo=True), b.get_state(halo=True)):
        assert torch.equal(x, y)
    assert a.sync_status() == b.sync_status()


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_restart_and_checkpoint_are_bitwise(variant, dtype):
    """30 steps in one call == 10 + 20 steps in two calls == 10 steps, a
    checkpoint through the host, a fresh solver, 20 more steps."""
    st = ics.bumps_state(300, 200, seed=8, periodic=True, count=6)
    kw = dict(dtype=dtype, bc_x=sw.PERIODIC, bc_y=sw.PERIODIC, variant=variant)
    a = sw.Solver(300, 200, **kw)
    a.set_state(*st)
    a.step(30)
    ta = a.sync_status()[0]
    b = sw.Solver(300, 200, **kw)
    b.set_state(*st)
    b.step(10)
    b.step(20)
    assert [x.numpy().tobytes() for x in a.get_state(halo=True)] == [x.numpy().tobytes() for x in b.get_state(halo=True)]
    assert b.sync_status()[0] == ta
    c1 = sw.Solver(300, 200, **kw)
    c1.set_state(*st)
    c1.step(10)
    t1 = c1.sync_status()[0]
    saved = c1.get_state()
    c2 = sw.Solver(300, 200, **kw)
    c2.set_state(*saved)
    c2.step(20)
    t2 = c2.sync_status()[0]
    for x, y in zip(a.get_state(), c2.get_state()):
        assert torch.equal(x, y)
    assert abs((t1 + t2) - ta) <= 1e-12 * ta


@pytest.mark.parametrize("variant", VARIANTS)
@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_graph_replays_equal_eager_launches(variant, dtype):
    """sw_step replayed as hipGraphs equals eager launches bitwise, call after
    call: odd call lengths alternate the current buffer, so two graphs are
    each replayed several times, with eager torch work and host reads of the
    state and time between the replays."""
    announce(f"graph replays {dtype} v{variant}")
    st = ics.random_state(192, 130, seed=12)
    kw = dict(dtype=dtype, bc_x=sw.REFLECT, bc_y=sw.PERIODIC, variant=variant)
    runs = []
    for graph in (False, True):
        s = sw.Solver(192, 130, **kw)
        s.set_graph(graph)
        s.set_state(*st)
        out = []
        for k in range(6):
            s.step(7)
            h, hu, hv = s.get_state(halo=True)
            torch.randn(4096, device="cuda").cumsum(0).sum().item()   # unrelated eager work and a sync
            out.append((h.numpy().tobytes(), hu.numpy().tobytes(), hv.numpy().tobytes(), s.sync_status()))
        runs.append(out)
    for k, (e, g) in enumerate(zip(*runs)):
        assert e[:3] == g[:3], f"call {k}"
        assert e[3] == g[3], f"call {k}: time / step counters"


def _peak(profile, lo, hi):
    k = lo + int(np.argmax(profile[lo:hi]))
    ym, y0, yp = profile[k - 1], profile[k], profile[k + 1]
    return k + 0.5 * (ym - yp) / (ym - 2 * y0 + yp)


@pytest.mark.parametrize("variant", [sw.VARIANT_FUSED, sw.VARIANT_TBLOCK, sw.VARIANT_GENERATED])
@pytest.mark.parametrize("axis", ["x", "y"])
def test_linear_gravity_wave_speed(variant, axis):
    """A small Gaussian rise on still water of depth 1 splits into two pulses
    moving at sqrt(g H): the right-moving peak's speed between steps 400 and
    1200 (fixed dt, periodic walls, FP64) is within 1 % of sqrt(g)."""
    n, w, sigma, eps, x0 = 2048, 4, 24.0, 1e-3, 512.0
    x = np.arange(n) + 0.5
    pulse = 1.0 + eps * np.exp(-((x - x0) ** 2) / (2 * sigma ** 2))
    h = np.tile(pulse, (w, 1))
    if axis == "y":
        h = h.T.copy()
    z = np.zeros_like(h)
    dt = 0.5 / math.sqrt(G)
    announce(f"gravity wave variant={variant} axis={axis}")
    s = sw.Solver(h.shape[1], h.shape[0], g=G, dtype="f64", bc_x=sw.PERIODIC, bc_y=sw.PERIODIC, cfl=0.0,
                  dt_fixed=dt, variant=variant)
    pos = []
    for nsteps in (400, 1200):
        s.state.cur = 0
        s.set_state(torch.from_numpy(h), torch.from_numpy(z), torch.from_numpy(z))
        s.reset_time()
        s.step(nsteps)
        s.sync_status()
        H = s.get_state()[0].numpy()
        prof = H[0] if axis == "x" else H[:, 0]
        pos.append(_peak(prof, int(x0) + 50, n - 10))
    speed = (pos[1] - pos[0]) / (800 * dt)
    assert abs(speed - math.sqrt(G)) / math.sqrt(G) < 0.01, speed
