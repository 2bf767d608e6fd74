"""Batched mode on the GPU (through the C ABI): every grid of a batch equals
the same grid advanced alone, bitwise; small grids match the oracle; graph
replays equal eager launches; per-grid dt, time and sticky flags."""
import numpy as np
import pytest
import torch

import oracle
from paper_1107_2157_amd import ics, sw
from swtest import G, announce, rel_maxnorm

pytestmark = pytest.mark.gpu

SHAPES = [(64, 64), (130, 65), (200, 64), (1, 1), (300, 17), (17, 300), (257, 129), (64, 1024)]


def states(shapes, seed0, periodic):
    out = []
    for k, (nx, ny) in enumerate(shapes):
        h, _, _ = ics.bumps_state(nx, ny, seed=seed0 + k, periodic=periodic)
        _, hu, hv = ics.random_state(nx, ny, seed=seed0 + k, amp_h=0.0, amp_m=0.02)
        out.append((h, hu, hv))
    return out


def make_batch(shapes, sts, dtype, bc, tuning, graph=True, **kw):
    b = sw.Batch(shapes, dtype=dtype, bc_x=bc, bc_y=bc, **kw)
    b.set_tuning(**tuning)
    b.set_graph(graph)
    for i, st in enumerate(sts):
        b.set_state(i, *st)
    return b


@pytest.mark.parametrize("dtype", ["f32", "f64"])
@pytest.mark.parametrize("bc", [sw.REFLECT, sw.PERIODIC])
@pytest.mark.parametrize("graph", [True, False])
@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_batch_equals_each_grid_alone(dtype, bc, graph, scheme):
    tun = dict(variant=2, rows=16, vec=2, occupancy=0, prefetch=2, order=0)
    sts = states(SHAPES, 100, bc == sw.PERIODIC)
    announce(f"batch {dtype} bc{bc} graph{graph} scheme{scheme}")
    b = make_batch(SHAPES, sts, dtype, bc, tun, graph, scheme=scheme)
    b.step(7)
    b.step(4)
    t_b, n_b, _ = b.sync_status()
    for i, (nx, ny) in enumerate(SHAPES):
        s = sw.Solver(nx, ny, dtype=dtype, bc_x=bc, bc_y=bc, scheme=scheme)
        s.set_tuning(**tun)
        s.set_state(*sts[i])
        s.step(7)
        s.step(4)
        t_s, _, n_s = s.sync_status()
        got = b.get_state(i, halo=True)
        ref = s.get_state(halo=True)
        for x, y in zip(got, ref):
            assert np.array_equal(x.numpy(), y.numpy()), (i, nx, ny)
        assert n_b[i] == n_s == 11 and t_b[i] == t_s


# Batches of 4 M cells or more per step advance as two chains of grids on
# two streams; every grid must still equal the same grid advanced alone.
SPLIT_SHAPES = {
    "widths_multiple_of_4": [(2048, 2048), (1024, 2048), (2048, 1024), (1500, 1300), (64, 64), (256, 8)],
    "ragged": [(2048, 2048), (1023, 2049), (2049, 1024), (1500, 1300), (1, 1), (300, 17), (17, 300)],
}


@pytest.mark.parametrize("shapes", sorted(SPLIT_SHAPES))
@pytest.mark.parametrize("bc", [sw.REFLECT, sw.PERIODIC])
@pytest.mark.parametrize("graph", [True, False])
def test_split_batch_equals_each_grid_alone(shapes, bc, graph):
    shp = SPLIT_SHAPES[shapes]
    assert sum(nx * ny for nx, ny in shp) >= 1 << 22
    tun = dict(variant=2, rows=8, vec=4, occupancy=0, prefetch=1, order=0)
    sts = states(shp, 700, bc == sw.PERIODIC)
    announce(f"split batch {shapes} bc{bc} graph{graph}")
    b = make_batch(shp, sts, "f32", bc, tun, graph)
    b.step(7)
    b.step(4)
    t_b, n_b, _ = b.sync_status()
    for i, (nx, ny) in enumerate(shp):
        s = sw.Solver(nx, ny, dtype="f32", bc_x=bc, bc_y=bc)
        s.set_tuning(**tun)
        s.set_state(*sts[i])
        s.step(7)
        s.step(4)
        t_s, _, n_s = s.sync_status()
        for x, y in zip(b.get_state(i, halo=True), s.get_state(halo=True)):
            assert np.array_equal(x.numpy(), y.numpy()), (i, nx, ny)
        assert n_b[i] == n_s == 11 and t_b[i] == t_s


@pytest.mark.parametrize("dtype,tol", [("f64", 1e-12), ("f32", 1e-5)])
@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_batch_matches_oracle(dtype, tol, scheme):
    shapes = [(96, 80), (33, 150), (128, 128), (1, 9)]
    sts = states(shapes, 300, False)
    b = make_batch(shapes, sts, dtype, sw.REFLECT, dict(variant=2), scheme=scheme)
    b.step(60)
    b.sync_status()
    for i, st in enumerate(sts):
        st = [a.to(torch.float32).to(torch.float64) if dtype == "f32" else a for a in st]
        H, U, V, _ = oracle.run(*(a.numpy() for a in st), 60, g=G, scheme=scheme)
        err = rel_maxnorm(b.get_state(i), (H[1:-1, 1:-1], U[1:-1, 1:-1], V[1:-1, 1:-1]))
        assert err <= tol, (i, err)


def test_graph_replays_equal_eager():
    """The cached graph is replayed several times with eager work and
    synchronisations between the replays; every replay equals an eager
    batch run step for step."""
    shapes = [(128, 64), (64, 200), (320, 96)]
    sts = states(shapes, 500, True)
    tun = dict(variant=2, rows=8, vec=2, order=1)
    bg = make_batch(shapes, sts, "f32", sw.PERIODIC, tun, graph=True)
    be = make_batch(shapes, sts, "f32", sw.PERIODIC, tun, graph=False)
    for rep in range(4):
        bg.step(5)
        be.step(5)
        torch.cuda.synchronize()
        _ = (torch.ones(1000, device="cuda") * 2).sum().item()      # unrelated eager work
        for i in range(len(shapes)):
            for x, y in zip(bg.get_state(i), be.get_state(i)):
                assert np.array_equal(x.numpy(), y.numpy()), (rep, i)
        assert bg.sync_status() == be.sync_status()


TUNINGS = {sw.SCHEME_PAPER: (dict(rows=8, vec=1, order=0), dict(rows=16, vec=2, order=1, occupancy=4, prefetch=2),
                             dict(rows=32, vec=4, order=0, prefetch=3), dict(rows=5, vec=2, order=1, prefetch=1),
                             dict(rows=8, vec=2, order=2, prefetch=2), dict(rows=3, vec=1, order=2, occupancy=4,
                                                                            prefetch=2)),
           sw.SCHEME_TRANSVERSE: (dict(rows=8, vec=1, order=0, prefetch=1), dict(rows=16, vec=2, order=1, prefetch=2),
                                  dict(rows=32, vec=4, order=0, prefetch=2), dict(rows=5, vec=2, order=1, prefetch=1),
                                  dict(rows=2, vec=1, order=0, prefetch=2), dict(rows=4, vec=1, order=2, prefetch=1))}


@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_tunings_bitwise_identical(scheme):
    shapes = [(200, 130), (64, 64), (513, 70)]
    sts = states(shapes, 700, False)
    ref = None
    for tun in TUNINGS[scheme]:
        b = make_batch(shapes, sts, "f32", sw.REFLECT, dict(variant=2, **tun), scheme=scheme)
        b.step(13)
        out = [[a.numpy() for a in b.get_state(i, halo=True)] for i in range(len(shapes))] + [b.sync_status()]
        if ref is None:
            ref = out
        else:
            for gi in range(len(shapes)):
                for x, y in zip(ref[gi], out[gi]):
                    assert np.array_equal(x, y), (tun, gi)
            assert ref[-1] == out[-1]


def test_batch_tile_span_limit():
    """The batch's fused tiles reach their rows through 32-bit buffer
    offsets as the single-grid kernel's do: with a grid 2^21 cells wide in
    FP64 in the batch, 40 rows per tile fit and 41 are refused when the shape
    is chosen (the other grid is small)."""
    b = sw.Batch([(2 ** 21, 1), (64, 64)], dtype="f64")
    b.set_tuning(variant=2, rows=40, vec=1)
    with pytest.raises(sw.SwError) as e:
        b.set_tuning(variant=2, rows=41, vec=1)
    assert e.value.status == sw.EINVAL


def test_per_grid_sticky_flag_and_dt():
    shapes = [(64, 64), (64, 64), (128, 64)]
    sts = states(shapes, 900, False)
    h, hu, hv = sts[1]
    h = h.clone()
    h[10, 10] = -1.0
    sts[1] = (h, hu, hv)
    b = make_batch(shapes, sts, "f32", sw.REFLECT, dict(variant=2))
    b.step(3)
    t, n, u = b.sync_status(raise_unstable=False)
    assert u == [0, 1, 0] and n == [3, 3, 3]
    with pytest.raises(sw.Unstable):
        b.sync_status()
    assert t[0] != t[2]            # independent CFL dt per grid


@pytest.mark.parametrize("scheme", [sw.SCHEME_PAPER, sw.SCHEME_TRANSVERSE])
def test_persistent_walk_equals_wave_per_tile(scheme):
    """The persistent schedule (order 2: resident waves, each walking a
    contiguous run of the LPT table, the next entry loaded ahead, dt kept and
    the signal-speed max flushed per grid) against one wave per tile, on a
    batch with enough tiles (about 17 000 at 2-row, 64-column tiles) that
    every wave walks several tiles and many runs cross from one grid into the
    next: bitwise equal states with halos, times and step counts, CFL dt."""
    rng = np.random.default_rng(11)
    shapes = [(int(64 * rng.integers(1, 7)), int(32 * rng.integers(1, 13))) for _ in range(40)]
    sts = states(shapes, 900, False)
    announce(f"persistent batch walk, scheme {scheme}, {len(shapes)} grids")
    outs = []
    for order in (0, 2):
        b = make_batch(shapes, sts, "f32", sw.REFLECT, dict(variant=2, rows=2, vec=1, order=order, prefetch=1),
                       scheme=scheme)
        b.step(9)
        outs.append(([[a.numpy() for a in b.get_state(i, halo=True)] for i in range(len(shapes))], b.sync_status()))
    (ra, sa), (rb, sb) = outs
    for gi in range(len(shapes)):
        for x, y in zip(ra[gi], rb[gi]):
            assert np.array_equal(x, y), gi
    assert sa == sb
