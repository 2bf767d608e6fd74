"""The region-expression front end on the CPU: the shipped program parses
with the extents the paper's face arithmetic implies, the committed kernel
is what the generator emits, the per-tile element ranges are those of a
one-cell stencil, the program's whole-array meaning (numpy interpretation)
is the oracle's step, and malformed programs are rejected with a reason."""
import numpy as np
import pytest

import oracle
from paper_1107_2157_amd import ics, regions

G = 9.8


def program_text():
    with open(regions.PROGRAM) as f:
        return f.read()


def test_extents_of_the_shipped_program():
    p = regions.load()
    assert p.inputs == ["H", "U", "V"] and p.outputs == ["oH", "oU", "oV"]
    for t in ("Hx", "Ux", "Vx"):
        assert p.arrays[t] == (1, 0)          # (nx + 1) x ny x faces
    for t in ("Hy", "Uy", "Vy"):
        assert p.arrays[t] == (0, 1)          # nx x (ny + 1) y faces
    for t in ("FU", "FV", "GV"):
        assert p.arrays[t] == (2, 2)          # flux parts on the whole array, halo included
    assert p.arrays["FUx"] == p.arrays["FVx"] == (1, 0) and p.arrays["GUy"] == p.arrays["GVy"] == (0, 1)
    assert [v for v, _ in p.stores] == ["newH", "newU", "newV"]
    assert p.views["newH"] == ("oH", (1, 1, 1, 1))
    assert set(p.elementals) == {"fu", "fv", "gv", "half", "advance"}
    assert set(p.stencils) == {"xface", "yface", "step2"}


def test_generated_kernel_is_up_to_date():
    assert regions.main(["--check"]) == 0


def test_tile_ranges_one_cell_stencil():
    boxes, out = regions.tile_ranges(regions.load(), 64, 8)
    assert out == (0, 64, 0, 8)
    for a in ("H", "U", "V"):
        assert boxes[a] == (0, 66, 0, 10)     # the tile plus one halo element on each side
    for t in ("Hx", "Ux", "Vx"):
        assert boxes[t] == (0, 65, 0, 8)      # 65 faces per row of 64 cells
    for t in ("Hy", "Uy", "Vy"):
        assert boxes[t] == (0, 64, 0, 9)


@pytest.mark.parametrize("bc", [(oracle.REFLECT, oracle.REFLECT), (oracle.PERIODIC, oracle.PERIODIC),
                                (oracle.REFLECT, oracle.PERIODIC)])
def test_interpretation_is_the_oracle_step(bc):
    """Run the program's statements as whole-array operations on halo arrays
    and compare with the oracle's step on the same state and dt."""
    nx, ny = 37, 23
    h, _, _ = ics.bumps_state(nx, ny, seed=5, periodic=False, count=2)
    _, hu, hv = ics.random_state(nx, ny, seed=6, amp_h=0.0, amp_m=0.03)
    H, U, V = (oracle.with_halo(np.asarray(a, dtype=np.float64)) for a in (h, hu, hv))
    oracle.fill_halo(H, U, V, bcx=bc[0], bcy=bc[1])
    dt = 0.4 / (np.sqrt(G * H.max()) + 0.1)
    rH, rU, rV = oracle.step(H, U, V, G, 1.0, 1.0, dt)
    outs = {k: np.zeros_like(H) for k in ("oH", "oU", "oV")}
    regions.interpret(regions.load(), {"H": H, "U": U, "V": V, **outs}, {"dt": dt, "dx": 1.0, "dy": 1.0, "g": G})
    for got, ref in zip((outs["oH"], outs["oU"], outs["oV"]), (rH, rU, rV)):
        scale = max(np.abs(ref[1:-1, 1:-1]).max(), 1e-3)
        assert np.abs(got[1:-1, 1:-1] - ref[1:-1, 1:-1]).max() <= 1e-13 * scale
    assert np.all(outs["oH"][0, :] == 0) and np.all(outs["oH"][:, 0] == 0)   # the view is the interior only


def test_interpretation_catches_a_planted_sign_error():
    """The comparison above is sensitive: flipping the sign of the flux
    difference in the half-step moves the result far from the oracle."""
    text = program_text().replace("0.5*(a + b) - c*(fb - fa)", "0.5*(a + b) + c*(fb - fa)")
    nx, ny = 16, 12
    h, hu, hv = ics.random_state(nx, ny, seed=8, amp_h=0.2, amp_m=0.05)
    H, U, V = (oracle.with_halo(np.asarray(a, dtype=np.float64)) for a in (h, hu, hv))
    oracle.fill_halo(H, U, V)
    rH, _, _ = oracle.step(H, U, V, G, 1.0, 1.0, 0.05)
    outs = {k: np.zeros_like(H) for k in ("oH", "oU", "oV")}
    regions.interpret(regions.parse(text), {"H": H, "U": U, "V": V, **outs},
                      {"dt": 0.05, "dx": 1.0, "dy": 1.0, "g": G})
    assert np.abs(outs["oH"][1:-1, 1:-1] - rH[1:-1, 1:-1]).max() > 1e-6


HEAD = """kernel k
scalar dt, dx, dy, g
in H, U, V
out oH, oU, oV
interior = [1, 1, 1, 1]
lo = [0, 1, 1, 1]
hi = [1, 0, 1, 1]
"""
TAIL = """pH = region_ptr(oH, interior)
pU = region_ptr(oU, interior)
pV = region_ptr(oV, interior)
pH = region_cpy(H, interior)
pU = region_cpy(U, interior)
pV = region_cpy(V, interior)
"""


@pytest.mark.parametrize("body,msg", [
    ("Hx = region_cpy(H, lo) + region_cpy(H, interior)\n", "extents differ"),       # an off-by-one region
    ("Hx = region_cpy(Q, lo)\n", "unknown array"),
    ("Hx = region_cpy(H, nowhere)\n", "unknown halo"),
    ("Hx = region_cpy(H, lo)\nHx = region_cpy(H, hi)\n", "assigned once"),
    ("Hx = region_cpy(oH, lo)\n", "output array"),
    ("Hx = H + 1\n", "without region_cpy"),
    ("Hx = 2*dt\n", "temporaries are arrays"),
    ("Hx = f(region_cpy(H, lo))\n", "unknown function"),
    ("bad = [1, 1, 1]\n", "left, right, down, up"),
    ("Hx = region_cpy(H, lo)**3\n", r"only \*\*2"),
])
def test_rejected_programs(body, msg):
    with pytest.raises(regions.RegionError, match=msg):
        regions.parse(HEAD + body + TAIL)


def test_rejected_store_extent_and_missing_store():
    with pytest.raises(regions.RegionError, match="extent"):
        regions.parse(HEAD + TAIL.replace("pU = region_cpy(U, interior)", "pU = region_cpy(U, lo)"))
    with pytest.raises(regions.RegionError, match="stores nothing"):
        regions.parse(HEAD)
    with pytest.raises(regions.RegionError, match="stored twice"):
        regions.parse(HEAD + TAIL + "pH = region_cpy(H, interior)\n")


def test_elemental_scalars_become_arguments():
    src = regions.generate(regions.load())
    assert "rgn_fu(T h, T u, T g)" in src and "rgn_half(T a, T b, T fa, T fb, T c)" in src
    assert "rgn_advance(T u, T fx1, T fx0, T fy1, T fy0, T dt, T dx, T dy)" in src
    assert "__syncthreads();" in src and "__shared__ T s_Hx[520];" in src and "s_FU" in src


# A program written without flux temporaries: the flux parts are evaluated
# inside the face and update expressions, once per shifted region.
UNHOISTED = """kernel k
scalar dt, dx, dy, g
in H, U, V
out oH, oU, oV
elemental fu(h, u) = u**2/h + 0.5*g*h**2
elemental fv(h, u, v) = u*v/h
elemental half(a, b, fa, fb, c) = 0.5*(a + b) - c*(fb - fa)
interior = [1, 1, 1, 1]
e = [1, 0, 1, 1]
w = [0, 1, 1, 1]
l = [0, 1, 0, 0]
r = [1, 0, 0, 0]
Ux = half(region_cpy(U, w), region_cpy(U, e), fu(region_cpy(H, w), region_cpy(U, w)), fu(region_cpy(H, e), region_cpy(U, e)), dt)
Vx = half(region_cpy(V, w), region_cpy(V, e), fv(region_cpy(H, w), region_cpy(U, w), region_cpy(V, w)), fv(region_cpy(H, e), region_cpy(U, e), region_cpy(V, e)), dt)
Hx = half(region_cpy(H, w), region_cpy(H, e), region_cpy(U, w), region_cpy(U, e), dt)
a = region_ptr(oH, interior)
b = region_ptr(oU, interior)
c = region_ptr(oV, interior)
a = region_cpy(H, interior) - dt*(region_cpy(Ux, r) - region_cpy(Ux, l))
b = region_cpy(U, interior) - dt*(fu(region_cpy(Hx, r), region_cpy(Ux, r)) - fu(region_cpy(Hx, l), region_cpy(Ux, l)))
c = region_cpy(V, interior) - dt*(fv(region_cpy(Hx, r), region_cpy(Ux, r), region_cpy(Vx, r)) - fv(region_cpy(Hx, l), region_cpy(Ux, l), region_cpy(Vx, l)))
"""


def test_hoisting_keeps_every_bit():
    """Elemental calls repeated on shifted regions are hoisted into
    temporaries (two cell fluxes on the inputs, two on the face states);
    the hoisted program computes bitwise the same outputs.  The shipped
    program evaluates its flux parts once per cell already: nothing to hoist."""
    assert regions.hoist(regions.load()).temps == regions.load().temps
    p = regions.parse(UNHOISTED)
    hp = regions.hoist(p)
    new = [n for n, _ in hp.temps if n not in p.arrays]
    assert sorted(new) == ["fu__H_U", "fu__Hx_Ux", "fv__H_U_V", "fv__Hx_Ux_Vx"]
    assert hp.arrays["fu__H_U"] == (2, 2) and hp.arrays["fu__Hx_Ux"] == (1, 0)
    nx, ny = 29, 19
    h, hu, hv = ics.random_state(nx, ny, seed=12, amp_h=0.2, amp_m=0.05)
    H, U, V = (oracle.with_halo(np.asarray(a, dtype=np.float64)) for a in (h, hu, hv))
    oracle.fill_halo(H, U, V, bcx=oracle.PERIODIC, bcy=oracle.REFLECT)
    res = []
    for prog in (p, hp):
        outs = {k: np.zeros_like(H) for k in ("oH", "oU", "oV")}
        regions.interpret(prog, {"H": H, "U": U, "V": V, **outs}, {"dt": 0.05, "dx": 1.0, "dy": 0.5, "g": G})
        res.append(outs)
    for k in ("oH", "oU", "oV"):
        assert np.array_equal(res[0][k], res[1][k])
    # a call used under one halo only is left in place
    text = HEAD + "Hx = fu2(region_cpy(H, lo), region_cpy(U, lo))\n" + TAIL
    text = text.replace("interior = [1, 1, 1, 1]", "elemental fu2(h, u) = u*u/h\ninterior = [1, 1, 1, 1]")
    q = regions.parse(text)
    assert regions.hoist(q).temps == q.temps


def test_tile_ranges_of_flux_temporaries():
    boxes, _ = regions.tile_ranges(regions.load(), 64, 8)
    assert boxes["FU"] == (0, 66, 1, 9)      # read at the x faces only: the tile's rows
    assert boxes["GV"] == (1, 65, 0, 10)     # read at the y faces only: the tile's columns
    assert boxes["FV"] == (0, 66, 0, 10)     # both
    assert boxes["FUx"] == (0, 65, 0, 8)


def test_stencil_expansion_equals_the_written_out_expression():
    """A stencil applied to arrays is its body with the arrays put in: the
    shipped program interprets bitwise as the same program with every
    stencil written out by hand."""
    text = program_text()
    expanded = regions.load()
    manual = regions.parse(UNHOISTED)
    assert manual.stencils == {}
    # write xface(U, FU) out by hand in a copy of the shipped program
    hand = "half(region_cpy(U, west), region_cpy(U, east), region_cpy(FU, west), region_cpy(FU, east), 0.5*dt/dx)"
    written = text.replace("Ux = xface(U, FU)", "Ux = " + hand)
    assert written != text
    w = regions.parse(written)
    assert dict(w.temps)["Ux"] == dict(expanded.temps)["Ux"]


@pytest.mark.parametrize("line,msg", [
    ("Hx = sx(Q)\n", "unknown array"),
    ("Hx = sx(oH)\n", "output array"),
    ("Hx = sx(H, U)\n", "takes 1 arrays"),
    ("stencil sx(A) = region_cpy(A, lo)\n", "defined twice"),
    ("stencil sy(A) = region_cpy(A, nowhere)\n", "unknown halo"),
    ("Hx = sx(H) + region_cpy(H, interior)\n", "extents differ"),
])
def test_rejected_stencils(line, msg):
    with pytest.raises(regions.RegionError, match=msg):
        regions.parse(HEAD + "stencil sx(A) = region_cpy(A, lo)\n" + line + TAIL)


def test_march_plan_of_the_shipped_program():
    """The row-march analysis of the (hoisted) step, against what the
    one-cell stencil implies: the inputs are read one row below and above
    the stored row (a ring of three rows, two warm-up rows), the x-face
    arrays only on the stored row; an x face i needs the cell i + 1, so it is
    valid on lanes 0..62, and a stored cell needs the faces on both sides
    (lanes 1..62: 62 of 64 columns per strip)."""
    m = regions.march_plan(regions.hoist(regions.load()))
    for a in ("H", "U", "V"):
        assert (m.lo[a], m.hi[a], m.valid[a]) == (-1, 1, (0, 63))
    for a in ("Hx", "Ux", "Vx", "FUx", "FVx"):
        assert (m.lo[a], m.hi[a], m.valid[a]) == (0, 0, (0, 62))
    for a in ("Hy", "Uy", "Vy", "GUy", "GVy"):
        assert (m.lo[a], m.hi[a]) == (-1, 0)       # the y faces below and above a stored row
    assert m.out_lanes == (1, 62) and m.warmup == 2
    assert m.order[:3] == ["H", "U", "V"]          # inputs first, then temporaries in program order
    src = regions.generate(regions.load())
    assert "k_rgn_wave_advance_march" in src


def test_march_rejects_reads_two_columns_away():
    """A well-formed program that stores H shifted one column left plus a
    temporary reading H one column right (every region nx wide) is valid
    region arithmetic, but it reads H two columns apart, and the row march
    shifts across lanes by one column at most: the planner says so."""
    text = (HEAD + "wa = [0, 2, 1, 1]\nwb = [2, 0, 1, 1]\nnone = [0, 0, 0, 0]\n"
            + "Hx = region_cpy(H, wb)\n"
            + TAIL.replace("pH = region_cpy(H, interior)\n", "pH = region_cpy(H, wa) + region_cpy(Hx, none)\n"))
    prog = regions.parse(text)
    assert prog.arrays["Hx"] == (0, 0)
    with pytest.raises(regions.RegionError, match="only -1, 0, 1"):
        regions.march_plan(prog)
