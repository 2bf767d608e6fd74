"""Strength of the oracle's pins: plant plausible mistakes in a copy of the
oracle source (on the CPU), and check that a quick battery of the same pins
(closed-form linear modes, lake at rest, conservation, symmetry, reflective
wall as a symmetry plane, CFL closed form) rejects every one of them, while
accepting the unmodified oracle."""
import math
import os

import numpy as np
import pytest

import oracle
from oracle import PERIODIC, REFLECT, SCHEME_PAPER, SCHEME_TRANSVERSE
from paper_1107_2157_amd import ics

from test_oracle_pins import amplification, interior, jacobians

G = 9.8

# (name, text to find, replacement) applied to sw_oracle.c
MUTATIONS = [
    ("x half-step sign", "double h = 0.5 * (hl + hr) + hx * (ul - ur);",
     "double h = 0.5 * (hl + hr) - hx * (ul - ur);"),
    ("y half-step uses F", "double u = 0.5 * (ud + uu) + hy * (flux_gu(g, hd, ud, vd) - flux_gu(g, hu, uu, vu));",
     "double u = 0.5 * (ud + uu) + hy * (flux_fu(g, hd, ud, vd) - flux_fu(g, hu, uu, vu));"),
    ("pressure term dropped", "return u * u / h + 0.5 * g * h * h;", "return u * u / h;"),
    ("update faces swapped", "int lt = i - 1, rt = i;", "int lt = i, rt = i - 1;"),
    ("wall momentum not negated", "AT(U, 0, j) = -AT(U, 1, j);", "AT(U, 0, j) = AT(U, 1, j);"),
    ("dx and dy swapped", "const double hx = 0.5 * dt / dx, hy = 0.5 * dt / dy;",
     "const double hx = 0.5 * dt / dy, hy = 0.5 * dt / dx;"),
    ("cfl takes min speed", "double si = (u > v ? u : v) + c;", "double si = (u < v ? u : v) + c;"),
    ("transverse sign", "h += hy * 0.25 * ((vd0 + vd1) - (vu0 + vu1));",
     "h -= hy * 0.25 * ((vd0 + vd1) - (vu0 + vu1));"),
    ("x flux of hv wrong", "static double flux_fv(double g, double h, double u, double v) { (void)g; return u * v / h; }",
     "static double flux_fv(double g, double h, double u, double v) { (void)g; return v * v / h; }"),
    ("periodic wrap off by one", "AT(H, 0, j) = AT(H, nx, j);", "AT(H, 0, j) = AT(H, nx - 1, j);"),
    ("update mixes momenta", "AT(oU, i, j) = AT(U, i, j) + mx", "AT(oU, i, j) = AT(V, i, j) + mx"),
    ("half-step average wrong", "double u = 0.5 * (ul + ur) + hx", "double u = 0.5 * (ul + ul) + hx"),
    ("y wall corner sign", "AT(V, i, 0) = -AT(V, i, 1);", "AT(V, i, 0) = AT(V, i, 1);"),
    ("y update dt/dy as dt/dx", "const double mx = dt / dx, my = dt / dy;",
     "const double mx = dt / dx, my = dt / dx;"),
]


def battery(orc: oracle.Oracle) -> list[str]:
    """Returns the names of the pins that fail."""
    bad = []

    def check(name, fn):
        try:
            ok = fn()
        except Exception:
            ok = False
        if not ok:
            bad.append(name)

    def linear(scheme, u0, v0, kx, ky):
        nx, ny, nsteps, h0, dx, dy = 16, 12, 5, 1.0, 1.0, 0.8
        dt = 0.5 * min(dx, dy) / (max(abs(u0), abs(v0)) + math.sqrt(G * h0))
        eps = 1e-7
        uhat = np.array([0.7 + 0.2j, -0.4 + 0.9j, 0.3 - 0.6j])
        alpha, beta = 2 * math.pi * kx / nx, 2 * math.pi * ky / ny
        jj, ii = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
        phase = np.exp(1j * (alpha * ii + beta * jj))
        base = np.array([h0, h0 * u0, h0 * v0])
        st = [base[c] + eps * np.real(uhat[c] * phase) for c in range(3)]
        out = orc.run(*st, nsteps, g=G, dx=dx, dy=dy, dt_fixed=dt, scheme=scheme, bcx=PERIODIC, bcy=PERIODIC)
        a, b = jacobians(h0, u0, v0)
        want = np.linalg.matrix_power(amplification(alpha, beta, dt / dx, dt / dy, a, b,
                                                    scheme == SCHEME_TRANSVERSE), nsteps) @ uhat
        return all(np.max(np.abs((interior(out[c]) - base[c]) / eps - np.real(want[c] * phase))) < 1e-5
                   for c in range(3))

    for scheme in (SCHEME_PAPER, SCHEME_TRANSVERSE):
        check(f"linear modes s{scheme}", lambda: linear(scheme, 0.4, -0.25, 3, 2) and linear(scheme, 0.0, 0.0, 1, 5))

    def cfl():
        h, u, v = 1.7, -0.9, 0.4
        st = [np.full((5, 7), x) for x in (h, h * u, h * v)]
        _, _, _, _, dts = orc.run(*st, 1, cfl=0.5, bcx=PERIODIC, bcy=PERIODIC, return_dts=True)
        return abs(dts[0] - 0.5 / (0.9 + math.sqrt(G * h))) < 1e-14

    check("cfl", cfl)

    def wall(scheme):
        ny, nx = 10, 14
        h, hu, hv = (a.numpy() for a in ics.random_state(nx, ny, seed=3))
        bh = np.block([[h, h[:, ::-1]], [h[::-1, :], h[::-1, ::-1]]])
        bu = np.block([[hu, -hu[:, ::-1]], [hu[::-1, :], -hu[::-1, ::-1]]])
        bv = np.block([[hv, hv[:, ::-1]], [-hv[::-1, :], -hv[::-1, ::-1]]])
        A = orc.run(h, hu, hv, 10, scheme=scheme, dt_fixed=0.05)
        B = orc.run(bh, bu, bv, 10, scheme=scheme, bcx=PERIODIC, bcy=PERIODIC, dt_fixed=0.05)
        return all(np.array_equal(interior(x), interior(y)[:ny, :nx]) for x, y in zip(A[:3], B[:3]))

    check("wall symmetry plane", lambda: wall(SCHEME_PAPER) and wall(SCHEME_TRANSVERSE))

    def mass():
        h, hu, hv = (a.numpy() for a in ics.random_state(20, 15, seed=1))
        m0 = math.fsum(h.ravel())
        H = orc.run(h, hu, hv, 20)[0]
        return abs(math.fsum(interior(H).ravel()) - m0) / m0 < 1e-12

    check("mass", mass)
    return bad


def test_unmodified_oracle_passes_battery():
    assert battery(oracle.default()) == []


@pytest.mark.parametrize("name,find,repl", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_mutant_is_rejected(tmp_path, name, find, repl):
    src = open(oracle.SRC).read()
    assert src.count(find) == 1, f"mutation anchor not unique: {find}"
    mpath = os.path.join(tmp_path, "mutant.c")
    with open(mpath, "w") as f:
        f.write(src.replace(find, repl))
    lib = oracle.compile_to(mpath, os.path.join(tmp_path, "libmutant.so"))
    assert battery(oracle.Oracle(lib)) != [], f"mutation '{name}' passed every pin"
