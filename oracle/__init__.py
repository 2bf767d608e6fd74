"""CPU FP64 oracle for the shallow-water two-step Lax-Wendroff step.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the CPU-baseline leg of ``bench.py``; never by the product package.  The C
loops in ``sw_oracle.c`` follow the paper's "Shallow Water Model" section
(conservation laws, CFL bound, the two Lax-Wendroff steps and the Fortran
face/update statements); this module only marshals numpy arrays.

Arrays passed here are ``(ny + 2, nx + 2)`` float64 with a one-cell halo.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sw_oracle.c")
LIB = os.path.join(HERE, "libswor.so")

REFLECT, PERIODIC = 0, 1
SCHEME_PAPER, SCHEME_TRANSVERSE = 0, 1
OK, EINVAL, ENOMEM, EUNSTABLE = 0, -1, -3, -5


def compile_to(src: str, out: str) -> str:
    """Compile an oracle source with strict IEEE semantics (no contraction)."""
    tmp = out + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c99",
                           "-shared", "-fPIC", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_to(SRC, LIB)
    return LIB


class Oracle:
    """The oracle bound to one compiled library (the default one, or a
    deliberately broken copy built by the mutation tests)."""

    def __init__(self, libpath: str):
        lib = ctypes.CDLL(libpath)
        P = ctypes.POINTER(ctypes.c_double)
        i, d = ctypes.c_int, ctypes.c_double
        lib.or_fill_halo.argtypes = [i, i, i, i, P, P, P]
        lib.or_fill_halo.restype = None
        lib.or_max_speed.argtypes = [i, i, d, P, P, P]
        lib.or_max_speed.restype = d
        lib.or_step.argtypes = [i, i, d, d, d, d, i, P, P, P, P, P, P]
        lib.or_step.restype = i
        lib.or_run.argtypes = [i, i, d, d, d, d, d, i, i, i, i, P, P, P, P, P,
                               ctypes.POINTER(ctypes.c_int)]
        lib.or_run.restype = i
        self.lib = lib

    def fill_halo(self, H, U, V, bcx=REFLECT, bcy=REFLECT):
        ny, nx = H.shape[0] - 2, H.shape[1] - 2
        self.lib.or_fill_halo(nx, ny, bcx, bcy, _ptr(H), _ptr(U), _ptr(V))

    def max_speed(self, H, U, V, g):
        ny, nx = H.shape[0] - 2, H.shape[1] - 2
        return self.lib.or_max_speed(nx, ny, g, _ptr(H), _ptr(U), _ptr(V))

    def step(self, H, U, V, g, dx, dy, dt, scheme=SCHEME_PAPER):
        """One step with a given dt; the input halo must be filled.  Returns
        new arrays whose interior holds U^{n+1} (halo left zero)."""
        ny, nx = H.shape[0] - 2, H.shape[1] - 2
        oH, oU, oV = (np.zeros_like(H) for _ in range(3))
        rc = self.lib.or_step(nx, ny, g, dx, dy, dt, scheme, _ptr(H), _ptr(U), _ptr(V),
                              _ptr(oH), _ptr(oU), _ptr(oV))
        if rc != OK:
            raise RuntimeError(f"or_step failed: {rc}")
        return oH, oU, oV

    def run(self, h, hu, hv, nsteps, g=9.8, dx=1.0, dy=1.0, cfl=0.5, dt_fixed=0.0,
            scheme=SCHEME_PAPER, bcx=REFLECT, bcy=REFLECT, return_dts=False, raise_unstable=True):
        """Advance an interior state ``(ny, nx)`` by ``nsteps``.

        Returns ``(H, U, V, t)`` as halo arrays ``(ny + 2, nx + 2)`` with the
        final halo filled (plus the per-step dts when asked).
        """
        H, U, V = with_halo(h), with_halo(hu), with_halo(hv)
        ny, nx = H.shape[0] - 2, H.shape[1] - 2
        dts = np.zeros(max(nsteps, 1), dtype=np.float64)
        t = ctypes.c_double(0.0)
        done = ctypes.c_int(0)
        rc = self.lib.or_run(nx, ny, g, dx, dy, cfl, dt_fixed, scheme, bcx, bcy, nsteps,
                             _ptr(H), _ptr(U), _ptr(V), ctypes.byref(t), _ptr(dts), ctypes.byref(done))
        if rc == EUNSTABLE and raise_unstable:
            raise Unstable(f"unstable after {done.value} steps")
        if rc not in (OK, EUNSTABLE):
            raise RuntimeError(f"or_run failed: {rc}")
        out = (H, U, V, t.value)
        if return_dts:
            out = out + (dts[:nsteps],)
        return out


class Unstable(RuntimeError):
    """A step produced h <= 0 or a non-finite value."""


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def with_halo(interior) -> np.ndarray:
    """Embed an ``(ny, nx)`` interior into a zero ``(ny + 2, nx + 2)`` array."""
    a = np.asarray(interior, dtype=np.float64)
    out = np.zeros((a.shape[0] + 2, a.shape[1] + 2), dtype=np.float64)
    out[1:-1, 1:-1] = a
    return out


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def fill_halo(*a, **k):
    return default().fill_halo(*a, **k)


def max_speed(*a, **k):
    return default().max_speed(*a, **k)


def step(*a, **k):
    return default().step(*a, **k)


def run(*a, **k):
    return default().run(*a, **k)
