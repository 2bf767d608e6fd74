"""Thin ctypes binding of libsw (``include/sw.h``).

Argument marshalling only: every step of the solver runs in the library's HIP
kernels.  PyTorch provides the device memory (plane tensors) and the stream.
If ``libsw.so`` is not built, loading fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

PKG = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(PKG, "libsw.so")

OK, EINVAL, ENOTSUP, ENOMEM, EHIP, EUNSTABLE = 0, -1, -2, -3, -4, -5
F32, F64 = 0, 1
REFLECT, PERIODIC = 0, 1
SCHEME_PAPER, SCHEME_TRANSVERSE = 0, 1
VARIANT_AUTO, VARIANT_CELL, VARIANT_FUSED, VARIANT_TBLOCK, VARIANT_UNFUSED, VARIANT_AOS, VARIANT_GENERATED = range(7)

_DT = {"f32": F32, "f64": F64, torch.float32: F32, torch.float64: F64}
_TORCH_DT = {F32: torch.float32, F64: torch.float64}


class SwError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status} ({detail})")
        self.status = status


class Unstable(SwError):
    """The sticky flag is set: some step produced h <= 0 or a non-finite value."""


class Grid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32)]


class Halo(ctypes.Structure):
    _fields_ = [("left", ctypes.c_int32), ("right", ctypes.c_int32),
                ("down", ctypes.c_int32), ("up", ctypes.c_int32)]


class Opts(ctypes.Structure):
    _fields_ = [("dtype", ctypes.c_int), ("bc_x", ctypes.c_int), ("bc_y", ctypes.c_int),
                ("scheme", ctypes.c_int), ("dy", ctypes.c_double), ("cfl", ctypes.c_double),
                ("dt_fixed", ctypes.c_double)]


class Layout(ctypes.Structure):
    _fields_ = [("pitch", ctypes.c_int64), ("origin", ctypes.c_int64),
                ("plane_elems", ctypes.c_int64), ("plane_offset", ctypes.c_int64),
                ("buffer_elems", ctypes.c_int64), ("elem_bytes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("variant", ctypes.c_int32), ("rows", ctypes.c_int32), ("vec", ctypes.c_int32),
                ("occupancy", ctypes.c_int32), ("prefetch", ctypes.c_int32), ("order", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class NetCfg(ctypes.Structure):
    _fields_ = [("layers", ctypes.c_int32), ("hidden", ctypes.c_int32), ("jump", ctypes.c_int32),
                ("bc_x", ctypes.c_int32), ("bc_y", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class Gate(ctypes.Structure):
    _fields_ = [("mass_rel_tol", ctypes.c_double), ("hmin", ctypes.c_double), ("project_mass", ctypes.c_int32),
                ("judge", ctypes.c_int32), ("l2_tol", ctypes.c_double)]


class State(ctypes.Structure):
    _fields_ = [("plane", (ctypes.c_void_p * 3) * 2), ("cur", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


_lib = None

# name -> (restype, argtypes); every symbol of include/sw.h
SIGNATURES = {
    "sw_layout_query": (ctypes.c_int, [Grid, ctypes.c_int, ctypes.POINTER(Layout)]),
    "sw_create": (ctypes.c_int, [Grid, Halo, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Opts),
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "sw_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sw_get_layout": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Layout)]),
    "sw_fill_halo": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(State), ctypes.c_void_p]),
    "sw_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(State), ctypes.c_int32, ctypes.c_void_p]),
    "sw_sync_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                      ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    "sw_reset_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sw_diagnostics": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(State), ctypes.c_void_p,
                                      ctypes.POINTER(ctypes.c_double)]),
    "sw_set_variant": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sw_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sw_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(State), ctypes.c_int32, ctypes.c_char_p,
                                   ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sw_batch_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(Grid), Halo, ctypes.c_double, ctypes.c_double,
                                       ctypes.POINTER(Opts), ctypes.POINTER(ctypes.c_void_p)]),
    "sw_batch_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sw_batch_arena_bytes": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)]),
    "sw_batch_bind": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sw_batch_view": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(State), ctypes.POINTER(Layout)]),
    "sw_batch_fill_halo": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sw_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p]),
    "sw_batch_sync_status": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32)]),
    "sw_batch_reset_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sw_batch_export": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_batch_import": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_batch_set_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sw_batch_get_tuning": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Tuning)]),
    "sw_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_batch_autotune": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p, ctypes.c_void_p,
                                         ctypes.POINTER(Tuning)]),
    "sw_surrogate_create": (ctypes.c_int, [ctypes.POINTER(NetCfg), ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                           ctypes.POINTER(ctypes.c_void_p)]),
    "sw_surrogate_destroy": (ctypes.c_int, [ctypes.c_void_p]),
    "sw_surrogate_params": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p),
                                           ctypes.POINTER(ctypes.c_int64)]),
    "sw_surrogate_sync_weights": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p]),
    "sw_surrogate_set_norm": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_float),
                                             ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "sw_surrogate_forward": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                            ctypes.c_void_p]),
    "sw_surrogate_activation": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p),
                                               ctypes.POINTER(ctypes.c_int64)]),
    "sw_surrogate_grad": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                         ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_surrogate_train_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                               ctypes.c_float, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_surrogate_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_surrogate_set_block_cap": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_surrogate_set_fused": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int32]),
    "sw_surrogate_advance": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(Gate),
                                            ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_step_noalloc": (ctypes.c_int, [Grid, Halo, ctypes.c_double, ctypes.c_double, ctypes.POINTER(Opts),
                                       ctypes.POINTER(State), ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]),
    "sw_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "sw_last_error_detail": (ctypes.c_char_p, []),
}


def lib():
    """Load libsw.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise RuntimeError(f"{LIBPATH} is not built; run `python -m paper_1107_2157_amd.build`")
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int, where: str):
    if status != OK:
        detail = lib().sw_last_error_detail().decode(errors="replace")
        cls = Unstable if status == EUNSTABLE else SwError
        raise cls(status, where, detail)


def layout_query(nx: int, ny: int, dtype="f32") -> Layout:
    out = Layout()
    check(lib().sw_layout_query(Grid(nx, ny), _DT[dtype], ctypes.byref(out)), "sw_layout_query")
    return out


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Solver:
    """One grid: a context plus its ping-pong state planes in device memory."""

    def __init__(self, nx: int, ny: int, g: float = 9.8, dx: float = 1.0, dtype="f32",
                 bc_x: int = REFLECT, bc_y: int = REFLECT, scheme: int = SCHEME_PAPER,
                 dy: float = 0.0, cfl: float = 0.5, dt_fixed: float = 0.0, device="cuda",
                 variant: int = VARIANT_AUTO):
        self.nx, self.ny = nx, ny
        self.dtype = _DT[dtype]
        self.torch_dtype = _TORCH_DT[self.dtype]
        opts = Opts(self.dtype, bc_x, bc_y, scheme, dy, cfl, dt_fixed)
        self.opts, self.g, self.dx = opts, g, dx
        ctx = ctypes.c_void_p()
        check(lib().sw_create(Grid(nx, ny), Halo(1, 1, 1, 1), g, dx, ctypes.byref(opts), ctypes.byref(ctx)),
              "sw_create")
        self.ctx = ctx
        self.layout = Layout()
        check(lib().sw_get_layout(ctx, ctypes.byref(self.layout)), "sw_get_layout")
        # one allocation per buffer; the rows of its three planes interleave
        L = self.layout
        self.buffers = [torch.zeros(L.buffer_elems, dtype=self.torch_dtype, device=device) for _ in range(2)]
        self.state = State()
        for b in range(2):
            for k in range(3):
                self.state.plane[b][k] = self.buffers[b].data_ptr() + k * L.plane_offset * L.elem_bytes
        self.state.cur = 0
        if variant != VARIANT_AUTO:
            self.set_variant(variant)

    def __del__(self):
        try:
            if getattr(self, "ctx", None) and _lib is not None:
                _lib.sw_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # ---- views -----------------------------------------------------------
    def halo_view(self, k: int, buf: int | None = None) -> torch.Tensor:
        """(ny + 2, nx + 2) strided view of plane k (0 h, 1 hu, 2 hv) with its halo."""
        b = self.state.cur if buf is None else buf
        L = self.layout
        return torch.as_strided(self.buffers[b], (self.ny + 2, self.nx + 2), (L.pitch, 1),
                                k * L.plane_offset + L.origin - L.pitch - 1)

    def interior(self, k: int, buf: int | None = None) -> torch.Tensor:
        return self.halo_view(k, buf)[1:-1, 1:-1]

    def set_state(self, h, hu, hv):
        """Write an interior state (any float dtype/device) into buf[cur]."""
        for k, a in enumerate((h, hu, hv)):
            self.interior(k).copy_(torch.as_tensor(a).to(self.torch_dtype))

    def get_state(self, halo: bool = False):
        """Copy of (h, hu, hv) of buf[cur] on the host as float64 tensors."""
        torch.cuda.synchronize()
        f = self.halo_view if halo else self.interior
        return tuple(f(k).to("cpu", torch.float64) for k in range(3))

    # ---- calls -----------------------------------------------------------
    def set_variant(self, variant: int):
        check(lib().sw_set_variant(self.ctx, variant), "sw_set_variant")

    def set_tuning(self, variant=0, rows=0, vec=0, occupancy=0, prefetch=0, order=0):
        check(lib().sw_set_tuning(self.ctx, ctypes.byref(Tuning(variant, rows, vec, occupancy, prefetch, order))),
              "sw_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        check(lib().sw_get_tuning(self.ctx, ctypes.byref(t)), "sw_get_tuning")
        return t.as_dict()

    def autotune(self, steps_per_trial: int = 5, cache_path: str | None = None, stream=None) -> dict:
        t = Tuning()
        path = cache_path.encode() if cache_path else None
        check(lib().sw_autotune(self.ctx, ctypes.byref(self.state), steps_per_trial, path,
                                _stream_handle(stream), ctypes.byref(t)), "sw_autotune")
        return t.as_dict()

    def fill_halo(self, stream=None):
        check(lib().sw_fill_halo(self.ctx, ctypes.byref(self.state), _stream_handle(stream)), "sw_fill_halo")

    def step(self, nsteps: int, stream=None):
        check(lib().sw_step(self.ctx, ctypes.byref(self.state), nsteps, _stream_handle(stream)), "sw_step")

    def step_noalloc(self, nsteps: int, status: torch.Tensor | None = None, stream=None):
        """sw_step_noalloc on this solver's planes: default launch shape, eager
        launches, the library's static per-device scalars instead of the
        context's.  status: optional float64 device tensor of 4 entries that
        receives (t, last dt, steps, unstable) of this call."""
        if status is not None and (not status.is_cuda or status.dtype != torch.float64 or status.numel() < 4
                                   or not status.is_contiguous()):
            raise ValueError("status: expected a contiguous float64 device tensor of at least 4 entries")
        ptr = ctypes.c_void_p(status.data_ptr()) if status is not None else None
        check(lib().sw_step_noalloc(Grid(self.nx, self.ny), Halo(1, 1, 1, 1), self.g, self.dx,
                                    ctypes.byref(self.opts), ctypes.byref(self.state), nsteps, ptr,
                                    _stream_handle(stream)), "sw_step_noalloc")

    def sync_status(self, stream=None):
        """(t, last_dt, steps); raises Unstable if the sticky flag is set."""
        t, dt, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
        check(lib().sw_sync_status(self.ctx, _stream_handle(stream), ctypes.byref(t), ctypes.byref(dt),
                                   ctypes.byref(n)), "sw_sync_status")
        return t.value, dt.value, n.value

    def set_graph(self, enable: bool):
        """Replay sw_step calls as hipGraphs (default) or launch eagerly."""
        check(lib().sw_set_graph(self.ctx, 1 if enable else 0), "sw_set_graph")

    def reset_time(self, stream=None):
        check(lib().sw_reset_time(self.ctx, _stream_handle(stream)), "sw_reset_time")

    def diagnostics(self, stream=None) -> dict:
        """Sums of h, hu, hv, max signal speed, min h and non-finite cell count of buf[cur]."""
        out = (ctypes.c_double * 6)()
        check(lib().sw_diagnostics(self.ctx, ctypes.byref(self.state), _stream_handle(stream), out),
              "sw_diagnostics")
        return {"mass": out[0], "sum_hu": out[1], "sum_hv": out[2], "max_speed": out[3], "min_h": out[4],
                "nonfinite": int(out[5])}


class Batch:
    """Many independent grids advanced together (sw_batch_*): one device
    arena (a torch uint8 tensor), one launch per step for all grids, the
    whole call replayed as one hipGraph."""

    def __init__(self, sides, g: float = 9.8, dx: float = 1.0, dtype="f32", bc_x: int = REFLECT,
                 bc_y: int = REFLECT, dy: float = 0.0, cfl: float = 0.5, dt_fixed: float = 0.0, device="cuda",
                 scheme: int = SCHEME_PAPER):
        shapes = [(s, s) if isinstance(s, int) else tuple(s) for s in sides]
        self.n = len(shapes)
        self.shapes = shapes
        self.dtype = _DT[dtype]
        self.torch_dtype = _TORCH_DT[self.dtype]
        grids = (Grid * self.n)(*[Grid(nx, ny) for nx, ny in shapes])
        opts = Opts(self.dtype, bc_x, bc_y, scheme, dy, cfl, dt_fixed)
        h = ctypes.c_void_p()
        check(lib().sw_batch_create(self.n, grids, Halo(1, 1, 1, 1), g, dx, ctypes.byref(opts), ctypes.byref(h)),
              "sw_batch_create")
        self.handle = h
        nbytes = ctypes.c_size_t()
        check(lib().sw_batch_arena_bytes(h, ctypes.byref(nbytes)), "sw_batch_arena_bytes")
        self.arena = torch.zeros(nbytes.value, dtype=torch.uint8, device=device)
        check(lib().sw_batch_bind(h, ctypes.c_void_p(self.arena.data_ptr())), "sw_batch_bind")

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.sw_batch_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def _view(self, i):
        st, lay = State(), Layout()
        check(lib().sw_batch_view(self.handle, i, ctypes.byref(st), ctypes.byref(lay)), "sw_batch_view")
        return st, lay

    def halo_view(self, i: int, k: int, buf: int | None = None) -> torch.Tensor:
        st, L = self._view(i)
        b = st.cur if buf is None else buf
        base = st.plane[b][k] - self.arena.data_ptr()
        eb = L.elem_bytes
        nx, ny = self.shapes[i]
        flat = self.arena[base: base + L.plane_elems * eb].view(self.torch_dtype)
        # as_strided's storage offset is absolute within the arena's storage
        return torch.as_strided(flat, (ny + 2, nx + 2), (L.pitch, 1),
                                flat.storage_offset() + L.origin - L.pitch - 1)

    def interior(self, i: int, k: int, buf: int | None = None) -> torch.Tensor:
        return self.halo_view(i, k, buf)[1:-1, 1:-1]

    def set_state(self, i: int, h, hu, hv):
        for k, a in enumerate((h, hu, hv)):
            self.interior(i, k).copy_(torch.as_tensor(a).to(self.torch_dtype))

    def get_state(self, i: int, halo: bool = False):
        torch.cuda.synchronize()
        f = self.halo_view if halo else self.interior
        return tuple(f(i, k).to("cpu", torch.float64) for k in range(3))

    def set_tuning(self, variant=0, rows=0, vec=0, occupancy=0, prefetch=0, order=0):
        check(lib().sw_batch_set_tuning(self.handle, ctypes.byref(Tuning(variant, rows, vec, occupancy, prefetch,
                                                                          order))), "sw_batch_set_tuning")

    def get_tuning(self) -> dict:
        t = Tuning()
        check(lib().sw_batch_get_tuning(self.handle, ctypes.byref(t)), "sw_batch_get_tuning")
        return t.as_dict()

    def set_graph(self, enable: bool):
        check(lib().sw_batch_set_graph(self.handle, 1 if enable else 0), "sw_batch_set_graph")

    def autotune(self, steps_per_trial: int = 3, cache_path: str | None = None, stream=None) -> dict:
        t = Tuning()
        path = cache_path.encode() if cache_path else None
        check(lib().sw_batch_autotune(self.handle, steps_per_trial, path, _stream_handle(stream), ctypes.byref(t)),
              "sw_batch_autotune")
        return t.as_dict()

    def fill_halo(self, stream=None):
        check(lib().sw_batch_fill_halo(self.handle, _stream_handle(stream)), "sw_batch_fill_halo")

    def step(self, nsteps: int, stream=None):
        check(lib().sw_batch_step(self.handle, nsteps, _stream_handle(stream)), "sw_batch_step")

    def sync_status(self, stream=None, raise_unstable=True):
        """Per-grid (t, steps, unstable) arrays."""
        t = (ctypes.c_double * self.n)()
        n = (ctypes.c_int64 * self.n)()
        u = (ctypes.c_int32 * self.n)()
        st = lib().sw_batch_sync_status(self.handle, _stream_handle(stream), t, n, u)
        if st != EUNSTABLE or raise_unstable:
            check(st, "sw_batch_sync_status")
        return list(t), list(n), list(u)

    def reset_time(self, stream=None):
        check(lib().sw_batch_reset_time(self.handle, _stream_handle(stream)), "sw_batch_reset_time")

    def export(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """All (equal-size) grids' current state as a dense [n][3][ny][nx] device tensor."""
        nx, ny = self.shapes[0]
        if out is None:
            out = torch.empty((self.n, 3, ny, nx), dtype=self.torch_dtype, device="cuda")
        elif (not isinstance(out, torch.Tensor) or tuple(out.shape) != (self.n, 3, ny, nx) or not out.is_cuda
              or out.dtype != self.torch_dtype or not out.is_contiguous()):
            raise ValueError(f"out: expected a contiguous {self.torch_dtype} device tensor of shape {(self.n, 3, ny, nx)}")
        check(lib().sw_batch_export(self.handle, ctypes.c_void_p(out.data_ptr()), _stream_handle()), "sw_batch_export")
        return out

    def load(self, dense: torch.Tensor):
        """Set every grid's current state from a dense [n][3][ny][nx] device tensor."""
        nx, ny = self.shapes[0]
        d = _device_tensor(dense, (self.n, 3, ny, nx), self.torch_dtype, "dense")
        check(lib().sw_batch_import(self.handle, ctypes.c_void_p(d.data_ptr()), _stream_handle()), "sw_batch_import")
        torch.cuda.synchronize()


# per layer (cin, cout) of the surrogate; master layout: W[co][tap][ci] then b[co]
SURROGATE_LAYERS = [(3, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 3)]


_hip = None


def _hip_d2d(dst: int, src: int, nbytes: int):
    """Synchronous device-to-device copy (library-owned memory <-> tensors)."""
    global _hip
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip.hipMemcpy.restype = ctypes.c_int
    rc = _hip.hipMemcpy(ctypes.c_void_p(dst), ctypes.c_void_p(src), nbytes, 3)
    if rc != 0:
        raise SwError(EHIP, "hipMemcpy", f"error {rc}")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _device_tensor(t, shape, dtype, name: str, convert: bool = True) -> torch.Tensor:
    """A contiguous device tensor of exactly this shape and dtype (converted
    if allowed), so the library never reads or writes past its end."""
    if not isinstance(t, torch.Tensor) or tuple(t.shape) != tuple(shape):
        got = tuple(t.shape) if isinstance(t, torch.Tensor) else type(t).__name__
        raise ValueError(f"{name}: expected shape {tuple(shape)}, got {got}")
    if not t.is_cuda:
        raise ValueError(f"{name}: expected a device tensor")
    if t.dtype != dtype:
        if not convert:
            raise ValueError(f"{name}: expected {dtype}, got {t.dtype}")
        t = t.to(dtype)
    return t.contiguous()


class Surrogate:
    """The learned surrogate (sw_surrogate_*) for H x W grids."""

    def __init__(self, H: int, W: int, max_batch: int, jump: int = 8, seed: int = 0,
                 bc_x: int = REFLECT, bc_y: int = REFLECT):
        cfg = NetCfg(6, 32, jump, bc_x, bc_y, 0, seed)
        h = ctypes.c_void_p()
        check(lib().sw_surrogate_create(ctypes.byref(cfg), H, W, max_batch, ctypes.byref(h)), "sw_surrogate_create")
        self.handle, self.H, self.W, self.max_batch, self.jump = h, H, W, max_batch, jump
        p, n = ctypes.c_void_p(), ctypes.c_int64()
        check(lib().sw_surrogate_params(h, ctypes.byref(p), ctypes.byref(n)), "sw_surrogate_params")
        self.nparams = n.value
        self._master_ptr = p.value
        self.loss = torch.zeros(1, dtype=torch.float32, device="cuda")

    def __del__(self):
        try:
            if getattr(self, "handle", None) and _lib is not None:
                _lib.sw_surrogate_destroy(self.handle)
                self.handle = None
        except Exception:
            pass

    def get_params(self) -> torch.Tensor:
        out = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        torch.cuda.synchronize()
        _hip_d2d(out.data_ptr(), self._master_ptr, self.nparams * 4)
        return out

    def set_params(self, params):
        t = torch.as_tensor(params, dtype=torch.float32).to("cuda").contiguous()
        if t.numel() != self.nparams:
            raise ValueError(f"expected {self.nparams} parameters, got {t.numel()}")
        torch.cuda.synchronize()
        _hip_d2d(self._master_ptr, t.data_ptr(), self.nparams * 4)
        check(lib().sw_surrogate_sync_weights(self.handle, _stream_handle()), "sw_surrogate_sync_weights")
        torch.cuda.synchronize()

    def set_norm(self, in_offset, in_scale, out_scale):
        f3 = ctypes.c_float * 3
        check(lib().sw_surrogate_set_norm(self.handle, f3(*in_offset), f3(*in_scale), f3(*out_scale)),
              "sw_surrogate_set_norm")

    def set_graph(self, enable: bool):
        """Unjudged rollouts replay captured graphs (True, the default) or launch eagerly."""
        check(lib().sw_surrogate_set_graph(self.handle, 1 if enable else 0), "sw_surrogate_set_graph")

    def set_block_cap(self, max_blocks: int):
        """Cap the persistent convolution / weight-gradient grids (0: one block per resident slot)."""
        check(lib().sw_surrogate_set_block_cap(self.handle, max_blocks), "sw_surrogate_set_block_cap")

    def set_fused(self, mode):
        """Rollout network form: 1 / True one fused launch per jump, 0 / False one launch
        per layer, 2 (the default) whichever the batch size favours."""
        check(lib().sw_surrogate_set_fused(self.handle, int(mode)), "sw_surrogate_set_fused")

    def forward(self, u: torch.Tensor) -> torch.Tensor:
        """u: [B][3][H][W] FP32 on the GPU -> normalised delta [B][H][W][4]."""
        B = u.shape[0] if isinstance(u, torch.Tensor) and u.dim() == 4 else -1
        u = _device_tensor(u, (B, 3, self.H, self.W), torch.float32, "u")
        out = torch.empty((B, self.H, self.W, 4), dtype=torch.float32, device="cuda")
        check(lib().sw_surrogate_forward(self.handle, _ptr(u), B, _ptr(out), _stream_handle()),
              "sw_surrogate_forward")
        return out

    def activation(self, layer: int, B: int) -> torch.Tensor:
        if not 1 <= B <= self.max_batch:
            raise ValueError(f"B = {B} outside [1, {self.max_batch}]")
        p, nb = ctypes.c_void_p(), ctypes.c_int64()
        check(lib().sw_surrogate_activation(self.handle, layer, ctypes.byref(p), ctypes.byref(nb)),
              "sw_surrogate_activation")
        torch.cuda.synchronize()
        if layer == 6:
            n = B * self.H * self.W * 4
            buf = torch.empty(n, dtype=torch.float32, device="cuda")
            shape = (B, self.H, self.W, 4)
            nbytes = n * 4
        else:
            ch = 8 if layer == 0 else 32
            shape = (B, self.H + 2, self.W + 2, ch)
            n = B * (self.H + 2) * (self.W + 2) * ch
            buf = torch.empty(n, dtype=torch.bfloat16, device="cuda")
            nbytes = n * 2
        _hip_d2d(buf.data_ptr(), p.value, nbytes)
        return buf.view(shape)

    def _pair(self, u, u8):
        B = u.shape[0] if isinstance(u, torch.Tensor) and u.dim() == 4 else -1
        shape = (B, 3, self.H, self.W)
        return B, _device_tensor(u, shape, torch.float32, "u"), _device_tensor(u8, shape, torch.float32, "u8")

    def grad(self, u, u8):
        B, u, u8 = self._pair(u, u8)
        g = torch.empty(self.nparams, dtype=torch.float32, device="cuda")
        check(lib().sw_surrogate_grad(self.handle, _ptr(u), _ptr(u8), B, _ptr(g), _ptr(self.loss), _stream_handle()),
              "sw_surrogate_grad")
        return g, self.loss

    def train_step(self, u, u8, lr: float):
        B, u, u8 = self._pair(u, u8)
        check(lib().sw_surrogate_train_step(self.handle, _ptr(u), _ptr(u8), B, lr, _ptr(self.loss),
                                            _stream_handle()), "sw_surrogate_train_step")
        return self.loss

    def advance(self, batch: "Batch", nsteps: int, mass_rel_tol=1e-4, hmin=0.0, project_mass=True,
                fallbacks: torch.Tensor | None = None, judge: bool = False, l2_tol: float = 1e-2,
                l2: torch.Tensor | None = None):
        """Gated rollout of `batch` by nsteps; fallbacks (int32, n) counts the
        rejected jumps; in judge mode l2 (float64, n) receives each grid's
        relative L2(h) against the plain solver."""
        for t, dt, name in ((fallbacks, torch.int32, "fallbacks"), (l2, torch.float64, "l2")):
            if t is not None and (t.dtype != dt or not t.is_cuda or not t.is_contiguous() or t.numel() < batch.n):
                raise ValueError(f"{name}: contiguous {dt} device tensor of {batch.n} entries expected")
        gate = Gate(mass_rel_tol, hmin, 1 if project_mass else 0, 1 if judge else 0, l2_tol)
        check(lib().sw_surrogate_advance(self.handle, batch.handle, nsteps, ctypes.byref(gate), _ptr(fallbacks),
                                         _ptr(l2), _stream_handle()), "sw_surrogate_advance")
