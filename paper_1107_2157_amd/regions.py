"""Region expressions: a small front end for the paper's data-parallel
kernels, and a generator of one HIP tile kernel from them.

The paper (sections "Region functions" and "Source-To-Source
Transformations") writes a stencil kernel as whole-array statements over
*regions*: ``region_cpy(A, halo)`` is the part of array ``A`` left after
trimming ``halo = [left, right, down, up]`` elements from its four sides,
``region_ptr(A, halo)`` the same part of an output array as a writable view.
Elemental functions act element by element.  Arrays carry their halo in
memory; global boundary values are applied outside the kernel.

This module reads such a program (the ``.rgn`` language below), checks it,
hoists elemental calls that the program repeats on shifted regions into
temporaries of their own (the same operations on the same values, so the
same bits, with fewer of them), and emits a HIP kernel in the paper's
generated design mapped onto gfx950:
one thread per output element; every input array is copied with the halo
its regions need into LDS by the thread block; array temporaries (face
quantities) are evaluated over the part of their extent the block needs and
kept in LDS; block barriers separate the phases; output views become one
store per thread.  It also interprets the program with numpy (the
whole-array semantics of the source), which gives the language its meaning
independently of the generated code.

The language, one statement per line (``#`` starts a comment)::

    kernel NAME
    scalar dt, dx, dy, g           # values the runtime passes in
    in H, U, V                     # state arrays with a one-element halo
    out oH, oU, oV                 # output arrays, same shape
    elemental f(a, b) = EXPR       # inline function of scalars
    west = [0, 1, 1, 1]            # a halo vector (may be reassigned)
    stencil s(A, B) = EXPR         # an expression over regions of array parameters,
                                   # expanded where it is applied: s(H, U)
    Hx = EXPR                      # an array temporary; its extent is the expression's
    pH = region_ptr(oH, interior)  # a writable view of an output array
    pH = EXPR                      # stores into the view

EXPR is built from numbers, scalars, ``region_cpy(ARRAY, HALO)``, calls of
elemental functions, ``+ - * /``, unary minus, ``**2`` and parentheses.
Every binary operation between arrays requires equal extents, so an
off-by-one region is reported before any code exists.  Extents are kept
symbolically as ``(nx + a, ny + b)``: the output views define ``nx x ny``.

    python -m paper_1107_2157_amd.regions [--check]

regenerates (or, with ``--check``, verifies) ``csrc/sw_rgn_wave_advance.hip``
from ``wave_advance.rgn``.
"""
from __future__ import annotations

import argparse
import os
import re
import sys
from dataclasses import dataclass, field

HERE = os.path.dirname(os.path.abspath(__file__))
PROGRAM = os.path.join(HERE, "wave_advance.rgn")
GENERATED = os.path.join(HERE, "csrc", "sw_rgn_wave_advance.hip")


class RegionError(ValueError):
    """A program the front end rejects (syntax, unknown name, extent mismatch)."""


# ---------------------------------------------------------------------------
# Expressions

@dataclass(frozen=True)
class Num:
    value: float


@dataclass(frozen=True)
class Sym:
    name: str                      # a scalar or an elemental function's parameter


@dataclass(frozen=True)
class Region:
    array: str
    halo: tuple                    # (left, right, down, up), resolved when parsed


@dataclass(frozen=True)
class Neg:
    a: object


@dataclass(frozen=True)
class Bin:
    op: str
    a: object
    b: object


@dataclass(frozen=True)
class Square:
    a: object


@dataclass(frozen=True)
class Call:
    fn: str
    args: tuple


_TOKEN = re.compile(r"\s*(?:(\d+\.\d*(?:[eE][-+]?\d+)?|\.\d+(?:[eE][-+]?\d+)?|\d+(?:[eE][-+]?\d+)?)"
                    r"|([A-Za-z_][A-Za-z_0-9]*)|(\*\*|[-+*/(),\[\]=]))")


def tokenize(text: str, line: int):
    pos, out = 0, []
    text = text.rstrip()
    while pos < len(text):
        m = _TOKEN.match(text, pos)
        if not m or m.end() == pos:
            raise RegionError(f"line {line}: cannot read {text[pos:]!r}")
        num, name, op = m.groups()
        out.append(("num", num) if num else ("name", name) if name else ("op", op))
        pos = m.end()
    return out


class _Parser:
    def __init__(self, toks, line, prog, array_params=()):
        self.toks, self.i, self.line, self.prog = toks, 0, line, prog
        self.array_params = tuple(array_params)     # names standing for arrays in a stencil's body

    def peek(self):
        return self.toks[self.i] if self.i < len(self.toks) else (None, None)

    def take(self, kind=None, value=None):
        k, v = self.peek()
        if k is None or (kind and k != kind) or (value and v != value):
            raise RegionError(f"line {self.line}: expected {value or kind}, found {v!r}")
        self.i += 1
        return v

    def done(self):
        if self.i != len(self.toks):
            raise RegionError(f"line {self.line}: unexpected {self.toks[self.i][1]!r}")

    def expr(self, params=()):
        e = self.term(params)
        while self.peek() in (("op", "+"), ("op", "-")):
            op = self.take()
            e = Bin(op, e, self.term(params))
        return e

    def term(self, params):
        e = self.unary(params)
        while self.peek() in (("op", "*"), ("op", "/")):
            op = self.take()
            e = Bin(op, e, self.unary(params))
        return e

    def unary(self, params):
        if self.peek() == ("op", "-"):
            self.take()
            return Neg(self.unary(params))
        e = self.atom(params)
        if self.peek() == ("op", "**"):
            self.take()
            if self.take("num") != "2":
                raise RegionError(f"line {self.line}: only **2 is supported")
            e = Square(e)
        return e

    def atom(self, params):
        k, v = self.peek()
        if k == "num":
            self.take()
            return Num(float(v))
        if (k, v) == ("op", "("):
            self.take()
            e = self.expr(params)
            self.take("op", ")")
            return e
        name = self.take("name")
        if name == "region_cpy":
            arr, halo = self.region_args()
            if arr in self.array_params:
                if halo not in self.prog.halos:
                    raise RegionError(f"line {self.line}: unknown halo {halo!r}")
                return Region(arr, self.prog.halos[halo])
            if arr not in self.prog.arrays:
                raise RegionError(f"line {self.line}: region_cpy of unknown array {arr!r}")
            if arr in self.prog.outputs:
                raise RegionError(f"line {self.line}: region_cpy of output array {arr!r}")
            if halo not in self.prog.halos:
                raise RegionError(f"line {self.line}: unknown halo {halo!r}")
            return Region(arr, self.prog.halos[halo])
        if name == "region_ptr":
            raise RegionError(f"line {self.line}: region_ptr may only start a view assignment")
        if name in self.prog.stencils and self.peek() == ("op", "("):
            return self.stencil_call(name)
        if self.peek() == ("op", "("):
            self.take()
            args = [self.expr(params)]
            while self.peek() == ("op", ","):
                self.take()
                args.append(self.expr(params))
            self.take("op", ")")
            if name not in self.prog.elementals:
                raise RegionError(f"line {self.line}: unknown function {name!r}")
            if len(args) != len(self.prog.elementals[name].params):
                raise RegionError(f"line {self.line}: {name} takes {len(self.prog.elementals[name].params)} arguments")
            return Call(name, tuple(args))
        if name in params or name in self.prog.scalars:
            return Sym(name)
        if name in self.prog.arrays:
            raise RegionError(f"line {self.line}: array {name!r} used without region_cpy")
        raise RegionError(f"line {self.line}: unknown name {name!r}")

    def stencil_call(self, name):
        """A stencil applied to arrays: its body with each array parameter
        replaced by the array passed for it."""
        st = self.prog.stencils[name]
        self.take("op", "(")
        args = [self.take("name")]
        while self.peek() == ("op", ","):
            self.take()
            args.append(self.take("name"))
        self.take("op", ")")
        if len(args) != len(st.params):
            raise RegionError(f"line {self.line}: {name} takes {len(st.params)} arrays")
        for a in args:
            if a not in self.prog.arrays and a not in self.array_params:
                raise RegionError(f"line {self.line}: {name} of unknown array {a!r}")
            if a in self.prog.outputs:
                raise RegionError(f"line {self.line}: {name} reads output array {a!r}")
        bind = dict(zip(st.params, args))
        return _rewrite(st.body, lambda x: Region(bind[x.array], x.halo)
                        if isinstance(x, Region) and x.array in bind else None)

    def region_args(self):
        """(ARRAY, HALO) of region_cpy / region_ptr: both plain names."""
        self.take("op", "(")
        arr = self.take("name")
        self.take("op", ",")
        halo = self.take("name")
        self.take("op", ")")
        return arr, halo


@dataclass
class Elemental:
    params: tuple
    body: object


@dataclass
class Stencil:
    params: tuple      # array parameters
    body: object       # expression over region_cpy(param, halo), scalars and elemental calls


@dataclass
class Program:
    name: str = ""
    scalars: list = field(default_factory=list)
    inputs: list = field(default_factory=list)
    outputs: list = field(default_factory=list)
    elementals: dict = field(default_factory=dict)
    stencils: dict = field(default_factory=dict)    # name -> Stencil (expanded where called)
    arrays: dict = field(default_factory=dict)      # name -> extent (a, b): (nx + a, ny + b)
    temps: list = field(default_factory=list)       # [(name, expr)] in order
    views: dict = field(default_factory=dict)       # view -> (output array, halo)
    stores: list = field(default_factory=list)      # [(view, expr)]
    halos: dict = field(default_factory=dict)


def extent_of(prog: Program, e, line: int):
    """Extent (a, b) of an array-valued expression (nx + a, ny + b), or None for a scalar."""
    if isinstance(e, (Num, Sym)):
        return None
    if isinstance(e, Region):
        a, b = prog.arrays[e.array]
        l, r, d, u = e.halo
        return (a - l - r, b - d - u)
    if isinstance(e, (Neg, Square)):
        return extent_of(prog, e.a, line)
    if isinstance(e, Bin):
        ea, eb = extent_of(prog, e.a, line), extent_of(prog, e.b, line)
        if ea is not None and eb is not None and ea != eb:
            raise RegionError(f"line {line}: extents differ: {fmt_extent(ea)} {e.op} {fmt_extent(eb)}")
        return ea if ea is not None else eb
    if isinstance(e, Call):
        ext = None
        for x in e.args:
            ex = extent_of(prog, x, line)
            if ex is not None and ext is not None and ex != ext:
                raise RegionError(f"line {line}: arguments of {e.fn} differ in extent: "
                                  f"{fmt_extent(ext)} and {fmt_extent(ex)}")
            ext = ext if ext is not None else ex
        return ext
    raise TypeError(e)


def fmt_extent(ext):
    def one(n, a):
        return n if a == 0 else f"{n}{a:+d}"
    return f"({one('nx', ext[0])}, {one('ny', ext[1])})"


def parse(text: str) -> Program:
    prog = Program()
    for ln, raw in enumerate(text.splitlines(), 1):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        head = line.split(None, 1)
        if head[0] == "kernel":
            prog.name = head[1].strip()
            continue
        if head[0] in ("scalar", "in", "out"):
            names = [x.strip() for x in head[1].split(",")]
            for n in names:
                if not re.fullmatch(r"[A-Za-z_]\w*", n):
                    raise RegionError(f"line {ln}: bad name {n!r}")
                if n in prog.arrays or n in prog.scalars:
                    raise RegionError(f"line {ln}: {n!r} declared twice")
            if head[0] == "scalar":
                prog.scalars += names
            else:
                (prog.inputs if head[0] == "in" else prog.outputs).extend(names)
                for n in names:
                    prog.arrays[n] = (2, 2)          # a one-element halo on every side
            continue
        if head[0] == "stencil":
            m = re.fullmatch(r"stencil\s+([A-Za-z_]\w*)\s*\(([^)]*)\)\s*=\s*(.+)", line)
            if not m:
                raise RegionError(f"line {ln}: bad stencil definition")
            fn, params = m.group(1), tuple(x.strip() for x in m.group(2).split(","))
            if fn in prog.elementals or fn in prog.stencils:
                raise RegionError(f"line {ln}: {fn!r} defined twice")
            for x in params:
                if not re.fullmatch(r"[A-Za-z_]\w*", x) or x in prog.arrays or x in prog.scalars:
                    raise RegionError(f"line {ln}: bad stencil parameter {x!r}")
            p = _Parser(tokenize(m.group(3), ln), ln, prog, params)
            body = p.expr()
            p.done()
            prog.stencils[fn] = Stencil(params, body)
            continue
        if head[0] == "elemental":
            m = re.fullmatch(r"elemental\s+([A-Za-z_]\w*)\s*\(([^)]*)\)\s*=\s*(.+)", line)
            if not m:
                raise RegionError(f"line {ln}: bad elemental definition")
            fn, params = m.group(1), tuple(x.strip() for x in m.group(2).split(","))
            p = _Parser(tokenize(m.group(3), ln), ln, prog)
            body = p.expr(params)
            p.done()
            if extent_of(prog, body, ln) is not None:
                raise RegionError(f"line {ln}: elemental {fn} must not read arrays")
            prog.elementals[fn] = Elemental(params, body)
            continue
        toks = tokenize(line, ln)
        if len(toks) < 3 or toks[0][0] != "name" or toks[1] != ("op", "="):
            raise RegionError(f"line {ln}: expected an assignment")
        target = toks[0][1]
        rest = toks[2:]
        if rest[0] == ("op", "["):                  # halo vector
            vals, i = [], 1
            while True:
                sign = -1 if rest[i] == ("op", "-") else 1
                i += sign < 0
                if rest[i][0] != "num" or "." in rest[i][1]:
                    raise RegionError(f"line {ln}: halo entries are integers")
                vals.append(sign * int(rest[i][1]))
                i += 1
                if rest[i] == ("op", "]"):
                    break
                if rest[i] != ("op", ","):
                    raise RegionError(f"line {ln}: bad halo vector")
                i += 1
            if len(vals) != 4 or min(vals) < 0 or i != len(rest) - 1:
                raise RegionError(f"line {ln}: a halo is [left, right, down, up], non-negative")
            prog.halos[target] = tuple(vals)
            continue
        if rest[0] == ("name", "region_ptr"):       # a view of an output array
            p = _Parser(rest[1:], ln, prog)
            arr, halo = p.region_args()
            p.done()
            if arr not in prog.outputs:
                raise RegionError(f"line {ln}: region_ptr needs an output array, not {arr!r}")
            if halo not in prog.halos:
                raise RegionError(f"line {ln}: unknown halo {halo!r}")
            if target in prog.views or target in prog.arrays:
                raise RegionError(f"line {ln}: {target!r} already defined")
            prog.views[target] = (arr, prog.halos[halo])
            continue
        p = _Parser(rest, ln, prog)
        e = p.expr()
        p.done()
        ext = extent_of(prog, e, ln)
        if target in prog.views:
            arr, halo = prog.views[target]
            a, b = prog.arrays[arr]
            vext = (a - halo[0] - halo[1], b - halo[2] - halo[3])
            if ext is not None and ext != vext:
                raise RegionError(f"line {ln}: {target} has extent {fmt_extent(vext)}, "
                                  f"the expression {fmt_extent(ext)}")
            if any(v == target for v, _ in prog.stores):
                raise RegionError(f"line {ln}: {target} stored twice")
            prog.stores.append((target, e))
            continue
        if target in prog.arrays or target in prog.scalars:
            raise RegionError(f"line {ln}: {target!r} already defined (temporaries are assigned once)")
        if ext is None:
            raise RegionError(f"line {ln}: {target} = a scalar expression; temporaries are arrays")
        prog.arrays[target] = ext
        prog.temps.append((target, e))
    if not prog.stores:
        raise RegionError("the program stores nothing")
    exts = set()
    for v, _ in prog.stores:
        arr, halo = prog.views[v]
        a, b = prog.arrays[arr]
        exts.add((a - halo[0] - halo[1], b - halo[2] - halo[3]))
    if exts != {(0, 0)}:
        raise RegionError(f"the stored views must all have extent (nx, ny); found {sorted(exts)}")
    return prog


def load(path: str = PROGRAM) -> Program:
    with open(path) as f:
        return parse(f.read())


# ---------------------------------------------------------------------------
# Hoisting elemental calls out of shifted regions.

def _call_key(e):
    """(fn, arrays, halo) if `e` applies an elemental function to regions of
    arrays that all use one halo vector, else None."""
    if not isinstance(e, Call) or not e.args or not all(isinstance(x, Region) for x in e.args):
        return None
    halos = {x.halo for x in e.args}
    if len(halos) != 1:
        return None
    return e.fn, tuple(x.array for x in e.args), e.args[0].halo


def _walk(e, fn):
    fn(e)
    if isinstance(e, (Neg, Square)):
        _walk(e.a, fn)
    elif isinstance(e, Bin):
        _walk(e.a, fn)
        _walk(e.b, fn)
    elif isinstance(e, Call):
        for x in e.args:
            _walk(x, fn)


def _rewrite(e, fn):
    r = fn(e)
    if r is not None:
        return r
    if isinstance(e, Neg):
        return Neg(_rewrite(e.a, fn))
    if isinstance(e, Square):
        return Square(_rewrite(e.a, fn))
    if isinstance(e, Bin):
        return Bin(e.op, _rewrite(e.a, fn), _rewrite(e.b, fn))
    if isinstance(e, Call):
        return Call(e.fn, tuple(_rewrite(x, fn) for x in e.args))
    return e


def hoist(prog: Program) -> Program:
    """A program that computes the same elements with fewer operations.
    An elemental function applied to the same arrays under two or more
    different halo vectors, f(region_cpy(A, h1), region_cpy(B, h1)) and
    f(region_cpy(A, h2), region_cpy(B, h2)), evaluates f twice on most
    elements.  Such calls become regions of a new temporary
    T = f(region_cpy(A, 0), region_cpy(B, 0)) over the arrays' whole extent:
    every element of T is the same operations on the same values, so each
    result is bitwise what the original statement computed."""
    zero = (0, 0, 0, 0)
    uses = {}
    for _, e in prog.temps + prog.stores:
        def note(x):
            k = _call_key(x)
            if k is not None:
                uses.setdefault(k[:2], set()).add(k[2])
        _walk(e, note)
    hoisted = {k: f"{k[0]}__{'_'.join(k[1])}" for k, halos in uses.items() if len(halos) > 1}
    if not hoisted:
        return prog
    out = Program(name=prog.name, scalars=list(prog.scalars), inputs=list(prog.inputs), outputs=list(prog.outputs),
                  elementals=dict(prog.elementals), stencils=dict(prog.stencils), arrays=dict(prog.arrays), temps=[],
                  views=dict(prog.views), stores=[], halos=dict(prog.halos))
    defined = set(prog.inputs)

    def sub(x):
        k = _call_key(x)
        if k is None or k[:2] not in hoisted:
            return None
        return Region(hoisted[k[:2]], k[2])

    def define_needed(e):
        # hoisted temporaries this statement reads, defined just before it
        def need(x):
            k = _call_key(x)
            if k is not None and k[:2] in hoisted:
                name = hoisted[k[:2]]
                if name not in defined:
                    fn, arrays = k[:2]
                    body = Call(fn, tuple(Region(a, zero) for a in arrays))
                    out.arrays[name] = prog.arrays[arrays[0]]
                    out.temps.append((name, body))
                    defined.add(name)
        _walk(e, need)

    for name, e in prog.temps:
        define_needed(e)
        out.temps.append((name, _rewrite(e, sub)))
        defined.add(name)
    for view, e in prog.stores:
        define_needed(e)
        out.stores.append((view, _rewrite(e, sub)))
    return out


# ---------------------------------------------------------------------------
# Whole-array semantics (numpy): the meaning of a program.

def interpret(prog: Program, arrays: dict, scalars: dict) -> dict:
    """Evaluate the program on numpy arrays.  ``arrays`` maps every input
    and output name to an array of shape (ny + 2, nx + 2) (rows = y); the
    outputs' viewed parts are overwritten.  Returns ``arrays``."""
    import numpy as np
    vals = dict(arrays)

    def region(name, halo):
        a = vals[name]
        l, r, d, u = halo
        return a[d:a.shape[0] - u, l:a.shape[1] - r]

    def ev(e, env):
        if isinstance(e, Num):
            return e.value
        if isinstance(e, Sym):
            return env[e.name] if e.name in env else scalars[e.name]
        if isinstance(e, Region):
            return region(e.array, e.halo)
        if isinstance(e, Neg):
            return -ev(e.a, env)
        if isinstance(e, Square):
            x = ev(e.a, env)
            return x * x
        if isinstance(e, Bin):
            a, b = ev(e.a, env), ev(e.b, env)
            return {"+": np.add, "-": np.subtract, "*": np.multiply, "/": np.divide}[e.op](a, b)
        if isinstance(e, Call):
            fn = prog.elementals[e.fn]
            return ev(fn.body, dict(zip(fn.params, (ev(x, env) for x in e.args))))
        raise TypeError(e)

    for name, e in prog.temps:
        vals[name] = np.array(ev(e, {}), dtype=np.float64)
    for view, e in prog.stores:
        arr, halo = prog.views[view]
        region(arr, halo)[...] = ev(e, {})
    return arrays


# ---------------------------------------------------------------------------
# Tile analysis and HIP generation.

def reads(e, out=None):
    """(array, (ox, oy)) pairs an expression reads: element k of the
    expression reads element k + (left, down) of the array."""
    out = [] if out is None else out
    if isinstance(e, Region):
        out.append((e.array, (e.halo[0], e.halo[2])))
    elif isinstance(e, (Neg, Square)):
        reads(e.a, out)
    elif isinstance(e, Bin):
        reads(e.a, out)
        reads(e.b, out)
    elif isinstance(e, Call):
        for x in e.args:
            reads(x, out)
    return out


def tile_ranges(prog: Program, tx: int, ty: int) -> dict:
    """Per array, the box [x0, x1) x [y0, y1) of its elements a tile of
    tx x ty output elements needs, relative to the tile's origin (element
    k of every view of the tile is element k + view origin of its array)."""
    need = {}

    def add(name, box):
        if name in need:
            b = need[name]
            need[name] = (min(b[0], box[0]), max(b[1], box[1]), min(b[2], box[2]), max(b[3], box[3]))
        else:
            need[name] = box

    out_box = (0, tx, 0, ty)
    for _, e in prog.stores:
        for arr, (ox, oy) in reads(e):
            add(arr, (ox, tx + ox, oy, ty + oy))
    for name, e in reversed(prog.temps):
        if name not in need:
            continue                                  # a temporary no output reads
        x0, x1, y0, y1 = need[name]
        for arr, (ox, oy) in reads(e):
            add(arr, (x0 + ox, x1 + ox, y0 + oy, y1 + oy))
    return need, out_box


def free_scalars(prog: Program, e, params, out=None) -> list:
    """Program scalars an elemental body reads (passed to it as trailing arguments)."""
    out = [] if out is None else out
    if isinstance(e, Sym) and e.name not in params and e.name not in out:
        out.append(e.name)
    elif isinstance(e, (Neg, Square)):
        free_scalars(prog, e.a, params, out)
    elif isinstance(e, Bin):
        free_scalars(prog, e.a, params, out)
        free_scalars(prog, e.b, params, out)
    elif isinstance(e, Call):
        for x in e.args:
            free_scalars(prog, x, params, out)
        el = prog.elementals[e.fn]
        for n in free_scalars(prog, el.body, el.params):
            if n not in params and n not in out:
                out.append(n)
    return out


def _c_num(v: float) -> str:
    r = repr(float(v))
    return f"T({r})"


def _emit(e, at, prog, boxes, env=None) -> str:
    """C expression of e at relative element `at` = (cx, cy) (C strings)."""
    env = env or {}
    if isinstance(e, Num):
        return _c_num(e.value)
    if isinstance(e, Sym):
        return env.get(e.name, e.name)
    if isinstance(e, Region):
        x0, x1, y0, y1 = boxes[e.array]
        ox, oy = e.halo[0], e.halo[2]
        w = x1 - x0
        return f"s_{e.array}[({at[1]} + {oy - y0}) * {w} + ({at[0]} + {ox - x0})]"
    if isinstance(e, Neg):
        return f"(-{_emit(e.a, at, prog, boxes, env)})"
    if isinstance(e, Square):
        return f"rgn_sq({_emit(e.a, at, prog, boxes, env)})"
    if isinstance(e, Bin):
        return f"({_emit(e.a, at, prog, boxes, env)} {e.op} {_emit(e.b, at, prog, boxes, env)})"
    if isinstance(e, Call):
        el = prog.elementals[e.fn]
        args = [_emit(x, at, prog, boxes, env) for x in e.args]
        args += [env.get(n, n) for n in free_scalars(prog, el.body, el.params)]
        return f"rgn_{e.fn}({', '.join(args)})"
    raise TypeError(e)


TILE_ROWS = (4, 8, 16)      # tile heights the generated file instantiates (64 columns each)
MARCH_ROWS = (4, 8, 16, 32)  # rows per wave of the row-march kernels
MARCH_PREFETCH = (1, 2, 3)   # input rows loaded ahead of the row being updated


# ---------------------------------------------------------------------------
# Row-march code generation.
#
# The second design keeps no LDS tile: a wave owns a strip of 64 columns
# (one lane per column) and walks up its rows.  Every array is placed in
# output coordinates: array X's element e sits at output position
# e - anchor(X), chosen so that its first read is at offset (0, 0).  A read
# of X by a statement evaluated at output position k then sits at k + d
# with d = read offset + anchor(reader) - anchor(X); d.x in {-1, 0, 1}
# becomes a lane shift (DPP), d.y an index into X's ring of rows.  At march
# row j every array holds its rows j + lo .. j + hi in registers (lo, hi =
# the least and greatest d.y at which anything needs it) and computes only
# row j + hi, in program order, so every value it reads is already there.
# Lanes whose values depend on a shift across the wave's edge are invalid;
# the strip's stored columns are the lanes valid for every output.

@dataclass
class MarchPlan:
    anchor: dict          # array -> (ax, ay)
    lo: dict              # array -> least row offset needed
    hi: dict              # array -> greatest row offset needed
    valid: dict           # array -> (first, last) valid lane
    order: list           # arrays in evaluation order (inputs, then temporaries)
    out_lanes: tuple      # (first, last) lane stored
    warmup: int           # march rows before the first stored one


def march_plan(prog: Program) -> MarchPlan:
    anchor, dys = {}, {}
    users = [(("store", v), e, (0, 0)) for v, e in prog.stores]

    def visit(e, a_e, need):
        for arr, (ox, oy) in reads(e):
            if arr not in anchor:
                anchor[arr] = (ox + a_e[0], oy + a_e[1])
            d = (ox + a_e[0] - anchor[arr][0], oy + a_e[1] - anchor[arr][1])
            if abs(d[0]) > 1:
                raise RegionError(f"row march: a read of {arr} {d[0]} columns away (only -1, 0, 1)")
            dys.setdefault(arr, set()).update(n + d[1] for n in need)

    for _, e, a in users:
        visit(e, a, {0})
    for name, e in reversed(prog.temps):
        if name not in anchor:
            continue                                     # read by nothing
        visit(e, anchor[name], dys[name])
    order = [x for x in prog.inputs if x in anchor] + [t for t, _ in prog.temps if t in anchor]
    lo = {x: min(dys[x]) for x in order}
    hi = {x: max(dys[x]) for x in order}
    valid = {x: (0, 63) for x in prog.inputs}

    def lanes(e, a_e):
        first, last = 0, 63
        for arr, (ox, oy) in reads(e):
            dx = ox + a_e[0] - anchor[arr][0]
            f, l = valid[arr]
            first, last = max(first, f - dx), min(last, l - dx)
        return first, last

    for name, e in prog.temps:
        if name in anchor:
            valid[name] = lanes(e, anchor[name])
    out = (0, 63)
    for _, e in prog.stores:
        f, l = lanes(e, (0, 0))
        out = (max(out[0], f), min(out[1], l))
    if out[1] < out[0]:
        raise RegionError("row march: no lane of a 64-lane strip is valid")
    warmup = max(hi[x] - lo[x] for x in order)
    return MarchPlan(anchor, lo, hi, valid, order, out, warmup)


def _emit_march(e, plan: MarchPlan, prog: Program, a_e, row) -> str:
    """C expression of e evaluated at output row offset `row` (relative to
    the march row) for an expression anchored at a_e."""
    if isinstance(e, Num):
        return _c_num(e.value)
    if isinstance(e, Sym):
        return e.name
    if isinstance(e, Region):
        ax, ay = plan.anchor[e.array]
        dx, dy = e.halo[0] + a_e[0] - ax, e.halo[2] + a_e[1] - ay
        reg = f"r_{e.array}[{row + dy - plan.lo[e.array]}]"
        return reg if dx == 0 else (f"rgn_next({reg})" if dx > 0 else f"rgn_prev({reg})")
    if isinstance(e, Neg):
        return f"(-{_emit_march(e.a, plan, prog, a_e, row)})"
    if isinstance(e, Square):
        return f"rgn_sq({_emit_march(e.a, plan, prog, a_e, row)})"
    if isinstance(e, Bin):
        return f"({_emit_march(e.a, plan, prog, a_e, row)} {e.op} {_emit_march(e.b, plan, prog, a_e, row)})"
    if isinstance(e, Call):
        el = prog.elementals[e.fn]
        args = [_emit_march(x, plan, prog, a_e, row) for x in e.args]
        args += list(free_scalars(prog, el.body, el.params))
        return f"rgn_{e.fn}({', '.join(args)})"
    raise TypeError(e)


def _march_kernel(prog: Program, plan: MarchPlan) -> list:
    L = []
    w = L.append
    first, last = plan.out_lanes
    width = last - first + 1
    order_out = {v: prog.outputs.index(prog.views[v][0]) for v, _ in prog.stores}
    w(f"// Row march: a wave owns {width} output columns (lanes {first}..{last} of 64) and ROWS rows;")
    w("// per array, rows j + lo .. j + hi of march row j in registers (anchor, lo, hi, valid lanes):")
    for x in plan.order:
        w(f"//   {x}: anchor {plan.anchor[x]}, rows {plan.lo[x]}..{plan.hi[x]}, lanes {plan.valid[x][0]}..{plan.valid[x][1]}")
    w("// PF input rows beyond the ring are loaded ahead into p_<array> (PF = 0: each")
    w("// row is loaded in the iteration that first reads it).  Tiles: block b runs")
    w("// on XCD b % 8 and every XCD takes a contiguous run of the row-block-major")
    w("// tile sequence, so tiles sharing warm-up rows meet in the same L2.")
    w("template <typename T, int ROWS, int PF>")
    w(f"__global__ __launch_bounds__(256) void k_rgn_{prog.name}_march(SwLaunch a, int nstrips, int nrb) {{")
    w("    const int lane = threadIdx.x & 63;")
    w("    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);")
    w("    const int per_xcd = gridDim.x >> 3;                  // the grid is a multiple of 8 blocks")
    w("    const int tile = (((int)(blockIdx.x & 7) * per_xcd + (int)(blockIdx.x >> 3)) << 2) + wave;")
    w("    const int s = tile % nstrips, rb = tile / nstrips;")
    w("    const int nx = a.nx, ny = a.ny;")
    w("    const int64_t pitch = a.pitch;")
    w("    const double dt_ = step_dt(a);")
    scal = {"dt": "(T)dt_", "dx": "(T)a.dx", "dy": "(T)a.dy", "g": "(T)a.g"}
    for sc in prog.scalars:
        w(f"    const T {sc} = {scal[sc]};")
    w("    double smax = 0.0;")
    w("    bool bad = false;")
    w("    if (rb < nrb) {")
    w(f"        const int col = s * {width} + lane - {first};              // output column of this lane")
    w(f"        const bool store_lane = lane >= {first} && lane <= {last} && col < nx;")
    w("        const int j0 = rb * ROWS, j1 = min(j0 + ROWS, ny);")
    for x in plan.order:
        w(f"        T r_{x}[{plan.hi[x] - plan.lo[x] + 1}];")
    for k, x in enumerate(prog.inputs):
        if x not in plan.anchor:
            continue
        ax, ay = plan.anchor[x]
        w(f"        const T *in_{x} = (const T *)a.in[{k}];")
        w(f"        const int cx_{x} = min(max(col + {ax} - 1, -1), nx);   // element - 1: the cell, clamped to the halo")
        w(f"        T p_{x}[PF > 0 ? PF : 1];")
        w("        if constexpr (PF > 0) {")
        w("            for (int k = 0; k < PF; ++k) {")
        w(f"                const int cy = min(max(j0 - {plan.warmup} + {plan.hi[x]} + k + {ay} - 1, -1), ny);")
        w(f"                p_{x}[k] = in_{x}[(int64_t)cy * pitch + cx_{x}];")
        w("            }")
        w("        }")
    w(f"        for (int j = j0 - {plan.warmup}; j < j1; ++j) {{")
    w("            // shift every ring down one row")
    for x in plan.order:
        n = plan.hi[x] - plan.lo[x] + 1
        if n > 1:
            w(f"            for (int r = 0; r < {n - 1}; ++r) r_{x}[r] = r_{x}[r + 1];")
    for k, x in enumerate(prog.inputs):
        if x not in plan.anchor:
            continue
        ax, ay = plan.anchor[x]
        top = plan.hi[x] - plan.lo[x]
        w(f"            if constexpr (PF > 0) {{   // input {x}: row j + {plan.hi[x]} from the prefetch ring")
        w(f"                r_{x}[{top}] = p_{x}[0];")
        w(f"                for (int k = 0; k + 1 < PF; ++k) p_{x}[k] = p_{x}[k + 1];")
        w(f"                const int cy = min(max(j + {plan.hi[x]} + PF + {ay} - 1, -1), ny);")
        w(f"                p_{x}[PF - 1] = in_{x}[(int64_t)cy * pitch + cx_{x}];")
        w("            } else {")
        w(f"                const int cy = min(max(j + {plan.hi[x]} + {ay} - 1, -1), ny);")
        w(f"                r_{x}[{top}] = in_{x}[(int64_t)cy * pitch + cx_{x}];")
        w("            }")
    for name, e in prog.temps:
        if name not in plan.anchor:
            continue
        top = plan.hi[name] - plan.lo[name]
        w(f"            r_{name}[{top}] = {_emit_march(e, plan, prog, plan.anchor[name], plan.hi[name])};")
    w("            if (j >= j0) {")
    outs = [None] * 3
    for v, e in prog.stores:
        outs[order_out[v]] = f"v_{v}"
        w(f"                const T v_{v} = {_emit_march(e, plan, prog, (0, 0), 0)};")
    w("                if (store_lane) {")
    w("                    const int64_t o = (int64_t)j * pitch + col;")
    for k in range(3):
        w(f"                    ((T *)a.out[{k}])[o] = {outs[k]};")
    w(f"                    const T sp = signal_speed(U3<T>{{{outs[0]}, {outs[1]}, {outs[2]}}}, (T)a.g);")
    w("                    bad |= !(sp <= finite_max<T>());")
    w("                    smax = fmax(smax, (double)sp);")
    w("                }")
    w("            }")
    w("        }")
    w("    }")
    w("    step_epilogue(a, smax, bad, dt_, blockIdx.x == 0 && wave == 0, (int)blockIdx.x * 4 + wave);")
    w("}")
    return L


def _kernel(prog: Program, tx: int, ty: int) -> list:
    """Lines of one tile kernel k_rgn_<name>_<ty> for tiles of tx x ty outputs."""
    boxes, _ = tile_ranges(prog, tx, ty)
    nt = tx * ty
    if nt % 64 or nt > 1024:
        raise RegionError("tx * ty must be a multiple of 64, at most 1024")
    order = {v: prog.outputs.index(prog.views[v][0]) for v, _ in prog.stores}
    L = []
    w = L.append
    w(f"// Tiles of {tx} x {ty} outputs; element ranges per tile, relative to the tile origin:")
    for name in prog.inputs + [t for t, _ in prog.temps]:
        if name in boxes:
            x0, x1, y0, y1 = boxes[name]
            w(f"//   {name}: x [{x0}, {x1}) y [{y0}, {y1}), extent {fmt_extent(prog.arrays[name])}")
    w(f"template <typename T>")
    w(f"__global__ __launch_bounds__({nt}) void k_rgn_{prog.name}_{ty}(SwLaunch a) {{")
    w(f"    constexpr int TX = {tx}, TY = {ty}, NT = {nt};")
    for name in prog.inputs + [t for t, _ in prog.temps]:
        if name in boxes:
            x0, x1, y0, y1 = boxes[name]
            w(f"    __shared__ T s_{name}[{(x1 - x0) * (y1 - y0)}];")
    w("    __shared__ double s_smax[NT / 64];")
    w("    __shared__ int s_bad[NT / 64];")
    w("    const int nx = a.nx, ny = a.ny;")
    w("    const int64_t pitch = a.pitch;")
    w("    const int i0 = blockIdx.x * TX, j0 = blockIdx.y * TY;")
    w("    const double dt_ = step_dt(a);")
    scal = {"dt": "(T)dt_", "dx": "(T)a.dx", "dy": "(T)a.dy", "g": "(T)a.g"}
    for sc in prog.scalars:
        if sc not in scal:
            raise RegionError(f"scalar {sc!r}: the runtime provides dt, dx, dy and g")
        w(f"    const T {sc} = {scal[sc]};")
    w("")
    w("    // copy-in: element p of an input array is cell p - (1, 1); positions past")
    w("    // the array (tiles at the high edges) are clamped and feed no stored element")
    for k, name in enumerate(prog.inputs):
        if name not in boxes:
            continue
        x0, x1, y0, y1 = boxes[name]
        wd, ht = x1 - x0, y1 - y0
        w(f"    for (int e = threadIdx.x; e < {wd * ht}; e += NT) {{")
        w(f"        const int x = e % {wd}, y = e / {wd};")
        w(f"        const int ci = min(i0 + {x0} + x, nx + 1) - 1, cj = min(j0 + {y0} + y, ny + 1) - 1;")
        w(f"        s_{name}[e] = ((const T *)a.in[{k}])[(int64_t)cj * pitch + ci];")
        w("    }")
    w("    __syncthreads();")
    level = {}
    for name, e in prog.temps:
        deps = [arr for arr, _ in reads(e) if arr in level]
        level[name] = 1 + max((level[d] for d in deps), default=0)
    for lv in sorted(set(level.values())):
        w("")
        w(f"    // array temporaries, level {lv}")
        for name, e in prog.temps:
            if level[name] != lv or name not in boxes:
                continue
            x0, x1, y0, y1 = boxes[name]
            wd, ht = x1 - x0, y1 - y0
            w(f"    for (int e = threadIdx.x; e < {wd * ht}; e += NT) {{")
            w(f"        const int mx = e % {wd} + {x0}, my = e / {wd} + {y0};")
            w(f"        s_{name}[e] = {_emit(e, ('mx', 'my'), prog, boxes)};")
            w("    }")
        w("    __syncthreads();")
    w("")
    w("    // output views: one element per thread")
    w("    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;")
    w("    const int i = i0 + tx, j = j0 + ty;")
    w("    double smax = 0.0;")
    w("    bool bad = false;")
    w("    if (i < nx && j < ny) {")
    outs = [None] * 3
    for v, e in prog.stores:
        outs[order[v]] = f"v_{v}"
        w(f"        const T v_{v} = {_emit(e, ('tx', 'ty'), prog, boxes)};")
    w("        const int64_t o = (int64_t)j * pitch + i;")
    for k in range(3):
        w(f"        ((T *)a.out[{k}])[o] = {outs[k]};")
    w(f"        const T sp = signal_speed(U3<T>{{{outs[0]}, {outs[1]}, {outs[2]}}}, (T)a.g);")
    w("        bad = !(sp <= finite_max<T>());")
    w("        smax = (double)sp;")
    w("    }")
    w("    // step epilogue, once per block: max speed of the new state for the next dt")
    w("    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;")
    w("    smax = wave_max(smax);")
    w("    const bool wbad = __ballot(bad) != 0;")
    w("    if (lane == 0) {")
    w("        s_smax[wave] = smax;")
    w("        s_bad[wave] = wbad;")
    w("    }")
    w("    __syncthreads();")
    w("    if (wave == 0) {")
    w("        const double m = lane < NT / 64 ? s_smax[lane] : 0.0;")
    w("        const bool b = lane < NT / 64 ? s_bad[lane] != 0 : false;")
    w("        step_epilogue(a, m, b, dt_, blockIdx.x == 0 && blockIdx.y == 0,")
    w("                      (int)(blockIdx.y * gridDim.x + blockIdx.x));")
    w("    }")
    w("}")
    return L


def generate(prog: Program, tx: int = 64, tile_rows=TILE_ROWS, source_name: str = "wave_advance.rgn",
             optimize: bool = True) -> str:
    """HIP source of the tile kernels for `prog`: one per tile height in
    `tile_rows` (tiles of tx x rows outputs, one thread each; with
    `optimize`, elemental calls on shifted regions are hoisted into
    temporaries first), the row-march kernels (rows per wave x input rows
    loaded ahead), and the launcher sw_launch_rgn(a, design, rows,
    prefetch, stream).
    The runtime around the translated statements (dt from the device-side
    CFL ring, the signal-speed reduction and sticky flag of the step
    epilogue) expects the outputs in the order h, hu, hv."""
    if optimize:
        prog = hoist(prog)
    if len(prog.inputs) != 3 or len(prog.outputs) != 3 or len(prog.stores) != 3:
        raise RegionError("the generated step kernel takes three input and three output arrays")
    L = []
    w = L.append
    w(f"// Generated by paper_1107_2157_amd/regions.py from {source_name}; do not edit.")
    w("//")
    w(f"// Kernel `{prog.name}`: one thread per output element; inputs and array")
    w("// temporaries staged in LDS per tile, barriers between dependency levels.")
    w("// Global boundary values are applied outside the kernel.")
    w('#include "sw_common.h"')
    w("")
    w("using namespace sw;")
    w("")
    w("namespace {")
    w("")
    w("template <typename T> __device__ __forceinline__ T rgn_sq(T x) { return x * x; }")
    for fn, el in prog.elementals.items():
        args = ", ".join(f"T {p}" for p in list(el.params) + free_scalars(prog, el.body, el.params))
        bodyc = _emit(el.body, ("0", "0"), prog, {})
        w(f"template <typename T> __device__ __forceinline__ T rgn_{fn}({args}) {{ return {bodyc}; }}")
    for ty in tile_rows:
        w("")
        L.extend(_kernel(prog, tx, ty))
    plan = march_plan(prog)
    w("")
    w("// x neighbours in the row march: the wave's edge lane receives 0 (it is never")
    w("// a stored column), which lets the compiler fold the shift into its consumer.")
    w("__device__ __forceinline__ float rgn_next(float x) {")
    w("    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x130, 0xf, 0xf, true));")
    w("}")
    w("__device__ __forceinline__ float rgn_prev(float x) {")
    w("    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x138, 0xf, 0xf, true));")
    w("}")
    w("__device__ __forceinline__ double rgn_next(double x) {")
    w("    const long long v = __double_as_longlong(x);")
    w("    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);")
    w("    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x130, 0xf, 0xf, true);")
    w("    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);")
    w("}")
    w("__device__ __forceinline__ double rgn_prev(double x) {")
    w("    const long long v = __double_as_longlong(x);")
    w("    const int lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);")
    w("    const int hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x138, 0xf, 0xf, true);")
    w("    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);")
    w("}")
    w("")
    L.extend(_march_kernel(prog, plan))
    w("")
    width = plan.out_lanes[1] - plan.out_lanes[0] + 1
    w(f"template <typename T> hipError_t launch_{prog.name}_march(const SwLaunch &a, int rows, int prefetch, hipStream_t s) {{")
    w(f"    const int nstrips = (a.nx + {width - 1}) / {width};")
    w("    const int nrb = (a.ny + rows - 1) / rows;")
    w("    int64_t blocks = ((int64_t)nstrips * nrb + 3) / 4;")
    w("    blocks = (blocks + 7) / 8 * 8;                   // whole runs per XCD; the extra tiles are idle")
    w("    if (blocks > 0x1fffffff) return hipErrorInvalidValue;   // 4 * blocks tile indices fit an int")
    first = True
    for r in MARCH_ROWS:
        for p in MARCH_PREFETCH:
            kw = "if" if first else "else if"
            first = False
            w(f"    {kw} (rows == {r} && prefetch == {p}) "
              f"k_rgn_{prog.name}_march<T, {r}, {p - 1}><<<(unsigned)blocks, 256, 0, s>>>(a, nstrips, nrb);")
    w(f"    else return hipErrorInvalidValue;")
    w("    return hipGetLastError();")
    w("}")
    w("")
    w(f"template <typename T> hipError_t launch_{prog.name}(const SwLaunch &a, int rows, hipStream_t s) {{")
    w(f"    const unsigned gx = (unsigned)((a.nx + {tx - 1}) / {tx});")
    for ty in tile_rows:
        w(f"    if (rows == {ty}) {{")
        w(f"        const dim3 grid(gx, (unsigned)((a.ny + {ty - 1}) / {ty}));")
        w(f"        if (grid.y > 65535u) return hipErrorInvalidValue;")
        w(f"        k_rgn_{prog.name}_{ty}<T><<<grid, {tx * ty}, 0, s>>>(a);")
        w("        return hipGetLastError();")
        w("    }")
    w("    return hipErrorInvalidValue;")
    w("}")
    w("")
    w("}  // namespace")
    w("")
    w(f"// Designs: 1 = LDS tiles of {', '.join(str(t) for t in tile_rows)} rows; "
      f"2 = row march of {', '.join(str(t) for t in MARCH_ROWS)} rows per wave.")
    w("bool sw_rgn_rows_supported(int design, int rows) {")
    w(f"    if (design == 1) return {' || '.join(f'rows == {t}' for t in tile_rows)};")
    w(f"    if (design == 2) return {' || '.join(f'rows == {t}' for t in MARCH_ROWS)};")
    w("    return false;")
    w("}")
    w("")
    w("hipError_t sw_launch_rgn(const SwLaunch &a, int design, int rows, int prefetch, hipStream_t s) {")
    w("    if (a.scheme != 0) return hipErrorInvalidValue;")
    w("    if (design == 2)")
    w(f"        return a.dtype == 0 ? launch_{prog.name}_march<float>(a, rows, prefetch, s)")
    w(f"                            : launch_{prog.name}_march<double>(a, rows, prefetch, s);")
    w("    if (prefetch != 0) return hipErrorInvalidValue;")
    w(f"    return a.dtype == 0 ? launch_{prog.name}<float>(a, rows, s) : launch_{prog.name}<double>(a, rows, s);")
    w("}")
    return "\n".join(L) + "\n"


def write_generated() -> bool:
    """Regenerate the kernel source from the program; write it only if it
    changed.  Returns True if the file was written."""
    src = generate(load(PROGRAM))
    if os.path.exists(GENERATED):
        with open(GENERATED) as f:
            if f.read() == src:
                return False
    with open(GENERATED, "w") as f:
        f.write(src)
    return True


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--check", action="store_true", help="fail if the generated file is not up to date")
    args = ap.parse_args(argv)
    src = generate(load(PROGRAM))
    if args.check:
        with open(GENERATED) as f:
            if f.read() != src:
                print(f"{GENERATED} is out of date; run python -m paper_1107_2157_amd.regions", file=sys.stderr)
                return 1
        return 0
    with open(GENERATED, "w") as f:
        f.write(src)
    print(f"wrote {GENERATED}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
