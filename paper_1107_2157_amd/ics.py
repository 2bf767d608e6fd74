"""Seeded synthetic initial states for the shallow-water workloads.

This module is shared input plumbing: it draws random numbers and lays out
initial water heights, and holds none of the solver's arithmetic (no fluxes,
no half-steps, no boundary handling, no time step).  Both the CPU oracle and
the HIP path are fed from here, so a parity test hands the same arrays to
both sides.

The paper (Section "Shallow Water Model") states no initial condition; the
recipes below are the workload definitions this library measures on:

* dam break: still water of depth 1 with a centred square of depth 2;
* Gaussian bumps: ``h = 1 + sum_k a_k exp(-r_k^2 / (2 sigma_k^2))`` at cell
  centres ``((i + 1/2) dx, (j + 1/2) dy)``, centres uniform over the domain,
  ``a ~ U[0.05, 0.5]``, ``sigma ~ U[16, 128]`` cells; periodic domains use the
  minimum-image distance.  The Gaussian is evaluated in its separable form
  ``exp(-dx^2/2s^2) * exp(-dy^2/2s^2)`` (it is the definition of the input,
  not of the method).
* random numbers come from SplitMix64 (Steele, Lea, Flood 2014); a double in
  [0, 1) is ``(x >> 11) * 2^-53``.  Draw order: bump count (when drawn:
  ``1 + floor(8 u)``), then per bump ``(cx, cy, a, sigma)``.

All arrays are returned as interior-only ``(ny, nx)`` float64 torch tensors
(row-major, x fastest); momenta ``hu = hv = 0`` unless stated.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import torch

_MASK = (1 << 64) - 1

# Seeds of the named workloads.
SEED_BUMPS_4096 = 2
SEED_BUMPS_16384 = 3
SEED_BATCH_SIDES = 4
SEED_BATCH_GRID0 = 4000
SEED_TRAJ0 = 5000
SEED_SURR_EVAL0 = 9000


class SplitMix64:
    """SplitMix64 generator (Steele, Lea & Flood, OOPSLA 2014)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (2.0 ** -53)


@dataclass(frozen=True)
class Bump:
    cx: float      # centre x (physical units)
    cy: float      # centre y
    amp: float     # amplitude a
    sigma: float   # width (physical units)


def draw_bumps(seed: int, nx: int, ny: int, dx: float = 1.0, dy: float = 1.0,
               count: int | None = None) -> list[Bump]:
    """Draw the bump parameters; ``count=None`` draws ``1 + floor(8u)``."""
    rng = SplitMix64(seed)
    if count is None:
        count = 1 + int(math.floor(8.0 * rng.uniform()))
    out = []
    for _ in range(count):
        cx = rng.uniform() * nx * dx
        cy = rng.uniform() * ny * dy
        amp = 0.05 + 0.45 * rng.uniform()
        sigma = (16.0 + 112.0 * rng.uniform()) * dx
        out.append(Bump(cx, cy, amp, sigma))
    return out


def _axis_gauss(n: int, d: float, c: float, sigma: float, periodic: bool,
                device) -> torch.Tensor:
    x = (torch.arange(n, dtype=torch.float64, device=device) + 0.5) * d
    r = x - c
    if periodic:
        length = n * d
        r = r - length * torch.round(r / length)
    return torch.exp(-(r * r) / (2.0 * sigma * sigma))


def bumps_height(nx: int, ny: int, bumps: list[Bump], periodic: bool,
                 dx: float = 1.0, dy: float = 1.0, device="cpu") -> torch.Tensor:
    """``h = 1 + sum of Gaussian bumps`` on the ``(ny, nx)`` interior."""
    h = torch.ones((ny, nx), dtype=torch.float64, device=device)
    for b in bumps:
        gx = _axis_gauss(nx, dx, b.cx, b.sigma, periodic, device)
        gy = _axis_gauss(ny, dy, b.cy, b.sigma, periodic, device)
        h.addr_(gy, gx, alpha=b.amp)
    return h


def bumps_band(nx: int, ny: int, row0: int, nrows: int, seed: int, periodic: bool,
               count: int | None = None, dx: float = 1.0, dy: float = 1.0, device="cpu"):
    """Rows ``[row0, row0 + nrows)`` of the ``(ny, nx)`` bump state (same
    bumps as the full grid), for runs on a horizontal band of it."""
    bumps = draw_bumps(seed, nx, ny, dx, dy, count)
    h = torch.ones((nrows, nx), dtype=torch.float64, device=device)
    for b in bumps:
        gx = _axis_gauss(nx, dx, b.cx, b.sigma, periodic, device)
        gy = _axis_gauss(ny, dy, b.cy, b.sigma, periodic, device)[row0:row0 + nrows]
        h.addr_(gy, gx, alpha=b.amp)
    z = torch.zeros_like(h)
    return h, z, z.clone()


def bumps_state(nx: int, ny: int, seed: int, periodic: bool, count: int | None = None,
                dx: float = 1.0, dy: float = 1.0, device="cpu"):
    """Gaussian-bump still-water state ``(h, hu, hv)``."""
    bumps = draw_bumps(seed, nx, ny, dx, dy, count)
    h = bumps_height(nx, ny, bumps, periodic, dx, dy, device)
    z = torch.zeros_like(h)
    return h, z, z.clone()


def dam_break_state(n: int = 128, device="cpu"):
    """Centred dam break: depth 2 on the square ``[3n/8, 5n/8)^2`` (0-based
    interior cells), depth 1 elsewhere, at rest.  For n = 128 the square is
    ``[48, 80)^2``, which is mirror-symmetric about both centre lines."""
    h = torch.ones((n, n), dtype=torch.float64, device=device)
    lo, hi = (3 * n) // 8, (5 * n) // 8
    h[lo:hi, lo:hi] = 2.0
    z = torch.zeros_like(h)
    return h, z, z.clone()


def batch_sides(count: int = 512, seed: int = SEED_BATCH_SIDES) -> list[int]:
    """Side lengths of the batched workload: ``64 * (1 + floor(16 u))``,
    i.e. uniform over {64, 128, ..., 1024}."""
    rng = SplitMix64(seed)
    return [64 * (1 + int(math.floor(16.0 * rng.uniform()))) for _ in range(count)]


def random_state(nx: int, ny: int, seed: int, amp_h: float = 0.3, amp_m: float = 0.1,
                 device="cpu"):
    """A generic positive state with moving water (for parity on non-trivial
    momenta): ``h in [1, 1 + amp_h)``, ``hu, hv in [-amp_m, amp_m)``, smooth
    enough to be meaningful and rough enough to exercise every term."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    h = 1.0 + amp_h * torch.rand((ny, nx), generator=g, dtype=torch.float64)
    hu = amp_m * (2.0 * torch.rand((ny, nx), generator=g, dtype=torch.float64) - 1.0)
    hv = amp_m * (2.0 * torch.rand((ny, nx), generator=g, dtype=torch.float64) - 1.0)
    return h.to(device), hu.to(device), hv.to(device)
