"""Leapfrog time stepping and the cell timestep criterion (test infrastructure only).

Sec. 2.5, time stepping: particles advance with second-order leapfrog in its
kick-drift-kick form, one global step size for every particle; the step size
is the smallest, over the cells, of the velocity dispersion of the cell divided
by the largest acceleration in it, times eta (0.25 in the simulations).  The
singlestep pipeline of Sec. 3.1 kicks, drifts and then moves the particles to
their new cells before the next force evaluation.

Storage and arithmetic (readings, stated where the paper is silent):

* positions and velocities are stored in FP32, accelerations arrive in FP32;
  a kick v + a dt and a drift x + v dt are evaluated in FP64 from the stored
  values (two roundings: the product, then the sum) and rounded once to FP32;
* a drifted coordinate is wrapped into the box as y - L floor(y / L) in FP64;
  if its FP32 rounding reaches L it is stored as 0 (the same point);
* the velocity dispersion of a cell is the root mean square, over its
  particles, of |v - mean(v)| (all three components, divided by n); cells with
  fewer than two particles or no nonzero acceleration do not constrain the
  step; a box with no constraining cell gets an infinite step;
* one leapfrog step of size dt: v += a(x) dt/2; x += v dt; rebin;
  v += a(x) dt/2, with a from the near-field force of this package (the far
  field is out of scope here).

Everything is plain NumPy in FP64 following those definitions; the force is
passed in (near_field gives the C oracle's near field).
"""
from __future__ import annotations

import numpy as np

from . import oracle as _orc


def kick(vel, acc, dt: float) -> np.ndarray:
    """FP32 velocities after a kick of dt: round32(v + a dt), evaluated in FP64."""
    v = np.asarray(vel, dtype=np.float32).astype(np.float64)
    a = np.asarray(acc, dtype=np.float32).astype(np.float64)
    return (v + a * float(dt)).astype(np.float32)


def drift(pos, vel, dt: float, box: float) -> np.ndarray:
    """FP32 positions after a drift of dt, wrapped into [0, box)."""
    x = np.asarray(pos, dtype=np.float32).astype(np.float64)
    v = np.asarray(vel, dtype=np.float32).astype(np.float64)
    L = float(box)
    y = x + v * float(dt)
    y = y - L * np.floor(y / L)
    f = y.astype(np.float32)
    f[f.astype(np.float64) >= L] = np.float32(0.0)
    return f


def cell_timestep(pos, vel, acc, box: float, K: int, eta: float = 0.25) -> float:
    """eta * min over constraining cells of sigma_v / max |a| (inf if no cell constrains)."""
    cells = _orc.bin_cells(pos, box, K).astype(np.int64)
    v = np.asarray(vel, dtype=np.float32).astype(np.float64)
    a = np.asarray(acc, dtype=np.float32).astype(np.float64)
    best = np.inf
    order = np.argsort(cells, kind="stable")
    bounds = np.searchsorted(cells[order], np.arange(K ** 3 + 1))
    for c in range(K ** 3):
        idx = order[bounds[c]:bounds[c + 1]]
        if idx.size < 2:
            continue
        amax = np.sqrt((a[idx] ** 2).sum(axis=1)).max()
        if not amax > 0:
            continue
        d = v[idx] - v[idx].mean(axis=0)
        sigma = np.sqrt((d ** 2).sum() / idx.size)
        best = min(best, sigma / amax)
    return float(eta * best)


def cell_max_accel(pos, acc, box: float, K: int) -> np.ndarray:
    """Largest |a| over the particles of each cell (FP64 from the FP32 values; 0 for an empty cell), [K^3].

    The per-cell input of the step-size criterion (Sec. 2.5, time stepping)."""
    cells = _orc.bin_cells(pos, box, K).astype(np.int64)
    a = np.asarray(acc, dtype=np.float32).astype(np.float64)
    out = np.zeros(K ** 3)
    np.maximum.at(out, cells, np.sqrt((a ** 2).sum(axis=1)))
    return out


def kdk_step(pos, vel, dt: float, box: float, force, acc=None):
    """One leapfrog step of size dt with accelerations force(pos) (FP64 [n, 3]); returns (pos, vel, acc)
    after the step: FP32 positions and velocities, and the accelerations at the new positions (the next
    step's first kick uses them).  acc, if given, is force(pos) already evaluated."""
    a0 = force(pos) if acc is None else np.asarray(acc, dtype=np.float64)
    vh = kick(vel, a0.astype(np.float32), 0.5 * dt)
    x1 = drift(pos, vh, dt, box)
    a1 = force(x1)
    v1 = kick(vh, a1.astype(np.float32), 0.5 * dt)
    return x1, v1, a1


def near_field(box: float, K: int, R: int, eps: float, kind: int, gm: float):
    """The near-field force of the C oracle as a force(pos) callable for kdk_step."""
    return lambda p: _orc.forces(p, box, K, R, eps, kind, gm)


def kdk_steps(pos, vel, dt, box: float, force):
    """Leapfrog steps of sizes dt[0], dt[1], ...; returns (pos, vel, acc) after the last."""
    x, v, a = pos, vel, None
    for h in np.atleast_1d(dt):
        x, v, a = kdk_step(x, v, float(h), box, force, a)
    return x, v, a
