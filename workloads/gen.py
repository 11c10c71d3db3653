"""Seeded synthetic inputs for the near-field force (Sec. 3.1 problem statement).

The paper measures on its own simulation (base_c000_ph000 at z=90.5, nearly
uniform, and at z=0.105, highly clustered; Table "tbl:timing").  Those snapshots
are not available, so these generators stand in for them with the same shapes:
about 67 particles per cell at R=2 (Sec. 2.5 "Code Parameters"), near-uniform
early times, and halo-dominated late times where the near field dominates the
runtime (Sec. 4.3, Fig. "timing_overiew").

All randomness comes from numpy's PCG64 (``numpy.random.default_rng(seed)``).
Positions are generated in float64 in a box of side ``box`` and cast to float32
at the end; a coordinate that rounds up to ``box`` after the cast is set to 0 so
that every coordinate lies in [0, box).

Recipes (one per workload; the readings where the workload description is
silent are stated next to each):

* ``tiny``      N=32^3 uniform, K=8, eps=(1/32)/40, G*m=1/N.
* ``clustered`` N=256^3, K=64; 50% uniform + 50% in 4096 Plummer halos with
  scale radius a=0.3 cell; halo particle counts from dN/dM ~ M^-1.9 on
  [1, 1000] (range is a reading), rescaled to N/2 by largest-remainder
  rounding; radii by the Plummer inverse CDF truncated at 10a; isotropic
  directions; periodic wrap.  eps=(1/256)/40, G*m=1/N.
* ``precision`` N=512^3, K=128; same generator at the same halo density per
  volume (32768 halos), a=0.3 cell.
* ``batched``   64 boxes; N_b log-uniform in [64^3, 192^3] (seed 4);
  K_b=max(5, round((N_b/48)^(1/3))); 30% clustered in round(N_b/4096) halos,
  a=0.3 cell; eps_b=N_b^(-1/3)/40; G*m_b=1/N_b; box b uses seed 4000+b.
* ``late``      N=2^27, K=256; 50% in 16384 halos with scale radius
  log-uniform in [0.05, 0.5] cell (halo count is a reading chosen so that the
  top 1% of cells hold about half of the particles); masses as ``clustered``.

Synthetic far-field coefficients (``taylor_coefficients``): the paper obtains
them from a convolution that is not part of this code, so every component of
total degree n is drawn as amp * z * r0^-n with z standard normal (PCG64, seed),
a decay like that of the derivatives of 1/r at r0 cell widths (reading: r0 = 3,
the nearest far-field cells; amp chosen per use).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Box:
    """One periodic box: float32 positions [n,3] in [0, box) and its parameters."""
    pos: np.ndarray          # float32 [n, 3]
    box: float               # side length L
    K: int                   # cells per side
    eps: float               # softening length (each kernel's own parameter)
    gm: float                # G * m per particle
    seed: int

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


@dataclasses.dataclass
class Workload:
    name: str
    boxes: List[Box]
    R: int = 2
    description: str = ""

    @property
    def n_total(self) -> int:
        return sum(b.n for b in self.boxes)

    def concat_positions(self) -> np.ndarray:
        return np.concatenate([b.pos for b in self.boxes], axis=0) if self.boxes else np.zeros((0, 3), np.float32)


def _finish(pos64: np.ndarray, box: float) -> np.ndarray:
    """Wrap into [0, box), cast to float32, and map coordinates that round up to box onto 0."""
    pos64 = np.mod(pos64, box)
    p = pos64.astype(np.float32)
    p[p >= np.float32(box)] = np.float32(0.0)
    return p


def uniform_positions(rng: np.random.Generator, n: int, box: float = 1.0) -> np.ndarray:
    """n positions uniform in [0, box)^3 (float32 draws, returned as float64)."""
    return rng.random((n, 3), dtype=np.float32).astype(np.float64) * box


def largest_remainder(weights: np.ndarray, total: int) -> np.ndarray:
    """Integers proportional to ``weights`` that sum exactly to ``total``.

    Floors of the scaled weights, then one extra unit each to the largest
    fractional remainders (ties broken by index).
    """
    w = np.asarray(weights, dtype=np.float64)
    if total == 0 or w.size == 0:
        return np.zeros(w.shape, dtype=np.int64)
    share = w / w.sum() * total
    base = np.floor(share).astype(np.int64)
    short = int(total - base.sum())
    if short > 0:
        order = np.lexsort((np.arange(w.size), -(share - base)))
        base[order[:short]] += 1
    return base


def power_law_masses(rng: np.random.Generator, n_halos: int, alpha: float = 1.9,
                     m_lo: float = 1.0, m_hi: float = 1000.0) -> np.ndarray:
    """n_halos draws from dN/dM ~ M^-alpha on [m_lo, m_hi] by inverse CDF."""
    u = rng.random(n_halos)
    e = 1.0 - alpha
    return (m_lo ** e + u * (m_hi ** e - m_lo ** e)) ** (1.0 / e)


def plummer_halo_positions(rng: np.random.Generator, counts: np.ndarray, scale: np.ndarray,
                           box: float = 1.0, r_max_over_a: float = 10.0) -> np.ndarray:
    """Particles of Plummer-profile halos with uniform random centres.

    counts[h] particles in halo h with scale radius scale[h].  The enclosed-mass
    fraction of a Plummer sphere is r^3/(r^2+a^2)^(3/2); radii are drawn by
    inverting it, restricted to r <= r_max_over_a * a (drawing the mass fraction
    uniformly below its value at the cut is the same as rejecting beyond it).
    Directions are isotropic.  The offsets from the centre are drawn in
    float32 (they are a random sample; their precision is immaterial) and added
    to float64 centres.  Positions are returned in float64, unwrapped.
    """
    counts = np.asarray(counts, dtype=np.int64)
    scale = np.broadcast_to(np.asarray(scale, dtype=np.float64), counts.shape)
    n = int(counts.sum())
    centres = rng.random((counts.size, 3)) * box
    hid = np.repeat(np.arange(counts.size, dtype=np.int32), counts)
    c = r_max_over_a
    m_cut = c ** 3 / (c * c + 1.0) ** 1.5
    f32 = np.float32
    x = rng.random(n, dtype=f32) * f32(m_cut)
    x = np.maximum(x, np.finfo(f32).tiny)
    a = scale.astype(f32)[hid]
    r = a / np.sqrt(x ** f32(-2.0 / 3.0) - f32(1.0))
    cos_t = rng.random(n, dtype=f32) * f32(2.0) - f32(1.0)
    phi = rng.random(n, dtype=f32) * f32(2.0 * np.pi)
    sin_t = np.sqrt(np.maximum(f32(0.0), f32(1.0) - cos_t * cos_t))
    out = np.repeat(centres, counts, axis=0)
    out[:, 0] += r * sin_t * np.cos(phi)
    out[:, 1] += r * sin_t * np.sin(phi)
    out[:, 2] += r * cos_t
    return out


_VERBOSE = False


def set_verbose(on: bool = True):
    """Print the progress of long generations to stderr."""
    global _VERBOSE
    _VERBOSE = bool(on)


def _say(msg: str):
    if _VERBOSE:
        import sys
        import time
        print(f"[gen {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _clustered_box(seed: int, n: int, K: int, frac_halo: float, n_halos: int,
                   scale_cells, box: float = 1.0, shuffle: bool = True) -> np.ndarray:
    """Uniform background plus Plummer halos; returns float32 positions."""
    rng = np.random.default_rng(seed)
    n_h = int(round(n * frac_halo)) if n_halos > 0 else 0
    n_u = n - n_h
    _say(f"box seed {seed}: {n_u} uniform")
    parts = [uniform_positions(rng, n_u, box)]
    if n_h > 0:
        _say(f"box seed {seed}: {n_h} in {n_halos} halos")
        masses = power_law_masses(rng, n_halos)
        counts = largest_remainder(masses, n_h)
        w = box / K
        if callable(scale_cells):
            a = scale_cells(rng, n_halos) * w
        else:
            a = np.full(n_halos, float(scale_cells) * w)
        parts.append(plummer_halo_positions(rng, counts, a, box))
    _say(f"box seed {seed}: wrap and cast")
    pos = _finish(np.concatenate(parts, axis=0), box)
    if shuffle and n > 1:
        _say(f"box seed {seed}: shuffle")
        pos = pos[rng.permutation(n)]
    return pos


def _tiny(seed: int = 1) -> Workload:
    n, K = 32 ** 3, 8
    rng = np.random.default_rng(seed)
    pos = _finish(uniform_positions(rng, n), 1.0)
    sp = 1.0 / round(n ** (1 / 3))
    return Workload("tiny", [Box(pos, 1.0, K, sp / 40.0, 1.0 / n, seed)],
                    description="N=32^3 uniform, K=8, spline eps=spacing/40, G*m=1/N")


def _clustered(seed: int = 2, side: int = 256, K: int = 64, n_halos: int = 4096, name="clustered") -> Workload:
    n = side ** 3
    pos = _clustered_box(seed, n, K, 0.5, n_halos, 0.3)
    return Workload(name, [Box(pos, 1.0, K, (1.0 / side) / 40.0, 1.0 / n, seed)],
                    description=f"N={side}^3, K={K}, 50% uniform + 50% in {n_halos} Plummer halos (a=0.3 cell), "
                                "dN/dM~M^-1.9 on [1,1000], eps=spacing/40, G*m=1/N")


def _precision(seed: int = 3) -> Workload:
    return _clustered(seed, 512, 128, 32768, name="precision")


def _log_uniform_scale(lo: float, hi: float) -> Callable:
    def f(rng, k):
        return np.exp(rng.random(k) * (math.log(hi) - math.log(lo)) + math.log(lo))
    return f


def _late(seed: int = 5, n: int = 2 ** 27, K: int = 256, n_halos: int = 16384) -> Workload:
    pos = _clustered_box(seed, n, K, 0.5, n_halos, _log_uniform_scale(0.05, 0.5))
    sp = 1.0 / n ** (1.0 / 3.0)
    size = f"2^{n.bit_length() - 1}" if n & (n - 1) == 0 else str(n)
    return Workload("late", [Box(pos, 1.0, K, sp / 40.0, 1.0 / n, seed)],
                    description=f"N={size}, K={K}, 50% in {n_halos} Plummer halos with scale radius "
                                "log-uniform in [0.05,0.5] cell, eps=spacing/40, G*m=1/N")


def batched_sizes(seed: int = 4, n_boxes: int = 64, lo: int = 64 ** 3, hi: int = 192 ** 3) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.round(np.exp(rng.random(n_boxes) * (math.log(hi) - math.log(lo)) + math.log(lo))).astype(np.int64)


def _batched(seed: int = 4, n_boxes: int = 64, lo: int = 64 ** 3, hi: int = 192 ** 3,
             per_cell: float = 48.0) -> Workload:
    sizes = batched_sizes(seed, n_boxes, lo, hi)
    boxes = []
    for b, nb in enumerate(sizes):
        nb = int(nb)
        K = max(5, int(round((nb / per_cell) ** (1.0 / 3.0))))
        nh = int(round(nb / 4096))
        pos = _clustered_box(4000 + b, nb, K, 0.3, nh, 0.3)
        boxes.append(Box(pos, 1.0, K, nb ** (-1.0 / 3.0) / 40.0, 1.0 / nb, 4000 + b))
    return Workload("batched", boxes,
                    description=f"{n_boxes} boxes, N_b log-uniform in [{lo},{hi}], K_b~(N_b/{per_cell})^(1/3), "
                                "30% in round(N_b/4096) Plummer halos (a=0.3 cell), eps_b=N_b^(-1/3)/40, G*m_b=1/N_b")


WORKLOADS: Dict[str, Callable[..., Workload]] = {
    "tiny": _tiny,
    "clustered": _clustered,
    "precision": _precision,
    "batched": _batched,
    "late": _late,
}


def workload(name: str, **kw) -> Workload:
    """Build a named workload: tiny, clustered, precision, batched, late.

    Keyword arguments override the recipe (seed, sizes) for scaled-down test cases.
    """
    return WORKLOADS[name](**kw)


def sample_sinks(n: int, m: int, seed: int = 99) -> np.ndarray:
    """m distinct sink indices out of n, uniform without replacement (sorted)."""
    if m >= n:
        return np.arange(n, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, size=m, replace=False)).astype(np.int64)


def taylor_coefficients(n_cells: int, p: int, seed: int = 7, amp: float = 1.0, r0: float = 3.0) -> np.ndarray:
    """[n_cells, (p+1)(p+2)(p+3)/6] float64: degree-n components drawn as amp * N(0,1) * r0^-n, components
    grouped by degree (lowest first; the order within a degree carries no meaning for the draw)."""
    rng = np.random.default_rng(seed)
    scale = np.concatenate([np.full((n + 1) * (n + 2) // 2, amp * r0 ** -n) for n in range(p + 1)])
    return rng.standard_normal((n_cells, scale.size)) * scale
