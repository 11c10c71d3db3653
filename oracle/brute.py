"""Independent brute-force near field for tiny inputs (test infrastructure only).

Enumerates every ordered pair (i, j) and every periodic image shift
s in {-1, 0, 1}^3 and keeps the pair when the image's cell offset
cell(x_j) + s*K - cell(x_i) lies in [-R, R]^3 (Sec. 3.1: the near field is the
cells within R, each particle taken at the image in that cell).  With
K >= 2R+1 at most one image per axis qualifies.

The spline polynomial is not typed in here: its three coefficients are solved
from the matching conditions (value, slope and curvature of the Newtonian
force at r = eps), so this module does not share the oracle's constants.
"""
from __future__ import annotations

import numpy as np


def spline_coefficients(eps: float) -> np.ndarray:
    """Coefficients (a, b, c) of F(r) = a r + b r^2 + c r^3 with F, F', F'' equal to
    those of 1/r^2 at r = eps (F(r) = force magnitude for unit G*m)."""
    e = float(eps)
    A = np.array([[e, e ** 2, e ** 3],
                  [1.0, 2 * e, 3 * e ** 2],
                  [0.0, 2.0, 6 * e]])
    rhs = np.array([e ** -2, -2 * e ** -3, 6 * e ** -4])
    return np.linalg.solve(A, rhs)


def force_magnitude(r: np.ndarray, eps: float, kind: int) -> np.ndarray:
    """|F|(r) for unit G*m: spline (kind 0) or Plummer (kind 1)."""
    r = np.asarray(r, dtype=np.float64)
    if kind == 1:
        return r / (r * r + eps * eps) ** 1.5
    a, b, c = spline_coefficients(eps)
    inner = a * r + b * r ** 2 + c * r ** 3
    with np.errstate(divide="ignore"):
        outer = 1.0 / (r * r)
    return np.where(r >= eps, outer, inner)


def cells_numpy(pos32: np.ndarray, box: float, K: int) -> np.ndarray:
    """Per-axis cell indices [n,3] by floor of the wrapped coordinate times K/L, clamped to K-1."""
    x = pos32.astype(np.float64)
    xt = x - box * np.floor(x / box)
    c = np.floor(xt * (K / box)).astype(np.int64)
    return np.minimum(c, K - 1), xt


def brute_forces(pos32: np.ndarray, box: float, K: int, R: int, eps: float, kind: int, gm: float):
    """All-pairs x 27-image near-field accelerations [n,3] and the kept-pair count."""
    c, xt = cells_numpy(np.asarray(pos32, dtype=np.float32), box, K)
    n = xt.shape[0]
    acc = np.zeros((n, 3))
    kept = 0
    shifts = np.array([(a, b, d) for a in (-1, 0, 1) for b in (-1, 0, 1) for d in (-1, 0, 1)], dtype=np.int64)
    for i in range(n):
        for s in shifts:
            off = c + s * K - c[i]                       # cell offset of each image
            keep = np.all(np.abs(off) <= R, axis=1)
            if not keep.any():
                continue
            d = (xt[keep] + s * box) - xt[i]
            kept += int(keep.sum())
            r = np.sqrt((d * d).sum(axis=1))
            nz = r > 0
            if nz.any():
                f = force_magnitude(r[nz], eps, kind) / r[nz]
                acc[i] += (d[nz] * f[:, None]).sum(axis=0)
    return gm * acc, kept


def brute_density(pos32: np.ndarray, box: float, K: int, R: int, b: float) -> np.ndarray:
    """All-pairs x 27-image kernel density: sum of max(0, 1 - r^2/b^2) over the near field, self included."""
    c, xt = cells_numpy(np.asarray(pos32, dtype=np.float32), box, K)
    n = xt.shape[0]
    rho = np.zeros(n)
    shifts = np.array([(a, e, d) for a in (-1, 0, 1) for e in (-1, 0, 1) for d in (-1, 0, 1)], dtype=np.int64)
    for i in range(n):
        for s in shifts:
            keep = np.all(np.abs(c + s * K - c[i]) <= R, axis=1)
            if keep.any():
                d = (xt[keep] + s * box) - xt[i]
                w = 1.0 - (d * d).sum(axis=1) / (b * b)
                rho[i] += w[w > 0].sum()
    return rho
