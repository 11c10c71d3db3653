"""ctypes front end of the C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

SPLINE = 0
PLUMMER = 1

_HERE = os.path.dirname(os.path.abspath(__file__))
SOURCE = os.path.join(_HERE, "oracle_nf.c")
_LIB = os.path.join(_HERE, "liboracle_nf.so")


def lib_path() -> str:
    return _LIB


def compile_oracle(src: str, out: str) -> str:
    """gcc -O3 with OpenMP and IEEE FP64 (no fast-math, no FMA contraction)."""
    tmp = out + ".tmp"
    cmd = ["gcc", "-O3", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-o", tmp, src, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(SOURCE):
        compile_oracle(SOURCE, _LIB)
    return _LIB


def _pos32(pos) -> np.ndarray:
    p = np.ascontiguousarray(pos, dtype=np.float32)
    if p.ndim != 2 or p.shape[1] != 3:
        raise ValueError("positions must be [n, 3]")
    return p


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} failed with code {rc}")


class Oracle:
    """One loaded build of oracle_nf.c."""

    def __init__(self, path: str):
        lib = ctypes.CDLL(path)
        c_i64, c_d, vp, ci = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p, ctypes.c_int
        lib.oracle_nf_bin.argtypes = [vp, c_i64, c_d, ci, vp]
        lib.oracle_nf_kernel.argtypes = [vp, c_i64, c_d, ci, vp]
        lib.oracle_nf_forces.argtypes = [vp, c_i64, c_d, ci, ci, c_d, ci, c_d, vp, c_i64, ci, ci, vp, vp, vp]
        lib.oracle_nf_count_pairs.argtypes = [vp, c_i64, c_d, ci, ci, vp]
        lib.oracle_nf_density.argtypes = [vp, c_i64, c_d, ci, ci, c_d, vp, c_i64, ci, vp]
        lib.oracle_nf_multipoles.argtypes = [vp, c_i64, c_d, ci, ci, c_d, vp]
        lib.oracle_nf_taylor.argtypes = [vp, c_i64, c_d, ci, ci, vp, vp]
        for f in (lib.oracle_nf_bin, lib.oracle_nf_kernel, lib.oracle_nf_forces, lib.oracle_nf_count_pairs,
                  lib.oracle_nf_density, lib.oracle_nf_multipoles, lib.oracle_nf_taylor):
            f.restype = ctypes.c_int
        self.lib = lib
        self.path = path

    def bin_cells(self, pos, box: float, K: int) -> np.ndarray:
        """Linear cell index of every particle by the oracle's cell rule."""
        p = _pos32(pos)
        out = np.empty(p.shape[0], dtype=np.int32)
        _check(self.lib.oracle_nf_bin(p.ctypes.data, p.shape[0], float(box), int(K), out.ctypes.data), "bin")
        return out

    def kernel_g(self, r, eps: float, kind: int = SPLINE) -> np.ndarray:
        """The softened inverse cube g(r) (0 at r=0)."""
        r = np.ascontiguousarray(r, dtype=np.float64)
        out = np.empty_like(r)
        _check(self.lib.oracle_nf_kernel(r.ctypes.data, r.size, float(eps), int(kind), out.ctypes.data), "kernel")
        return out

    def forces(self, pos, box: float, K: int, R: int, eps: float, kind: int = SPLINE, gm: float = 1.0,
               sinks: Optional[np.ndarray] = None, neumaier: bool = False, threads: int = 0,
               return_pairs: bool = False, return_mag: bool = False):
        """FP64 near-field accelerations [m,3] of the sinks (all particles by default).

        With return_mag, also the per-sink sum of pair-term magnitudes (G*m * sum |d| g)."""
        p = _pos32(pos)
        n = p.shape[0]
        if sinks is None:
            m, sp = n, None
        else:
            sk = np.ascontiguousarray(sinks, dtype=np.int64)
            m, sp = sk.size, sk.ctypes.data
        acc = np.zeros((m, 3), dtype=np.float64)
        mag = np.zeros(m, dtype=np.float64) if return_mag else None
        pairs = ctypes.c_int64(0)
        rc = self.lib.oracle_nf_forces(p.ctypes.data if n else None, n, float(box), int(K), int(R), float(eps),
                                       int(kind), float(gm), sp, m, int(bool(neumaier)), int(threads),
                                       acc.ctypes.data if m else None,
                                       mag.ctypes.data if (return_mag and m) else None, ctypes.byref(pairs))
        _check(rc, "forces")
        out = [acc]
        if return_pairs:
            out.append(int(pairs.value))
        if return_mag:
            out.append(mag)
        return out[0] if len(out) == 1 else tuple(out)

    def density(self, pos, box: float, K: int, R: int, b: float, sinks: Optional[np.ndarray] = None,
                threads: int = 0) -> np.ndarray:
        """Near-field kernel density sum max(0, 1 - r^2/b^2), self pair included (FP64)."""
        p = _pos32(pos)
        n = p.shape[0]
        if sinks is None:
            m, sp = n, None
        else:
            sk = np.ascontiguousarray(sinks, dtype=np.int64)
            m, sp = sk.size, sk.ctypes.data
        rho = np.zeros(m, dtype=np.float64)
        _check(self.lib.oracle_nf_density(p.ctypes.data if n else None, n, float(box), int(K), int(R), float(b),
                                          sp, m, int(threads), rho.ctypes.data if m else None), "density")
        return rho

    def multipoles(self, pos, box: float, K: int, p: int = 8, m: float = 1.0) -> np.ndarray:
        """Complete Cartesian moments about each cell centre in cell widths, [K^3, (p+1)(p+2)(p+3)/6] FP64."""
        q = _pos32(pos)
        ncomp = (p + 1) * (p + 2) * (p + 3) // 6
        out = np.zeros((K ** 3, ncomp), dtype=np.float64)
        _check(self.lib.oracle_nf_multipoles(q.ctypes.data if q.shape[0] else None, q.shape[0], float(box), int(K),
                                             int(p), float(m), out.ctypes.data), "multipoles")
        return out

    def taylor_forces(self, pos, box: float, K: int, p: int, taylor, acc=None) -> np.ndarray:
        """acc + far-field acceleration -grad Phi of the cell Taylor series (FP64 [n, 3])."""
        q = _pos32(pos)
        n = q.shape[0]
        T = np.ascontiguousarray(taylor, dtype=np.float64)
        out = np.zeros((n, 3)) if acc is None else np.array(acc, dtype=np.float64, copy=True)
        _check(self.lib.oracle_nf_taylor(q.ctypes.data if n else None, n, float(box), int(K), int(p), T.ctypes.data,
                                         out.ctypes.data if n else None), "taylor")
        return out

    def count_pairs(self, pos, box: float, K: int, R: int = 2) -> int:
        """Exact number of (sink, source) pairs, self pairs included, from cell occupancy."""
        p = _pos32(pos)
        out = ctypes.c_int64(0)
        _check(self.lib.oracle_nf_count_pairs(p.ctypes.data if p.shape[0] else None, p.shape[0], float(box),
                                              int(K), int(R), ctypes.byref(out)), "count_pairs")
        return int(out.value)


_default: Optional[Oracle] = None


def default() -> Oracle:
    global _default
    if _default is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _default = Oracle(_LIB)
    return _default


def bin_cells(pos, box, K):
    return default().bin_cells(pos, box, K)


def kernel_g(r, eps, kind=SPLINE):
    return default().kernel_g(r, eps, kind)


def forces(pos, box, K, R, eps, kind=SPLINE, gm=1.0, sinks=None, neumaier=False, threads=0, return_pairs=False,
           return_mag=False):
    return default().forces(pos, box, K, R, eps, kind, gm, sinks, neumaier, threads, return_pairs, return_mag)


def count_pairs(pos, box, K, R=2):
    return default().count_pairs(pos, box, K, R)


def density(pos, box, K, R, b, sinks=None, threads=0):
    return default().density(pos, box, K, R, b, sinks, threads)


def multipoles(pos, box, K, p=8, m=1.0):
    return default().multipoles(pos, box, K, p, m)


def taylor_forces(pos, box, K, p, taylor, acc=None):
    return default().taylor_forces(pos, box, K, p, taylor, acc)


def multipole_exponents(p: int):
    """(a, b, k) of each component, in the order used by the multipole arrays."""
    return [(a, b, n - a - b) for n in range(p + 1) for a in range(n, -1, -1) for b in range(n - a, -1, -1)]


def forces_boxes(boxes: Sequence, R: int = 2, kind: int = SPLINE, threads: int = 0) -> np.ndarray:
    """Concatenated accelerations for a list of independent boxes (workloads.Box)."""
    out = [forces(b.pos, b.box, b.K, R, b.eps, kind, b.gm, threads=threads) for b in boxes]
    return np.concatenate(out, axis=0) if out else np.zeros((0, 3))
