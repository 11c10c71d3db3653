"""FP64 CPU oracle for the near-field force -- TEST INFRASTRUCTURE ONLY.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the HIP path.

* ``oracle_nf.c`` (built into ``liboracle_nf.so``): the cell-walk FP64 oracle
  written from Sec. 3.1 of the paper (near field = cells within R, explicit
  periodic images, direct sum), the spline and Plummer softening laws of
  Sec. 2.5 / Sec. 5.2, the cell rule, and an exact pair counter.
* the kernel density estimate fused into the same pass (Sec. 3.3), weight
  max(0, 1 - r^2/b^2) over the near field, self pair included (a reading).
* cell multipoles (Sec. 3.1, order p = 8): complete Cartesian moments about
  each cell centre, positions in cell widths (a reading of the basis).
* far field from per-cell Taylor series (Sec. 3.1): -grad of the series about
  each cell centre, co-added to a force array.
* ``kdk.py``: leapfrog kick / drift in the stored FP32 format, the cell
  timestep criterion, and kick-drift-kick steps over a force callable.
* ``brute.py``: an independent NumPy all-pairs x 27-image enumeration for tiny
  inputs, which keeps a pair exactly when its cell offset lies in [-R, R]^3.

Parity status: the spline's inner polynomial is not printed in the paper; it
is pinned to the reading (value, slope and curvature matching 1/r^2 at r=eps)
but "parity unpinned" against the original code.
"""
from .oracle import (lib_path, build, compile_oracle, Oracle, default, bin_cells, kernel_g,
                     forces, count_pairs, density, multipoles, multipole_exponents, taylor_forces, forces_boxes,
                     SOURCE,
                     SPLINE, PLUMMER)

__all__ = ["lib_path", "build", "compile_oracle", "Oracle", "default", "bin_cells", "kernel_g",
           "forces", "count_pairs", "density", "multipoles", "multipole_exponents", "taylor_forces",
           "forces_boxes", "SOURCE",
           "SPLINE", "PLUMMER"]
