"""MI355X-native near-field force of the Abacus N-body method (arXiv:2110.11398).

The compute path is the HIP library ``libabacus_nf.so`` (hand-written gfx950
kernels behind a C ABI, ``include/abacus_nf.h``).  This package is its thin
Python binding: it marshals torch device pointers and streams into the C
calls and does none of the method's arithmetic.  Importing works without a
GPU; every call that computes needs the built library and a GPU and raises
otherwise.
"""
from .abacus_nf import (SPLINE, PLUMMER, SUM_FP32, SUM_COMP32, SUM_FP64, ARRAY_PERM, ARRAY_CELL_START, ARRAY_SPOS,
                        ARRAY_CELL_KEY, ARRAY_CELL_AMAX2, NearFieldError, Cells, Tuning, build_cells, forces, sync, near_field,
                        library, library_path, strerror, version)

__all__ = ["SPLINE", "PLUMMER", "SUM_FP32", "SUM_COMP32", "SUM_FP64", "ARRAY_PERM", "ARRAY_CELL_START", "ARRAY_SPOS",
           "ARRAY_CELL_KEY", "ARRAY_CELL_AMAX2", "NearFieldError", "Cells", "Tuning", "build_cells", "forces", "sync", "near_field",
           "library", "library_path", "strerror", "version"]
