"""ctypes binding of libabacus_nf (argument marshalling only).

Names follow the C ABI: ``build_cells``, ``forces``, ``sync``.  Positions and
accelerations are torch tensors on the current HIP device; the stream is
torch's current stream unless one is given.  All arithmetic happens in the
library's kernels; if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes
import os
from typing import Iterable, List, Optional, Sequence, Tuple

HERE = os.path.dirname(os.path.abspath(__file__))
# ABACUS_NF_LIBRARY selects another build of the same library (for comparing builds)
_LIB_PATH = os.environ.get("ABACUS_NF_LIBRARY") or os.path.join(HERE, "libabacus_nf.so")

SPLINE, PLUMMER = 0, 1
SUM_FP32, SUM_COMP32, SUM_FP64 = 0, 1, 2
ARRAY_PERM, ARRAY_CELL_START, ARRAY_SPOS, ARRAY_CELL_KEY, ARRAY_CELL_AMAX2 = 0, 1, 2, 3, 4

OK, EINVAL, ENOMEM, EDEVICE, ECAPACITY, ENONFINITE, ESTATE, ELIMIT = 0, -1, -2, -3, -4, -5, -6, -7


class BoxDesc(ctypes.Structure):
    _fields_ = [("offset", ctypes.c_int64), ("n", ctypes.c_int64), ("box", ctypes.c_double),
                ("K", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    """Mirror of abacus_nf_tuning (zero fields mean library default)."""
    _fields_ = [("sinks_per_lane", ctypes.c_int32), ("chunk", ctypes.c_int32), ("unroll", ctypes.c_int32),
                ("max_lanes", ctypes.c_int32), ("part_sources", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("occupancy", ctypes.c_int32), ("reserved", ctypes.c_int32), ("item_capacity", ctypes.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class NearFieldError(RuntimeError):
    def __init__(self, code: int, what: str = ""):
        self.code = code
        super().__init__(f"{what}: {strerror(code)} ({code})" if what else f"{strerror(code)} ({code})")


_lib = None


def library_path() -> str:
    return _LIB_PATH


def library():
    """Load libabacus_nf.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(the near-field path has no fallback)")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    sig = {
        "abacus_nf_build_cells": [vp, i64, ctypes.POINTER(BoxDesc), i32, i32, vp, ctypes.POINTER(vp)],
        "abacus_nf_forces": [vp, ctypes.POINTER(d), ctypes.c_int, ctypes.POINTER(d), ctypes.c_int, vp, vp],
        "abacus_nf_forces_density": [vp, ctypes.POINTER(d), ctypes.c_int, ctypes.POINTER(d), ctypes.c_int,
                                     ctypes.POINTER(d), vp, vp, vp],
        "abacus_nf_forces_f64": [vp, ctypes.POINTER(d), ctypes.c_int, ctypes.POINTER(d), ctypes.c_int, vp, vp],
        "abacus_nf_multipoles": [vp, i32, ctypes.POINTER(d), vp, vp],
        "abacus_nf_taylor_forces": [vp, i32, vp, vp, vp],
        "abacus_nf_kick": [vp, ctypes.POINTER(d), vp, vp, vp],
        "abacus_nf_reorder": [vp, ctypes.POINTER(vp), i32, vp, vp],
        "abacus_nf_drift": [vp, ctypes.POINTER(d), vp, vp, vp],
        "abacus_nf_timestep": [vp, vp, vp, d, ctypes.POINTER(d), vp],
        "abacus_nf_timestep_noalloc": [vp, vp, vp, d, ctypes.POINTER(d), vp],
        "abacus_nf_kdk_step": [vp, ctypes.POINTER(d), ctypes.POINTER(d), ctypes.c_int, ctypes.POINTER(d),
                               ctypes.c_int, vp, vp, vp, vp],
        "abacus_nf_sync": [vp],
        "abacus_nf_free_cells": [vp],
        "abacus_nf_interactions": [vp, vp, ctypes.POINTER(i64)],
        "abacus_nf_cells_size": [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)],
        "abacus_nf_copy_cells": [vp, ctypes.c_int, vp, i64, vp],
        "abacus_nf_set_tuning": [vp, ctypes.POINTER(Tuning)],
        "abacus_nf_get_tuning": [vp, ctypes.POINTER(Tuning)],
        "abacus_nf_autotune": [vp, ctypes.POINTER(d), ctypes.c_int, ctypes.POINTER(d), ctypes.c_int, vp, vp, i32,
                               ctypes.c_char_p, ctypes.POINTER(Tuning)],
        "abacus_nf_autotune_density": [vp, ctypes.POINTER(d), ctypes.c_int, ctypes.POINTER(d), ctypes.c_int,
                                       ctypes.POINTER(d), vp, vp, vp, i32, ctypes.c_char_p, ctypes.POINTER(Tuning)],
        "abacus_nf_set_timing": [vp, i32],
        "abacus_nf_last_times": [vp, ctypes.POINTER(ctypes.c_float)],
        "abacus_nf_version": [],
    }
    for name, args in sig.items():
        if not hasattr(lib, name):   # an older build of the library (see ABACUS_NF_LIBRARY)
            continue
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = ctypes.c_int
    lib.abacus_nf_strerror.argtypes = [ctypes.c_int]
    lib.abacus_nf_strerror.restype = ctypes.c_char_p
    _lib = lib
    return lib


def strerror(code: int) -> str:
    try:
        return library().abacus_nf_strerror(int(code)).decode()
    except RuntimeError:
        return f"error {code}"


def version() -> int:
    return library().abacus_nf_version()


def _check(rc: int, what: str):
    if rc != OK:
        raise NearFieldError(rc, what)


def _stream_handle(stream) -> Optional[int]:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else (int(stream) if stream else None)


def _doubles(vals: Sequence[float]):
    arr = (ctypes.c_double * len(vals))(*[float(v) for v in vals])
    return arr


class Cells:
    """A built cell structure (handle of abacus_nf_build_cells)."""

    def __init__(self):
        self._h = ctypes.c_void_p(None)
        self.boxes: List[Tuple[int, float, int]] = []
        self.n_total = 0

    # -- C ABI wrappers
    def build(self, pos, boxes: Iterable[Tuple[int, float, int]], R: int = 2, stream=None) -> "Cells":
        """abacus_nf_build_cells on pos (float32 [N,3] device tensor); boxes = [(n, L, K), ...] in order."""
        import torch
        if not (isinstance(pos, torch.Tensor) and pos.is_cuda and pos.dtype == torch.float32 and pos.dim() == 2
                and pos.shape[1] == 3 and pos.is_contiguous()):
            raise ValueError("pos must be a contiguous float32 [N,3] tensor on the GPU")
        boxes = [(int(n), float(L), int(K)) for n, L, K in boxes]
        desc = (BoxDesc * len(boxes))()
        off = 0
        for i, (n, L, K) in enumerate(boxes):
            desc[i].offset, desc[i].n, desc[i].box, desc[i].K, desc[i].reserved = off, n, L, K, 0
            off += n
        rc = library().abacus_nf_build_cells(ctypes.c_void_p(pos.data_ptr() if pos.numel() else None),
                                             int(pos.shape[0]), desc, len(boxes), int(R),
                                             ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(self._h))
        _check(rc, "abacus_nf_build_cells")
        self.boxes = boxes
        self.n_total = int(pos.shape[0])
        self._pos_ref = pos  # keep the input alive until the enqueued work has read it
        return self

    def forces(self, eps: Sequence[float], gm: Sequence[float], kind: int = SPLINE, mode: int = SUM_COMP32,
               out=None, stream=None):
        """abacus_nf_forces into out (float32 [N,3] device tensor, allocated if None)."""
        import torch
        if out is None:
            out = torch.empty((self.n_total, 3), dtype=torch.float32, device="cuda")
        if not (out.is_cuda and out.dtype == torch.float32 and out.shape == (self.n_total, 3) and out.is_contiguous()):
            raise ValueError("out must be a contiguous float32 [N,3] GPU tensor")
        rc = library().abacus_nf_forces(self._h, _doubles(eps), int(kind), _doubles(gm), int(mode),
                                        ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                        ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_forces")
        return out

    def forces_f64(self, eps: Sequence[float], gm: Sequence[float], kind: int = SPLINE, mode: int = SUM_COMP32,
                   out=None, stream=None):
        """abacus_nf_forces_f64 into out (float64 [N,3] device tensor, allocated if None)."""
        import torch
        if out is None:
            out = torch.empty((self.n_total, 3), dtype=torch.float64, device="cuda")
        if not (out.is_cuda and out.dtype == torch.float64 and out.shape == (self.n_total, 3) and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 [N,3] GPU tensor")
        rc = library().abacus_nf_forces_f64(self._h, _doubles(eps), int(kind), _doubles(gm), int(mode),
                                            ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                            ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_forces_f64")
        return out

    def forces_density(self, eps: Sequence[float], gm: Sequence[float], b: Sequence[float], kind: int = SPLINE,
                       mode: int = SUM_COMP32, out=None, rho=None, stream=None):
        """abacus_nf_forces_density: accelerations [N,3] and kernel densities [N] (device tensors)."""
        import torch
        if out is None:
            out = torch.empty((self.n_total, 3), dtype=torch.float32, device="cuda")
        if rho is None:
            rho = torch.empty(self.n_total, dtype=torch.float32, device="cuda")
        if not (out.is_cuda and out.dtype == torch.float32 and out.shape == (self.n_total, 3) and out.is_contiguous()):
            raise ValueError("out must be a contiguous float32 [N,3] GPU tensor")
        if not (rho.is_cuda and rho.dtype == torch.float32 and rho.shape == (self.n_total,) and rho.is_contiguous()):
            raise ValueError("rho must be a contiguous float32 [N] GPU tensor")
        rc = library().abacus_nf_forces_density(self._h, _doubles(eps), int(kind), _doubles(gm), int(mode),
                                                _doubles(b), ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                                ctypes.c_void_p(rho.data_ptr() if rho.numel() else None),
                                                ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_forces_density")
        return out, rho

    def multipoles(self, order: int = 8, mass: Optional[Sequence[float]] = None, out=None, stream=None):
        """abacus_nf_multipoles: [n_cells, (order+1)(order+2)(order+3)/6] float64 device tensor."""
        import torch
        n, nc = self.size()
        ncomp = (order + 1) * (order + 2) * (order + 3) // 6
        if mass is None:
            mass = [1.0] * len(self.boxes)
        if out is None:
            out = torch.empty((nc, ncomp), dtype=torch.float64, device="cuda")
        if not (out.is_cuda and out.dtype == torch.float64 and out.shape == (nc, ncomp) and out.is_contiguous()):
            raise ValueError("out must be a contiguous float64 [n_cells, components] GPU tensor")
        rc = library().abacus_nf_multipoles(self._h, int(order), _doubles(mass),
                                            ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                            ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_multipoles")
        return out

    def taylor_forces(self, order: int, taylor, acc, stream=None):
        """abacus_nf_taylor_forces: acc (float32 [N,3] device) += far field of the cell Taylor series
        taylor (float64 [n_cells, components] device)."""
        import torch
        n, nc = self.size()
        ncomp = (order + 1) * (order + 2) * (order + 3) // 6
        if not (taylor.is_cuda and taylor.dtype == torch.float64 and taylor.shape == (nc, ncomp)
                and taylor.is_contiguous()):
            raise ValueError("taylor must be a contiguous float64 [n_cells, components] GPU tensor")
        if not (acc.is_cuda and acc.dtype == torch.float32 and acc.shape == (n, 3) and acc.is_contiguous()):
            raise ValueError("acc must be a contiguous float32 [N,3] GPU tensor")
        rc = library().abacus_nf_taylor_forces(self._h, int(order), ctypes.c_void_p(taylor.data_ptr() or None),
                                               ctypes.c_void_p(acc.data_ptr() or None),
                                               ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_taylor_forces")
        return acc

    def _vec3(self, t, what):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == torch.float32
                and t.shape == (self.n_total, 3) and t.is_contiguous()):
            raise ValueError(f"{what} must be a contiguous float32 [N,3] GPU tensor")
        return ctypes.c_void_p(t.data_ptr() if t.numel() else None)

    def kick(self, dt: Sequence[float], acc, vel, stream=None):
        """abacus_nf_kick: vel += acc * dt (per box), in place."""
        rc = library().abacus_nf_kick(self._h, _doubles(dt), self._vec3(acc, "acc"), self._vec3(vel, "vel"),
                                      ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_kick")
        return vel

    def drift(self, dt: Sequence[float], vel, pos, stream=None):
        """abacus_nf_drift: pos += vel * dt wrapped into each box, in place (the cells must be built again)."""
        rc = library().abacus_nf_drift(self._h, _doubles(dt), self._vec3(vel, "vel"), self._vec3(pos, "pos"),
                                       ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_drift")
        return pos

    def timestep(self, vel, acc=None, eta: float = 0.25, stream=None) -> List[float]:
        """abacus_nf_timestep: eta * min over cells of sigma_v / max|a|, per box (blocks on the stream).
        With acc=None the per-cell maxima of |a| come from the last forces call on this handle."""
        out = (ctypes.c_double * len(self.boxes))()
        a = self._vec3(acc, "acc") if acc is not None else ctypes.c_void_p(None)
        rc = library().abacus_nf_timestep(self._h, self._vec3(vel, "vel"), a, float(eta), out,
                                          ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_timestep")
        return list(out)

    def timestep_noalloc(self, vel, acc=None, eta: float = 0.25, stream=None) -> List[float]:
        """abacus_nf_timestep_noalloc: the same criterion with the library's fixed scratch (no allocation)."""
        out = (ctypes.c_double * len(self.boxes))()
        a = self._vec3(acc, "acc") if acc is not None else ctypes.c_void_p(None)
        rc = library().abacus_nf_timestep_noalloc(self._h, self._vec3(vel, "vel"), a, float(eta), out,
                                                  ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_timestep_noalloc")
        return list(out)

    def reorder(self, arrays, ids=None, stream=None):
        """abacus_nf_reorder: gather the [N,3] float32 arrays (positions included) and optional int64 ids
        into the cell order of the last build, in place."""
        import torch
        ptrs = (ctypes.c_void_p * max(1, len(arrays)))(*[self._vec3(t, "array").value for t in arrays])
        if ids is not None and not (ids.is_cuda and ids.dtype == torch.int64 and ids.shape == (self.n_total,)
                                    and ids.is_contiguous()):
            raise ValueError("ids must be a contiguous int64 [N] GPU tensor")
        rc = library().abacus_nf_reorder(self._h, ptrs, len(arrays),
                                         ctypes.c_void_p(ids.data_ptr() if ids is not None and ids.numel() else None),
                                         ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_reorder")
        return arrays

    def kdk_step(self, dt: Sequence[float], eps: Sequence[float], gm: Sequence[float], pos, vel, acc,
                 kind: int = SPLINE, mode: int = SUM_COMP32, stream=None):
        """abacus_nf_kdk_step: one leapfrog step (half kick, drift, rebuild, forces, half kick), in place.
        acc must hold the accelerations at the current positions."""
        rc = library().abacus_nf_kdk_step(self._h, _doubles(dt), _doubles(eps), int(kind), _doubles(gm), int(mode),
                                          self._vec3(pos, "pos"), self._vec3(vel, "vel"), self._vec3(acc, "acc"),
                                          ctypes.c_void_p(_stream_handle(stream)))
        _check(rc, "abacus_nf_kdk_step")
        self._pos_ref = pos
        return pos, vel, acc

    def interactions(self, stream=None) -> int:
        v = ctypes.c_int64(0)
        _check(library().abacus_nf_interactions(self._h, ctypes.c_void_p(_stream_handle(stream)), ctypes.byref(v)),
               "abacus_nf_interactions")
        return int(v.value)

    def size(self) -> Tuple[int, int]:
        n, c = ctypes.c_int64(0), ctypes.c_int64(0)
        _check(library().abacus_nf_cells_size(self._h, ctypes.byref(n), ctypes.byref(c)), "abacus_nf_cells_size")
        return int(n.value), int(c.value)

    def copy(self, which: int, stream=None):
        """Copy one internal array (ARRAY_*) into a new device tensor."""
        import torch
        n, nc = self.size()
        if which == ARRAY_SPOS:
            t = torch.empty((n, 4), dtype=torch.float32, device="cuda")
        elif which == ARRAY_CELL_AMAX2:
            t = torch.empty(nc, dtype=torch.float64, device="cuda")
        elif which == ARRAY_CELL_START:
            t = torch.empty(nc + 1, dtype=torch.int32, device="cuda")
        else:
            t = torch.empty(n, dtype=torch.int32, device="cuda")
        nbytes = t.numel() * t.element_size()
        _check(library().abacus_nf_copy_cells(self._h, int(which), ctypes.c_void_p(t.data_ptr() if nbytes else 1),
                                              nbytes, ctypes.c_void_p(_stream_handle(stream))), "abacus_nf_copy_cells")
        return t

    def set_tuning(self, **kw):
        t = self.get_tuning() if kw else Tuning()
        for k, v in kw.items():
            setattr(t, k, int(v))
        _check(library().abacus_nf_set_tuning(self._h, ctypes.byref(t)), "abacus_nf_set_tuning")

    def reset_tuning(self):
        _check(library().abacus_nf_set_tuning(self._h, None), "abacus_nf_set_tuning")

    def get_tuning(self) -> Tuning:
        t = Tuning()
        _check(library().abacus_nf_get_tuning(self._h, ctypes.byref(t)), "abacus_nf_get_tuning")
        return t

    def autotune(self, eps, gm, kind=SPLINE, mode=SUM_COMP32, out=None, reps: int = 2,
                 cache_path: Optional[str] = None, stream=None) -> Tuning:
        import torch
        if out is None:
            out = torch.empty((self.n_total, 3), dtype=torch.float32, device="cuda")
        t = Tuning()
        rc = library().abacus_nf_autotune(self._h, _doubles(eps), int(kind), _doubles(gm), int(mode),
                                          ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                          ctypes.c_void_p(_stream_handle(stream)), int(reps),
                                          cache_path.encode() if cache_path else None, ctypes.byref(t))
        _check(rc, "abacus_nf_autotune")
        return t

    def autotune_density(self, eps, gm, b, kind=SPLINE, mode=SUM_COMP32, out=None, rho=None, reps: int = 2,
                         cache_path: Optional[str] = None, stream=None) -> Tuning:
        """abacus_nf_autotune_density: tune the force pass with the fused density estimate."""
        import torch
        if out is None:
            out = torch.empty((self.n_total, 3), dtype=torch.float32, device="cuda")
        if rho is None:
            rho = torch.empty(self.n_total, dtype=torch.float32, device="cuda")
        t = Tuning()
        rc = library().abacus_nf_autotune_density(self._h, _doubles(eps), int(kind), _doubles(gm), int(mode),
                                                  _doubles(b), ctypes.c_void_p(out.data_ptr() if out.numel() else None),
                                                  ctypes.c_void_p(rho.data_ptr() if rho.numel() else None),
                                                  ctypes.c_void_p(_stream_handle(stream)), int(reps),
                                                  cache_path.encode() if cache_path else None, ctypes.byref(t))
        _check(rc, "abacus_nf_autotune_density")
        return t

    def set_timing(self, on: bool = True):
        _check(library().abacus_nf_set_timing(self._h, int(bool(on))), "abacus_nf_set_timing")

    def last_times(self):
        """[build_cells, work list, force kernel, finalize] milliseconds of the last timed calls (-1 = not run)."""
        ms = (ctypes.c_float * 4)()
        _check(library().abacus_nf_last_times(self._h, ms), "abacus_nf_last_times")
        return [float(x) for x in ms]

    def free(self):
        if self._h.value:
            library().abacus_nf_free_cells(self._h)
            self._h = ctypes.c_void_p(None)

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def build_cells(pos, boxes, R: int = 2, cells: Optional[Cells] = None, stream=None) -> Cells:
    """abacus_nf_build_cells: sort particles into cells (reuses `cells` if given)."""
    return (cells or Cells()).build(pos, boxes, R, stream)


def forces(cells: Cells, eps, kind=SPLINE, gm=None, mode=SUM_COMP32, acc=None, stream=None):
    """abacus_nf_forces: near-field accelerations in input order."""
    return cells.forces(eps, gm, kind, mode, acc, stream)


def sync(stream=None):
    """abacus_nf_sync: wait for the stream and raise the first deferred device error."""
    _check(library().abacus_nf_sync(ctypes.c_void_p(_stream_handle(stream))), "abacus_nf_sync")


def near_field(pos, box: float, K: int, eps: float, gm: float, kind: int = SPLINE, mode: int = SUM_COMP32,
               R: int = 2, stream=None):
    """One periodic box: build the cells, compute the accelerations, synchronize."""
    c = build_cells(pos, [(pos.shape[0], box, K)], R, stream=stream)
    out = c.forces([eps], [gm], kind, mode, stream=stream)
    sync(stream)
    c.free()
    return out
