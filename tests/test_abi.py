"""The C-ABI library builds, loads and exports every declared symbol, and
rejects bad arguments synchronously, before touching a device (CPU only)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "abacus_nf.h")


@pytest.fixture(scope="module")
def lib():
    import paper_2110_11398_amd as nf
    if not os.path.exists(nf.library_path()):
        from paper_2110_11398_amd import build
        build.build()
    return nf.library()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(abacus_nf_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("abacus_nf_build_cells", "abacus_nf_forces", "abacus_nf_sync"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert missing == []


def test_strerror_and_version(lib):
    import paper_2110_11398_amd as nf
    assert nf.version() >= 10000
    for code in (0, -1, -2, -3, -4, -5, -6, -7):
        assert nf.strerror(code) and "unknown" not in nf.strerror(code)
    assert "unknown" in nf.strerror(-99)


def _boxes(*specs):
    from paper_2110_11398_amd.abacus_nf import BoxDesc
    arr = (BoxDesc * len(specs))()
    for i, (off, n, L, K) in enumerate(specs):
        arr[i].offset, arr[i].n, arr[i].box, arr[i].K, arr[i].reserved = off, n, L, K, 0
    return arr


@pytest.mark.parametrize("case", [
    "null_handle_ptr", "null_boxes", "negative_n", "no_boxes", "R_zero", "R_four", "K_too_small",
    "offset_gap", "sizes_mismatch", "box_nonpositive", "box_nan", "null_pos", "reserved_set", "too_many_cells",
])
def test_build_cells_rejects_bad_arguments(lib, case):
    h = ctypes.c_void_p(None)
    pos = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    args = dict(pos=pos, n=10, boxes=_boxes((0, 10, 1.0, 8)), nb=1, R=2, out=ctypes.byref(h))
    if case == "null_handle_ptr":
        args["out"] = None
    elif case == "null_boxes":
        args["boxes"] = None
    elif case == "negative_n":
        args["n"] = -1
    elif case == "no_boxes":
        args["nb"] = 0
    elif case == "R_zero":
        args["R"] = 0
    elif case == "R_four":
        args["R"] = 4
        args["boxes"] = _boxes((0, 10, 1.0, 12))
    elif case == "K_too_small":
        args["boxes"] = _boxes((0, 10, 1.0, 4))
    elif case == "offset_gap":
        args["boxes"] = _boxes((0, 5, 1.0, 8), (6, 4, 1.0, 8))
        args["nb"] = 2
    elif case == "sizes_mismatch":
        args["boxes"] = _boxes((0, 9, 1.0, 8))
    elif case == "box_nonpositive":
        args["boxes"] = _boxes((0, 10, 0.0, 8))
    elif case == "box_nan":
        args["boxes"] = _boxes((0, 10, float("nan"), 8))
    elif case == "null_pos":
        args["pos"] = None
    elif case == "reserved_set":
        b = _boxes((0, 10, 1.0, 8))
        b[0].reserved = 1
        args["boxes"] = b
    elif case == "too_many_cells":
        args["boxes"] = _boxes((0, 10, 1.0, 1291))
    rc = lib.abacus_nf_build_cells(args["pos"], args["n"], args["boxes"], args["nb"], args["R"], None, args["out"])
    assert rc == -1
    assert h.value is None


def test_other_entry_points_reject_null_handles(lib):
    d = (ctypes.c_double * 1)(0.01)
    assert lib.abacus_nf_forces(None, d, 0, d, 0, None, None) == -1
    assert lib.abacus_nf_free_cells(None) == 0
    v = ctypes.c_int64()
    assert lib.abacus_nf_interactions(None, None, ctypes.byref(v)) == -1
    assert lib.abacus_nf_cells_size(None, ctypes.byref(v), ctypes.byref(v)) == -1
    assert lib.abacus_nf_copy_cells(None, 0, ctypes.c_void_p(1), 4, None) == -1
    assert lib.abacus_nf_set_tuning(None, None) == -1
    assert lib.abacus_nf_set_timing(None, 1) == -1
    assert lib.abacus_nf_autotune(None, d, 0, d, 0, None, None, 1, None, None) == -1


def test_product_path_has_no_fallback(tmp_path, monkeypatch):
    """Without the built library the binding raises instead of computing anything."""
    import paper_2110_11398_amd.abacus_nf as b
    monkeypatch.setattr(b, "_LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(b, "_lib", None)
    with pytest.raises(RuntimeError):
        b.library()


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2110_11398_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text and "oracle_nf" not in text, f
