"""CPU-side checks of the C ABI: libarb.so loads and exports every function include/arb.h
declares (no compute calls: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SO = os.path.join(ROOT, "paper_2002_10047_amd", "libarb.so")
HDR = os.path.join(ROOT, "include", "arb.h")


def declared():
    src = re.sub(r"/\*.*?\*/", "", open(HDR).read(), flags=re.S)
    return sorted(set(re.findall(r"\b(arb_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_core_entry_points():
    names = declared()
    for core in ["arb_orient", "arb_count", "arb_count_async", "arb_permute_u64", "arb_features",
                 "arb_mlp_forward", "arb_mlp_backward", "arb_adam_step", "arb_last_error"]:
        assert core in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(SO):
        from paper_2002_10047_amd import build
        build.build()
    lib = ctypes.CDLL(SO)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_error_strings_and_workspace_sizes():
    lib = ctypes.CDLL(SO)
    lib.arb_error_string.restype = ctypes.c_char_p
    assert lib.arb_error_string(0) == b"ok"
    assert lib.arb_error_string(3) == b"workspace too small"
    lib.arb_orient_workspace.restype = ctypes.c_size_t
    lib.arb_orient_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64]
    lib.arb_count_workspace.restype = ctypes.c_size_t
    lib.arb_count_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
    a = lib.arb_orient_workspace(1000, 10000)
    b = lib.arb_orient_workspace(100000, 10000)
    assert 0 < a < b
    assert lib.arb_count_workspace(1000, 5000, 4) > 1000 * 8


def test_invalid_arguments_rejected_without_device():
    # null graph pointers fail argument checks before any HIP call
    lib = ctypes.CDLL(SO)
    lib.arb_orient.restype = ctypes.c_int
    lib.arb_orient.argtypes = [ctypes.c_void_p, ctypes.c_double, ctypes.c_int] + [ctypes.c_void_p] * 6 + \
        [ctypes.c_size_t, ctypes.c_void_p]
    assert lib.arb_orient(None, 1.0, 0, None, None, None, None, None, None, 0, None) == 1
    lib.arb_last_error.restype = ctypes.c_int
    assert lib.arb_last_error() == 1


def test_binding_wraps_every_declared_function():
    src = open(os.path.join(ROOT, "paper_2002_10047_amd", "arb.py")).read()
    missing = [n for n in declared() if f"def {n}(" not in src]
    assert not missing, missing
