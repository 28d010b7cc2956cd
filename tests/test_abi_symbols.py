"""The C-ABI library loads without a GPU and exports every function the header
declares; the Python binding declares the same names."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mt_tersoff.h")
LIB = os.path.join(ROOT, "paper_1909_11474_amd", "libmt_tersoff.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(\w+)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_three_entry_points():
    names = declared_functions()
    for n in ("tersoff_eval", "fitness_eval", "fitness_grad", "tersoff_eval_tf", "fitness_eval_tf", "fitness_grad_tf",
              "mt_set_create",
              "mt_set_attach_reference", "mt_set_destroy", "mt_last_error", "mt_autotune"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for n in declared_functions():
        assert hasattr(lib, n), n
    lib.mt_version.restype = ctypes.c_char_p
    assert b"gfx950" in lib.mt_version()
    lib.mt_last_error.restype = ctypes.c_char_p
    assert lib.mt_last_error() is not None


def test_binding_declares_the_header_names():
    from paper_1909_11474_amd import _lib
    assert sorted(_lib.SIGNATURES) == declared_functions()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_argument_errors_without_gpu():
    """Argument checks happen before any device work, so they run here."""
    from paper_1909_11474_amd import _lib as L
    lib = L.load()
    h = ctypes.c_void_p()
    off = (ctypes.c_int64 * 2)(0, 8)
    # R2 <= R1
    assert lib.mt_set_create(ctypes.byref(h), 1, off, ctypes.c_void_p(1), ctypes.c_void_p(1),
                             3.2, 2.8, 16, None) == L.MT_EINVAL
    assert b"cutoff" in lib.mt_last_error()
    # capacity out of range
    assert lib.mt_set_create(ctypes.byref(h), 1, off, ctypes.c_void_p(1), ctypes.c_void_p(1),
                             2.8, 3.2, 99, None) == L.MT_EINVAL
    # empty structure
    off2 = (ctypes.c_int64 * 3)(0, 8, 8)
    assert lib.mt_set_create(ctypes.byref(h), 2, off2, ctypes.c_void_p(1), ctypes.c_void_p(1),
                             2.8, 3.2, 16, None) == L.MT_EINVAL
    assert lib.tersoff_eval(None, None, 1, 0, 0, None, None, None, None, None, None, None) == L.MT_EINVAL
    assert lib.tersoff_eval_tf(None, None, 1, 0, 0, None, None, None, None, None, None, None) == L.MT_EINVAL
    w = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    assert lib.fitness_eval_tf(None, None, 1, w, 0, 0, None, None) == L.MT_EINVAL
    assert lib.mt_set_destroy(None) == L.MT_OK
