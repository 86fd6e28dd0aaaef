"""Host-side checks of the C-ABI library (no GPU needed).

The library loads, exports every symbol include/libsketch.h declares, and
rejects invalid arguments before touching a device.
"""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2508_21189_amd", "lib", "libsketch.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libsketch.so not built")


def header_functions():
    src = open(os.path.join(ROOT, "include", "libsketch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sketch_\w+|lstsq_\w+|rsvd\w*)\s*\(", src)))


def test_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    names = header_functions()
    assert "sketch_apply" in names and "sketch_create" in names
    for name in names:
        assert hasattr(lib, name), name


def test_binding_lists_header_symbols():
    from paper_2508_21189_amd import libsketch
    assert set(header_functions()) <= set(libsketch.exported_symbols())


@pytest.mark.parametrize("kind,d,n,zeta", [(0, 10, 100, 3), (0, 8, 100, 0), (0, 8, 100, 9), (0, 0, 10, 1),
                                           (2, 33, 30, 1), (99, 5, 6, 1), (7, 4, 4, 1)])
def test_create_rejects_invalid_parameters(kind, d, n, zeta):
    lib = ctypes.CDLL(LIB)
    lib.sketch_create.restype = ctypes.c_void_p
    lib.sketch_create.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.c_int64, ctypes.c_int, ctypes.c_uint64]
    lib.sketch_last_error.restype = ctypes.c_char_p
    assert not lib.sketch_create(kind, d, n, zeta, 1)
    assert lib.sketch_last_error()


def test_null_handle_calls_fail_cleanly():
    lib = ctypes.CDLL(LIB)
    lib.sketch_apply.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_int64, ctypes.c_int, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                 ctypes.c_size_t, ctypes.c_void_p]
    assert lib.sketch_apply(None, 0, 0, 4, None, 4, 0, None, 4, None, 0, None) == -1
    assert lib.sketch_destroy(None) == 0
