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


def _header_struct_fields(name):
    src = open(os.path.join(ROOT, "include", "libsketch.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    body = re.search(r"typedef struct\s*\{([^}]*)\}\s*%s\s*;" % name, src).group(1)
    return [(t.strip(), f.strip()) for t, f in re.findall(r"(int|double)\s+(\w+)\s*;", body)]


@pytest.mark.parametrize("cname,pyname", [("sk_solve_info", "SolveInfo"), ("sk_lsqr_info", "LsqrInfo"),
                                           ("sk_rsvd_info", "RsvdInfo"), ("sk_gn_info", "GnInfo"),
                                           ("sk_nystrom_info", "NystromInfo"), ("sk_extremes_info", "ExtremesInfo")])
def test_info_structs_match_header(cname, pyname):
    import ctypes as ct
    from paper_2508_21189_amd import libsketch
    st = getattr(libsketch, pyname)
    want = [(f, {"int": ct.c_int, "double": ct.c_double}[t]) for t, f in _header_struct_fields(cname)]
    assert [(f, t) for f, t in st._fields_] == want


def test_driver_null_handle_fails_cleanly():
    from paper_2508_21189_amd import libsketch
    lib = libsketch.load()
    info = libsketch.LsqrInfo()
    rc = lib.lstsq_sketch_precond(None, 4, None, 4, 0, None, 0, None, None, 1e-10, 10, 1, ctypes.byref(info), None)
    assert rc == libsketch.SK_E_INVAL
    assert lib.lstsq_sketch_solve(None, 4, None, 4, None, None, None, None) == libsketch.SK_E_INVAL
    out = ctypes.c_double(0)
    assert lib.lstsq_residual(None, 4, None, 4, None, None, ctypes.byref(out), None) == libsketch.SK_E_INVAL
    assert "invalid" in libsketch.last_error()
    sig = ctypes.c_void_p(0)
    assert lib.rsvd(None, 1, 4, None, 4, None, 4, None, None, 4, None, None) == libsketch.SK_E_INVAL
    assert lib.gen_nystrom(None, None, 1, 4, None, 4, None, 4, None, 4, None, None) == libsketch.SK_E_INVAL
    assert lib.gen_nystrom_svd(None, None, 1, 4, None, 4, None, 4, None, None, 4, None, None) == libsketch.SK_E_INVAL
    assert lib.nystrom_psd(None, 1, None, 4, None, 4, None, None, None) == libsketch.SK_E_INVAL
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    assert lib.sketch_sv_extremes(None, 10, 0, ctypes.byref(a), ctypes.byref(b), None, None) == libsketch.SK_E_INVAL


def test_ls_problem_layout_matches_header(tmp_path):
    """The binding's sk_ls_problem has the C compiler's field offsets and size."""
    import shutil
    import subprocess
    from paper_2508_21189_amd import libsketch
    if not shutil.which("gcc"):
        pytest.skip("no C compiler")
    fields = [f for f, _ in libsketch.LsProblem._fields_]
    body = "".join('printf("%%zu ", offsetof(sk_ls_problem, %s));' % f for f in fields)
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "libsketch.h"\n'
                   'int main(void) { %s printf("%%zu\\n", sizeof(sk_ls_problem)); return 0; }\n' % body)
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    want = [getattr(libsketch.LsProblem, f).offset for f in fields] + [ctypes.sizeof(libsketch.LsProblem)]
    assert got == want


def test_batched_rejects_invalid_problems_before_any_work():
    from paper_2508_21189_amd import libsketch
    lib = libsketch.load()
    assert lib.lstsq_sketch_solve_batched(None, 0, 4, 4, None, 0, None) == libsketch.SK_E_INVAL
    arr = (libsketch.LsProblem * 2)()
    for p in arr:  # k = 0 and null pointers: invalid
        p.n, p.k, p.dtype = 100, 0, 1
        p.status = 7
    assert lib.lstsq_sketch_solve_batched(arr, 2, 4, 4, None, 0, None) == libsketch.SK_E_INVAL
    assert [p.status for p in arr] == [libsketch.SK_E_INVAL] * 2
    assert "problem 0" in libsketch.last_error()
    size = ctypes.c_size_t(0)
    assert lib.lstsq_batched_workspace_size(arr, 2, 4, 4, ctypes.byref(size)) == libsketch.SK_E_INVAL


def test_batch_plan_validates_before_any_device_call():
    """lstsq_batched_create checks every problem before it touches the device: an empty problem (n = 0, null
    pointers) is refused with SK_E_INVAL and a message naming it, and no plan is returned."""
    from paper_2508_21189_amd import libsketch
    lib = libsketch.load()
    arr = (libsketch.LsProblem * 1)()
    h = ctypes.c_void_p()
    assert lib.lstsq_batched_create(arr, 1, 4, 4, 0, ctypes.byref(h)) == libsketch.SK_E_INVAL
    assert h.value is None and "problem 0" in libsketch.last_error()
