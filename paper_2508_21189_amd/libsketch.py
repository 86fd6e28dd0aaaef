"""Python binding of libsketch (ctypes). Argument marshalling only.

Every computation runs in the HIP library (libsketch.so, built for gfx950 by
paper_2508_21189_amd.build). PyTorch tensors supply device memory and the
current stream; nothing here computes a result. If the library is missing the
import fails loudly: there is no fallback path.
"""
import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsketch.so")

SK_SPARSESTACK, SK_GAUSSIAN, SK_SRTT, SK_SPARSERTT, SK_IDENTITY_TEST = 0, 1, 2, 3, 99
SK_F64, SK_F32, SK_BF16 = 0, 1, 2
SK_ROW_MAJOR, SK_COL_MAJOR = 0, 1
SK_OK, SK_E_INVAL, SK_E_NOMEM, SK_E_HIP, SK_E_NOTSUP = 0, -1, -2, -3, -4
SK_W_RANKDEF, SK_W_NOCONV = 1, 2

KINDS = {"sparsestack": SK_SPARSESTACK, "gaussian": SK_GAUSSIAN, "srtt": SK_SRTT, "sparsertt": SK_SPARSERTT,
         "identity": SK_IDENTITY_TEST}
_DT = {torch.float64: SK_F64, torch.float32: SK_F32, torch.bfloat16: SK_BF16}
_TORCH = {SK_F64: torch.float64, SK_F32: torch.float32, SK_BF16: torch.bfloat16}

_lib = None

_i64 = ctypes.c_int64
_vp = ctypes.c_void_p


class SketchError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("libsketch error %d: %s" % (code, msg))
        self.code = code


def load():
    """Load libsketch.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libsketch.so not built: run `python -m paper_2508_21189_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    lib.sketch_create.restype = _vp
    lib.sketch_create.argtypes = [ctypes.c_int, _i64, _i64, ctypes.c_int, ctypes.c_uint64]
    lib.sketch_destroy.argtypes = [_vp]
    lib.sketch_last_error.restype = ctypes.c_char_p
    lib.sketch_info.argtypes = [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(_i64), ctypes.POINTER(_i64),
                                ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_uint64)]
    lib.sketch_apply.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64, _vp, _i64, ctypes.c_int, _vp, _i64, _vp,
                                 ctypes.c_size_t, _vp]
    lib.sketch_apply_T.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64, _vp, _i64, ctypes.c_int, _vp, _i64, _vp,
                                   ctypes.c_size_t, _vp]
    lib.sketch_workspace_size.argtypes = [_vp, ctypes.c_int, ctypes.c_int, _i64, ctypes.POINTER(ctypes.c_size_t)]
    lib.sketch_adjoint.argtypes = [_vp, _i64, _vp, _i64, _vp, _i64, _vp]
    lib.sketch_pattern.argtypes = [_vp, _vp, _vp, _vp]
    lib.sketch_timing.argtypes = [_vp, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_i64)]
    if hasattr(lib, "sketch_apply_noalloc"):
        lib.sketch_apply_noalloc.argtypes = [_vp, ctypes.c_int, _i64, _vp, _i64, ctypes.c_int, _vp, _i64, _vp]
        lib.sketch_noalloc_scratch_bytes.restype = ctypes.c_size_t
        lib.sketch_noalloc_scratch_bytes.argtypes = []
    _bind_drivers(lib)
    _lib = lib
    return lib


def _bind_drivers(lib):
    """Argument types of the driver entry points (present once built)."""
    for name, args in _DRIVER_SIGS.items():
        fn = getattr(lib, name, None)
        if fn is not None:
            fn.argtypes = args
            fn.restype = ctypes.c_int


class SolveInfo(ctypes.Structure):
    """sk_solve_info."""
    _fields_ = [("rank", ctypes.c_int), ("sigma_max", ctypes.c_double), ("sigma_min_kept", ctypes.c_double),
                ("t_sketch_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class LsqrInfo(ctypes.Structure):
    """sk_lsqr_info."""
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("rnorm_est", ctypes.c_double),
                ("arnorm_est", ctypes.c_double), ("anorm_est", ctypes.c_double), ("t_sketch_ms", ctypes.c_double),
                ("t_qr_ms", ctypes.c_double), ("t_lsqr_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class RsvdInfo(ctypes.Structure):
    """sk_rsvd_info."""
    _fields_ = [("t_sketch_ms", ctypes.c_double), ("t_orth_ms", ctypes.c_double), ("t_project_ms", ctypes.c_double),
                ("t_svd_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double), ("jacobi_sweeps", ctypes.c_int)]


class GnInfo(ctypes.Structure):
    """sk_gn_info."""
    _fields_ = [("rank", ctypes.c_int), ("jacobi_sweeps", ctypes.c_int), ("t_sketch_ms", ctypes.c_double),
                ("t_core_ms", ctypes.c_double), ("t_factors_ms", ctypes.c_double), ("t_total_ms", ctypes.c_double)]


class NystromInfo(ctypes.Structure):
    """sk_nystrom_info."""
    _fields_ = [("nu", ctypes.c_double), ("t_sketch_ms", ctypes.c_double), ("t_core_ms", ctypes.c_double),
                ("t_total_ms", ctypes.c_double), ("jacobi_sweeps", ctypes.c_int)]


class ExtremesInfo(ctypes.Structure):
    """sk_extremes_info."""
    _fields_ = [("steps", ctypes.c_int), ("alpha_at_3_4", ctypes.c_double), ("beta_at_3_4", ctypes.c_double),
                ("t_build_ms", ctypes.c_double), ("t_iter_ms", ctypes.c_double)]


def _as_dict(st):
    return {name: getattr(st, name) for name, _ in st._fields_}


class LsProblem(ctypes.Structure):
    """sk_ls_problem (one problem of lstsq_sketch_solve_batched)."""
    _fields_ = [("n", _i64), ("k", _i64), ("dtype", ctypes.c_int), ("A", _vp), ("lda", _i64), ("b", _vp),
                ("x", _vp), ("seed", ctypes.c_uint64), ("status", ctypes.c_int), ("rank", ctypes.c_int),
                ("t_ms", ctypes.c_double)]


_DRIVER_SIGS = {
    "lstsq_sketch_solve": [_vp, _i64, _vp, _i64, _vp, _vp, ctypes.POINTER(SolveInfo), _vp],
    "lstsq_sketch_precond": [_vp, _i64, _vp, _i64, ctypes.c_int, _vp, _i64, _vp, _vp, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, ctypes.POINTER(LsqrInfo), _vp],
    "lstsq_residual": [_vp, _i64, _vp, _i64, _vp, _vp, ctypes.POINTER(ctypes.c_double), _vp],
    "lstsq_sketch_solve_async": [_vp, _i64, _vp, _i64, _vp, _vp, _vp, _vp, ctypes.c_size_t, _vp],
    "lstsq_solve_workspace_size": [_vp, _i64, ctypes.POINTER(ctypes.c_size_t)],
    "rsvd": [_vp, ctypes.c_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(RsvdInfo), _vp],
    "gen_nystrom": [_vp, _vp, ctypes.c_int, _i64, _vp, _i64, _vp, _i64, _vp, _i64, ctypes.POINTER(GnInfo), _vp],
    "gen_nystrom_svd": [_vp, _vp, ctypes.c_int, _i64, _vp, _i64, _vp, _i64, _vp, _vp, _i64, ctypes.POINTER(GnInfo),
                        _vp],
    "nystrom_psd": [_vp, ctypes.c_int, _vp, _i64, _vp, _i64, _vp, ctypes.POINTER(NystromInfo), _vp],
    "sketch_sv_extremes": [_vp, ctypes.c_int, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                           ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ExtremesInfo), _vp],
    "lstsq_batched_workspace_size": [ctypes.POINTER(LsProblem), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_size_t)],
    "lstsq_sketch_solve_batched": [ctypes.POINTER(LsProblem), ctypes.c_int, ctypes.c_int, ctypes.c_int, _vp,
                                   ctypes.c_size_t, _vp],
    "lstsq_batched_create": [ctypes.POINTER(LsProblem), ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                             ctypes.POINTER(_vp)],
    "lstsq_batched_workspace": [_vp, ctypes.POINTER(ctypes.c_size_t)],
    "lstsq_batched_bind": [_vp, _vp, ctypes.c_size_t, _vp],
    "lstsq_batched_launch": [_vp, _vp],
    "lstsq_batched_enqueue": [_vp, _vp],
    "lstsq_batched_results": [_vp, ctypes.POINTER(LsProblem), _vp],
    "lstsq_batched_info": [_vp, _vp],
    "lstsq_batched_destroy": [_vp],
    "sk_gemm_workspace_size": [ctypes.c_int, _i64, _i64, _i64, ctypes.POINTER(ctypes.c_size_t)],
    "sk_gemm": [ctypes.c_int, ctypes.c_int, ctypes.c_int, _i64, _i64, _i64, ctypes.c_double, _vp, _i64, _vp, _i64,
                ctypes.c_double, _vp, _i64, _vp, ctypes.c_size_t, _vp],
}

SK_BATCH_AUTOTUNE = 1
SK_BATCH_NOTUNE = 2


class BatchInfo(ctypes.Structure):
    """sk_batch_info."""
    _fields_ = [("graph_launches", _i64), ("kernel_nodes", ctypes.c_int), ("sketch_workgroups", ctypes.c_int),
                ("solve_workgroups", ctypes.c_int), ("sketch_items", ctypes.c_int), ("reduce_items", ctypes.c_int),
                ("tuned", ctypes.c_int), ("pad_", ctypes.c_int), ("workspace_bytes", ctypes.c_size_t)]


SOLVE_RESULT_BYTES = 24  # sk_solve_result: int rank, int pad, double sigma_max, double sigma_min_kept


def read_solve_result(buf):
    """(rank, sigma_max, sigma_min_kept) from a device sk_solve_result."""
    h = buf.cpu().numpy().tobytes()
    import struct
    r, _, smax, smin = struct.unpack("iidd", h[:24])
    return r, smax, smin


def exported_symbols():
    """Names the header declares; used by the load test."""
    return ["sketch_create", "sketch_destroy", "sketch_last_error", "sketch_info", "sketch_apply", "sketch_apply_T",
            "sketch_workspace_size", "sketch_adjoint", "sketch_pattern", "sketch_timing", "sketch_apply_noalloc",
            "sketch_noalloc_scratch_bytes"] + list(_DRIVER_SIGS)


def last_error():
    return load().sketch_last_error().decode()


def check(rc):
    if rc < 0:
        raise SketchError(rc, last_error())
    return rc


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


class Sketch:
    """Owns a libsketch handle: sketch_create(kind, d, n, zeta, seed)."""

    def __init__(self, kind, d, n, zeta=1, seed=0):
        lib = load()
        k = KINDS[kind] if isinstance(kind, str) else int(kind)
        h = lib.sketch_create(k, int(d), int(n), int(zeta), ctypes.c_uint64(int(seed) & 0xFFFFFFFFFFFFFFFF))
        if not h:
            raise SketchError(SK_E_INVAL, last_error())
        self.h = ctypes.c_void_p(h)
        self.kind, self.d, self.n, self.zeta, self.seed = k, int(d), int(n), int(zeta), int(seed)
        if k == SK_SPARSERTT:  # zeta = 0 asks for the default column sparsity
            z = ctypes.c_int(0)
            check(lib.sketch_info(self.h, None, None, None, ctypes.byref(z), None))
            self.zeta = z.value

    def close(self):
        if getattr(self, "h", None):
            load().sketch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace_size(self, op, dtype, m):
        b = ctypes.c_size_t(0)
        check(load().sketch_workspace_size(self.h, int(op), _DT[dtype], int(m), ctypes.byref(b)))
        return b.value

    def apply(self, A, out_dtype=None, out=None, ws=None, stream=None):
        """SA = S @ A for an (n x m) CUDA tensor A (float64/float32/bfloat16), row-major
        (stride(1) == 1) or column-major (stride(0) == 1, e.g. a transposed view)."""
        assert A.is_cuda and A.dim() == 2 and A.shape[0] == self.n
        m = A.shape[1]
        if A.stride(1) == 1 and (A.stride(0) >= m or m == 1):
            layout, lda = SK_ROW_MAJOR, A.stride(0)
        else:
            assert A.stride(0) == 1, "A must be row-major or column-major"
            layout, lda = SK_COL_MAJOR, A.stride(1)
        odt = out_dtype or (torch.float64 if A.dtype == torch.float64 else torch.float32)
        if out is None:
            out = torch.empty((self.d, m), dtype=odt, device=A.device)
        assert out.shape == (self.d, m) and out.stride(1) == 1 and out.dtype == odt
        wsp, wsb = (None, 0) if ws is None else (_ptr(ws), ws.numel() * ws.element_size())
        check(load().sketch_apply(self.h, _DT[A.dtype], layout, m, _ptr(A), lda, _DT[odt], _ptr(out),
                                  out.stride(0), wsp, wsb, _stream(stream)))
        return out

    def apply_noalloc(self, A, out_dtype=None, out=None, stream=None):
        """SA = S @ A through sketch_apply_noalloc (row-major A, SparseStack): the
        library's fixed device scratch array instead of any workspace."""
        assert A.is_cuda and A.dim() == 2 and A.shape[0] == self.n and A.stride(1) == 1
        m = A.shape[1]
        odt = out_dtype or (torch.float64 if A.dtype == torch.float64 else torch.float32)
        if out is None:
            out = torch.empty((self.d, m), dtype=odt, device=A.device)
        assert out.shape == (self.d, m) and out.stride(1) == 1 and out.dtype == odt
        check(load().sketch_apply_noalloc(self.h, _DT[A.dtype], m, _ptr(A), A.stride(0), _DT[odt], _ptr(out),
                                          out.stride(0), _stream(stream)))
        return out

    def apply_T(self, A, out_dtype=None, out=None, ws=None, stream=None):
        """Y = A @ S^T for a (rows x n) CUDA tensor A, row-major (stride(1) == 1)
        or column-major (stride(0) == 1, e.g. a transposed view)."""
        assert A.is_cuda and A.dim() == 2 and A.shape[1] == self.n
        rows = A.shape[0]
        if A.stride(1) == 1 and (A.stride(0) >= self.n or rows == 1):
            layout, lda = SK_ROW_MAJOR, A.stride(0)
        else:
            assert A.stride(0) == 1, "A must be row-major or column-major"
            layout, lda = SK_COL_MAJOR, A.stride(1)
        odt = out_dtype or (torch.float64 if A.dtype == torch.float64 else torch.float32)
        if out is None:
            out = torch.empty((rows, self.d), dtype=odt, device=A.device)
        assert out.shape == (rows, self.d) and out.stride(1) == 1 and out.dtype == odt
        wsp, wsb = (None, 0) if ws is None else (_ptr(ws), ws.numel() * ws.element_size())
        check(load().sketch_apply_T(self.h, _DT[A.dtype], layout, rows, _ptr(A), lda, _DT[odt], _ptr(out),
                                    out.stride(0), wsp, wsb, _stream(stream)))
        return out

    def adjoint(self, Y, stream=None):
        """Z = S^T @ Y (float64, SparseStack only)."""
        assert Y.is_cuda and Y.dtype == torch.float64 and Y.shape[0] == self.d and Y.stride(1) == 1
        Z = torch.empty((self.n, Y.shape[1]), dtype=torch.float64, device=Y.device)
        check(load().sketch_adjoint(self.h, Y.shape[1], _ptr(Y), Y.stride(0), _ptr(Z), Z.stride(0), _stream(stream)))
        return Z

    def timing(self, mode):
        """sketch_timing: 1 enable/reset, 0 disable/reset, 2 query -> (total_ms, launches)."""
        ms, cnt = ctypes.c_double(0), _i64(0)
        check(load().sketch_timing(self.h, int(mode), ctypes.byref(ms), ctypes.byref(cnt)))
        return ms.value, cnt.value

    def pattern(self, device="cuda", stream=None):
        """(bucket int32 [n, zeta], sign int8 [n, zeta]) from the device hash."""
        b = torch.empty((self.n, self.zeta), dtype=torch.int32, device=device)
        s = torch.empty((self.n, self.zeta), dtype=torch.int8, device=device)
        check(load().sketch_pattern(self.h, _ptr(b), _ptr(s), _stream(stream)))
        return b, s

    # -- least-squares drivers -------------------------------------------------
    def _check_system(self, A, b):
        assert A.is_cuda and A.dtype == torch.float64 and A.dim() == 2 and A.shape[0] == self.n
        assert A.stride(1) == 1
        assert b.is_cuda and b.dtype == torch.float64 and b.shape == (self.n,) and b.is_contiguous()

    def lstsq_solve(self, A, b, stream=None):
        """Sketch-and-solve: returns (x, status, info dict)."""
        self._check_system(A, b)
        m = A.shape[1]
        x = torch.empty(m, dtype=torch.float64, device=A.device)
        info = SolveInfo()
        rc = check(load().lstsq_sketch_solve(self.h, m, _ptr(A), A.stride(0), _ptr(b), _ptr(x), ctypes.byref(info),
                                             _stream(stream)))
        return x, rc, _as_dict(info)

    def solve_workspace_size(self, m):
        """Bytes of workspace lstsq_sketch_solve_async needs for m columns."""
        out = ctypes.c_size_t(0)
        check(load().lstsq_solve_workspace_size(self.h, int(m), ctypes.byref(out)))
        return out.value

    def lstsq_solve_async(self, A, b, x, ws, result=None, stream=None):
        """Sketch-and-solve enqueued on `stream` with no host synchronization and
        no allocation (x, ws and the optional device result buffer of 24 bytes
        (SOLVE_RESULT_BYTES) are caller tensors); capturable into a HIP graph."""
        self._check_system(A, b)
        assert x.is_cuda and x.dtype == torch.float64 and x.shape == (A.shape[1],)
        res = _ptr(result) if result is not None else None
        return check(load().lstsq_sketch_solve_async(self.h, A.shape[1], _ptr(A), A.stride(0), _ptr(b), _ptr(x), res,
                                                     _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))

    def lstsq_precond(self, A, b, tol=1e-10, maxit=100, warm_start=True, A_sketch=None, stream=None):
        """Sketch-and-precondition LSQR: returns (x, status, info dict).

        A_sketch: optional float32/bfloat16/float64 copy of A that is sketched instead of A.
        """
        self._check_system(A, b)
        m = A.shape[1]
        x = torch.empty(m, dtype=torch.float64, device=A.device)
        info = LsqrInfo()
        if A_sketch is not None:
            assert A_sketch.is_cuda and A_sketch.shape == A.shape and A_sketch.stride(1) == 1
            sdt, sp, sld = _DT[A_sketch.dtype], _ptr(A_sketch), A_sketch.stride(0)
        else:
            sdt, sp, sld = SK_F64, None, 0
        rc = check(load().lstsq_sketch_precond(self.h, m, _ptr(A), A.stride(0), sdt, sp, sld, _ptr(b), _ptr(x),
                                               float(tol), int(maxit), int(bool(warm_start)), ctypes.byref(info),
                                               _stream(stream)))
        return x, rc, _as_dict(info)

    def residual(self, A, b, x, stream=None):
        """||b - A x||_2 computed on the device in float64."""
        self._check_system(A, b)
        out = ctypes.c_double(0)
        check(load().lstsq_residual(self.h, A.shape[1], _ptr(A), A.stride(0), _ptr(b), _ptr(x), ctypes.byref(out),
                                    _stream(stream)))
        return out.value

    # -- randomized SVD ----------------------------------------------------------
    def rsvd(self, A, want_u=True, want_vt=True, stream=None):
        """Alg. 1 with this sketch (k = d): returns (U, sigma, Vt, status, info dict)."""
        assert A.is_cuda and A.dim() == 2 and A.shape[1] == self.n and A.stride(1) == 1
        assert A.dtype in (torch.float32, torch.float64)
        rows, k = A.shape[0], self.d
        dev = A.device
        U = torch.empty((rows, k), dtype=torch.float64, device=dev) if want_u else None
        Vt = torch.empty((k, self.n), dtype=torch.float64, device=dev) if want_vt else None
        sig = torch.empty(k, dtype=torch.float64, device=dev)
        info = RsvdInfo()
        rc = check(load().rsvd(self.h, _DT[A.dtype], rows, _ptr(A), A.stride(0),
                               _ptr(U) if U is not None else None, k,
                               _ptr(sig), _ptr(Vt) if Vt is not None else None, self.n,
                               ctypes.byref(info), _stream(stream)))
        return U, sig, Vt, rc, _as_dict(info)


def gen_nystrom(S_omega, S_psi, A, form="outer", stream=None):
    """Generalized Nystrom with Omega = S_omega^T (k x cols sketch) and Psi = S_psi^T (p x rows sketch).

    form "outer" (Alg. 4): returns (F, G, status, info), A ~ F G^T.
    form "svd" (Alg. 5): returns (U, sigma, V, status, info), A ~ U diag(sigma) V^T.
    """
    assert A.is_cuda and A.dim() == 2 and A.stride(1) == 1 and A.dtype in (torch.float32, torch.float64)
    rows, cols = A.shape
    assert S_omega.n == cols and S_psi.n == rows
    k = S_omega.d
    dev = A.device
    info = GnInfo()
    lib = load()
    if form == "outer":
        F = torch.empty((rows, k), dtype=torch.float64, device=dev)
        G = torch.empty((cols, k), dtype=torch.float64, device=dev)
        rc = check(lib.gen_nystrom(S_omega.h, S_psi.h, _DT[A.dtype], rows, _ptr(A), A.stride(0), _ptr(F), k, _ptr(G),
                                   k, ctypes.byref(info), _stream(stream)))
        return F, G, rc, _as_dict(info)
    if form == "svd":
        U = torch.empty((rows, k), dtype=torch.float64, device=dev)
        V = torch.empty((cols, k), dtype=torch.float64, device=dev)
        sig = torch.empty(k, dtype=torch.float64, device=dev)
        rc = check(lib.gen_nystrom_svd(S_omega.h, S_psi.h, _DT[A.dtype], rows, _ptr(A), A.stride(0), _ptr(U), k,
                                       _ptr(sig), _ptr(V), k, ctypes.byref(info), _stream(stream)))
        return U, sig, V, rc, _as_dict(info)
    raise ValueError("form must be 'outer' or 'svd'")


def sv_extremes(S, steps=300, start_seed=0, stream=None):
    """Injectivity and dilation of a SparseStack S on Q = [e_1 ... e_n] (Fig. 2):
    returns (alpha, beta, status, info), the extreme eigenvalues of S^T S
    estimated by `steps` Lanczos steps on the device."""
    a, b = ctypes.c_double(0), ctypes.c_double(0)
    info = ExtremesInfo()
    rc = check(load().sketch_sv_extremes(S.h, int(steps), ctypes.c_uint64(int(start_seed) & 0xFFFFFFFFFFFFFFFF),
                                         ctypes.byref(a), ctypes.byref(b), ctypes.byref(info), _stream(stream)))
    return a.value, b.value, rc, _as_dict(info)


def nystrom_psd(S, A, stream=None):
    """Alg. 2 with Omega = S^T (S a k x n sketch): returns (U, lambda, status, info), A ~ U diag(lambda) U^T."""
    assert A.is_cuda and A.dim() == 2 and A.shape[0] == A.shape[1] == S.n and A.stride(1) == 1
    assert A.dtype in (torch.float32, torch.float64)
    n, k = S.n, S.d
    U = torch.empty((n, k), dtype=torch.float64, device=A.device)
    lam = torch.empty(k, dtype=torch.float64, device=A.device)
    info = NystromInfo()
    rc = check(load().nystrom_psd(S.h, _DT[A.dtype], _ptr(A), A.stride(0), _ptr(U), k, _ptr(lam), ctypes.byref(info),
                                  _stream(stream)))
    return U, lam, rc, _as_dict(info)


def _batched_array(problems):
    """sk_ls_problem array for [(A, b, seed), ...] (A n x k row-major, b n elements of A's dtype, CUDA)."""
    arr = (LsProblem * len(problems))()
    xs = []
    # one allocation for every solution (each x a view of k elements)
    ks = [int(A.shape[1]) for A, _, _ in problems]
    offs = [0]
    for k in ks:
        offs.append(offs[-1] + ((k + 31) // 32) * 32)
    xall = torch.empty(max(1, offs[-1]), dtype=torch.float64, device=problems[0][0].device) if problems else None
    for i, (A, b, seed) in enumerate(problems):
        assert A.is_cuda and A.dim() == 2 and A.stride(1) == 1 and A.dtype in _DT
        assert b.is_cuda and b.dtype == A.dtype and b.numel() == A.shape[0] and b.is_contiguous()
        assert A.device == xall.device
        x = xall[offs[i]:offs[i] + ks[i]]
        xs.append(x)
        arr[i] = LsProblem(A.shape[0], A.shape[1], _DT[A.dtype], _ptr(A), A.stride(0), _ptr(b), _ptr(x),
                           int(seed) & 0xFFFFFFFFFFFFFFFF, 0, 0, 0.0)
    return arr, xs


def batched_workspace_size(problems, d_per_k=4, zeta=4):
    arr, _ = _batched_array(problems)
    nbytes = ctypes.c_size_t(0)
    check(load().lstsq_batched_workspace_size(arr, len(problems), d_per_k, zeta, ctypes.byref(nbytes)))
    return nbytes.value


class BatchPlan:
    """A batch plan (lstsq_batched_create ... destroy) over [(A, b, seed), ...]: bind() a workspace once,
    then launch() runs the whole batch as one graph launch; results() waits and returns
    (statuses, ranks, t_ms, status of the call). xs holds the solution vectors."""

    def __init__(self, problems, d_per_k=4, zeta=4, flags=0):
        self.arr, self.xs = _batched_array(problems)
        self.n = len(problems)
        self.keep = problems  # the tensors must outlive the plan
        h = _vp()
        check(load().lstsq_batched_create(self.arr, self.n, d_per_k, zeta, flags, ctypes.byref(h)))
        self.h = h
        self.ws = None

    def workspace_bytes(self):
        nbytes = ctypes.c_size_t(0)
        check(load().lstsq_batched_workspace(self.h, ctypes.byref(nbytes)))
        return nbytes.value

    def bind(self, ws=None, stream=None):
        if ws is None:
            ws = torch.empty(self.workspace_bytes() + 256, dtype=torch.uint8, device="cuda")
            off = (-ws.data_ptr()) % 256
            ws = ws[off:]
        self.ws = ws
        check(load().lstsq_batched_bind(self.h, _ptr(ws), ws.numel(), _stream(stream)))
        return ws

    def launch(self, stream=None):
        check(load().lstsq_batched_launch(self.h, _stream(stream)))

    def enqueue(self, stream=None):
        check(load().lstsq_batched_enqueue(self.h, _stream(stream)))

    def results(self, stream=None):
        rc = check(load().lstsq_batched_results(self.h, self.arr, _stream(stream)))
        return [p.status for p in self.arr], [p.rank for p in self.arr], [p.t_ms for p in self.arr], rc

    def info(self):
        inf = BatchInfo()
        check(load().lstsq_batched_info(self.h, ctypes.byref(inf)))
        return inf

    def close(self):
        if self.h is not None:
            load().lstsq_batched_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gemm(A, B, transA=False, transB=False, alpha=1.0, beta=0.0, C=None, stream=None):
    """sk_gemm: C = alpha op(A) op(B) + beta C for 2-D row-major CUDA tensors (float32 or float64; rows may be
    padded: stride(1) == 1). Returns C."""
    dt = _DT[A.dtype]
    assert A.dtype == B.dtype and A.is_cuda and B.is_cuda and A.stride(1) == 1 and B.stride(1) == 1
    M = A.shape[1] if transA else A.shape[0]
    K = A.shape[0] if transA else A.shape[1]
    N = B.shape[0] if transB else B.shape[1]
    assert (B.shape[1] if transB else B.shape[0]) == K
    if C is None:
        C = torch.zeros(M, N, dtype=A.dtype, device=A.device)
    assert C.shape == (M, N) and C.stride(1) == 1 and C.dtype == A.dtype
    nbytes = ctypes.c_size_t(0)
    check(load().sk_gemm_workspace_size(dt, M, N, K, ctypes.byref(nbytes)))
    ws = torch.empty(max(1, nbytes.value), dtype=torch.uint8, device=A.device)
    check(load().sk_gemm(dt, int(transA), int(transB), M, N, K, float(alpha), _ptr(A), A.stride(0), _ptr(B),
                         B.stride(0), float(beta), _ptr(C), C.stride(0), _ptr(ws), nbytes.value, _stream(stream)))
    return C


def solve_batched(problems, d_per_k=4, zeta=4, ws=None, stream=None):
    """lstsq_sketch_solve_batched over [(A, b, seed), ...]: problem p is sketched by its own SparseStack
    (d = d_per_k * k, zeta blocks, key seed). Returns (xs, statuses, ranks, t_ms, status of the call)."""
    arr, xs = _batched_array(problems)
    wsp, wsb = (None, 0) if ws is None else (_ptr(ws), ws.numel() * ws.element_size())
    rc = check(load().lstsq_sketch_solve_batched(arr, len(problems), d_per_k, zeta, wsp, wsb, _stream(stream)))
    return xs, [p.status for p in arr], [p.rank for p in arr], [p.t_ms for p in arr], rc
