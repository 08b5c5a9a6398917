"""Python binding of the MI355X sketch-and-precondition least-squares library.

Thin ctypes layer over the C ABI in ``include/sap.h`` (same names): it only
marshals torch device tensors into pointers and passes the current HIP stream.
Every step of the method runs in the HIP kernels of ``libsap.so``; there is no
fallback path.  Importing works without a GPU; calling needs the built library
and a GPU, and raises otherwise.
"""
import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_build", "libsap.so")

SAP_OK, SAP_EINVAL, SAP_ENOMEM, SAP_RANK_DEFICIENT, SAP_NOT_CONVERGED, SAP_PENDING, SAP_EDEVICE, SAP_ECANCELED = range(8)
STATUS_NAMES = {0: "SAP_OK", 1: "SAP_EINVAL", 2: "SAP_ENOMEM", 3: "SAP_RANK_DEFICIENT",
                4: "SAP_NOT_CONVERGED", 5: "SAP_PENDING", 6: "SAP_EDEVICE", 7: "SAP_ECANCELED"}
SAP_F64, SAP_F32, SAP_BF16 = 0, 1, 2
SAP_MODE_FP64, SAP_MODE_MIXED_FP32, SAP_MODE_MIXED_FP32_REFINE, SAP_MODE_MIXED_BF16SA = 0, 1, 2, 3

# Every symbol the header declares (checked by the CPU test suite).
EXPORTS = ["sap_create", "sap_destroy", "sap_last_error", "sap_status_string", "sps_generate",
           "sps_apply", "sps_apply_noalloc", "sap_qr", "sap_trsv", "sap_solve", "sap_lsqr", "sap_profile_enable",
           "sap_profile_read", "sap_solve_batch", "sap_serve_start", "sap_submit", "sap_poll",
           "sap_cancel", "sap_serve_stats", "sap_embedding_dim", "sap_iteration_estimate", "sap_choose_d",
           "sps_apply_csr", "sap_solve_csr", "sap_solve_hbm", "sap_solve_sstep"]
PROF_PASS, PROF_APPLY = 0, 1

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f64 = ctypes.c_double


class SpsSketch(ctypes.Structure):
    _fields_ = [("m", _i64), ("d", _i32), ("zeta", _i32), ("seed", _u64), ("stream", _u64),
                ("idx", _vp), ("sign", _vp)]


class SapProblem(ctypes.Structure):
    _fields_ = [("m", _i64), ("n", _i32), ("A", _vp), ("lda", _i64), ("a_type", _i32), ("b", _vp)]


class SapCsr(ctypes.Structure):
    _fields_ = [("m", _i64), ("n", _i32), ("nnz", _i64), ("indptr", _vp), ("indices", _vp), ("values", _vp),
                ("v_type", _i32)]


class SapHbmParams(ctypes.Structure):
    _fields_ = [("alpha", _f64), ("beta", _f64), ("eta_scale", _f64), ("gradient_descent", _i32), ("pad_", _i32)]


class SapSstepParams(ctypes.Structure):
    _fields_ = [("s", _i32), ("pad_", _i32), ("eta_scale", _f64)]


class SapParams(ctypes.Structure):
    _fields_ = [("d", _i32), ("zeta", _i32), ("seed", _u64), ("tol", _f64), ("maxiter", _i32),
                ("mode", _i32), ("max_refine", _i32), ("fixed_iters", _i32)]


class SapInfo(ctypes.Structure):
    _fields_ = [("status", _i32), ("iters", _i32), ("refinements", _i32), ("resid_est", _f64), ("normar_est", _f64), ("t_generate_ms", _f64),
                ("t_apply_ms", _f64), ("t_qr_ms", _f64), ("t_iterate_ms", _f64),
                ("t_queue_ms", _f64), ("t_total_ms", _f64), ("d_used", _i32), ("pad_", _i32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_} | {
            "status_name": STATUS_NAMES.get(self.status, str(self.status))}


class SapError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def lib():
    """Load libsap.so (built in-tree by ``build.py``).  Raises if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2506_03070_amd/build.py "
                               "(there is no fallback implementation)")
        L = ctypes.CDLL(LIB_PATH)
        L.sap_create.argtypes = [ctypes.POINTER(_vp), ctypes.c_int, ctypes.c_size_t]
        L.sap_create.restype = ctypes.c_int
        L.sap_destroy.argtypes = [_vp]
        L.sap_destroy.restype = None
        L.sap_last_error.argtypes = [_vp]
        L.sap_last_error.restype = ctypes.c_char_p
        L.sap_status_string.argtypes = [ctypes.c_int]
        L.sap_status_string.restype = ctypes.c_char_p
        L.sps_generate.argtypes = [_vp, ctypes.POINTER(SpsSketch), _vp]
        L.sps_generate.restype = ctypes.c_int
        L.sps_apply.argtypes = [_vp, ctypes.POINTER(SpsSketch), _vp, _i64, ctypes.c_int, _vp, _i32, _vp,
                                _i64, ctypes.c_int, _vp]
        L.sps_apply.restype = ctypes.c_int
        L.sps_apply_noalloc.argtypes = L.sps_apply.argtypes
        L.sps_apply_noalloc.restype = ctypes.c_int
        L.sap_qr.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _vp]
        L.sap_qr.restype = ctypes.c_int
        L.sap_trsv.argtypes = [_vp, _vp, _i64, _i32, _i32, _vp, _vp, _vp]
        L.sap_trsv.restype = ctypes.c_int
        L.sap_solve.argtypes = [_vp, ctypes.POINTER(SapProblem), ctypes.POINTER(SapParams), _vp,
                                ctypes.POINTER(SapInfo), _vp]
        L.sap_solve.restype = ctypes.c_int
        L.sap_lsqr.argtypes = [_vp, ctypes.POINTER(SapProblem), _vp, _i64, _vp, _f64, _i32, _vp,
                               ctypes.POINTER(SapInfo), _vp]
        L.sap_lsqr.restype = ctypes.c_int
        L.sap_solve_batch.argtypes = [_vp, _i32, ctypes.POINTER(SapProblem), ctypes.POINTER(SapParams),
                                      ctypes.POINTER(_vp), ctypes.POINTER(SapInfo), _vp]
        L.sap_solve_batch.restype = ctypes.c_int
        L.sap_serve_start.argtypes = [_vp, ctypes.c_size_t, _i32]
        L.sap_serve_start.restype = ctypes.c_int
        L.sap_submit.argtypes = [_vp, ctypes.POINTER(SapProblem), ctypes.POINTER(SapParams), _vp,
                                 ctypes.POINTER(_u64), _vp]
        L.sap_submit.restype = ctypes.c_int
        L.sap_poll.argtypes = [_vp, _u64, ctypes.POINTER(SapInfo), _i32]
        L.sap_poll.restype = ctypes.c_int
        L.sap_cancel.argtypes = [_vp, _u64]
        L.sap_cancel.restype = ctypes.c_int
        L.sap_serve_stats.argtypes = [_vp, ctypes.POINTER(_i64)]
        L.sap_serve_stats.restype = ctypes.c_int
        L.sap_profile_enable.argtypes = [_vp, ctypes.c_int]
        L.sap_profile_enable.restype = ctypes.c_int
        L.sap_profile_read.argtypes = [_vp, _i32, ctypes.POINTER(_i64), ctypes.POINTER(_f64), ctypes.c_int]
        L.sap_profile_read.restype = ctypes.c_int
        L.sap_embedding_dim.argtypes = [_i64, _i32, _f64, _f64, ctypes.POINTER(_i32)]
        L.sap_embedding_dim.restype = ctypes.c_int
        L.sap_iteration_estimate.argtypes = [_i32, _i32, _f64, ctypes.POINTER(_i32)]
        L.sap_iteration_estimate.restype = ctypes.c_int
        L.sap_choose_d.argtypes = [_vp, ctypes.POINTER(SapProblem), _i32, _f64, ctypes.POINTER(_i32), _vp]
        L.sap_choose_d.restype = ctypes.c_int
        L.sps_apply_csr.argtypes = [_vp, ctypes.POINTER(SpsSketch), ctypes.POINTER(SapCsr), _vp, _vp, _i64, _vp]
        L.sps_apply_csr.restype = ctypes.c_int
        L.sap_solve_csr.argtypes = [_vp, ctypes.POINTER(SapCsr), _vp, ctypes.POINTER(SapParams), _vp,
                                    ctypes.POINTER(SapInfo), _vp]
        L.sap_solve_csr.restype = ctypes.c_int
        L.sap_solve_hbm.argtypes = [_vp, ctypes.POINTER(SapProblem), ctypes.POINTER(SapParams),
                                    ctypes.POINTER(SapHbmParams), _vp, ctypes.POINTER(SapInfo), _vp]
        L.sap_solve_hbm.restype = ctypes.c_int
        L.sap_solve_sstep.argtypes = [_vp, ctypes.POINTER(SapProblem), ctypes.POINTER(SapParams),
                                      ctypes.POINTER(SapSstepParams), _vp, ctypes.POINTER(SapInfo), _vp]
        L.sap_solve_sstep.restype = ctypes.c_int
        _lib = L
    return _lib


def _torch():
    import torch
    return torch


def _stream():
    return _torch().cuda.current_stream().cuda_stream


def _dev(t, dtype=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    return t.data_ptr()


def _ld(t):
    """Leading dimension of a 2-D tensor whose rows are contiguous (torch
    reports an arbitrary stride for a dimension of size 1)."""
    if t.dim() != 2 or t.stride(1) != 1:
        raise ValueError("expected a 2-D tensor with contiguous rows")
    return t.stride(0) if t.shape[0] > 1 else t.shape[1]


def _dtype_code(t):
    torch = _torch()
    return {torch.float64: SAP_F64, torch.float32: SAP_F32, torch.bfloat16: SAP_BF16}[t.dtype]


class Context:
    """Owns a sap_ctx (device, HBM-budgeted workspace)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._ptr = _vp()
        st = lib().sap_create(ctypes.byref(self._ptr), device, hbm_budget)
        if st != SAP_OK:
            raise SapError(st, "sap_create failed")
        self.device = device

    @property
    def handle(self):
        return self._ptr

    def last_error(self):
        return lib().sap_last_error(self._ptr).decode()

    def check(self, st, allow=(SAP_OK,)):
        if st not in allow:
            raise SapError(st, self.last_error())
        return st

    def profile(self, enable=True):
        self.check(lib().sap_profile_enable(self._ptr, 1 if enable else 0))

    def profile_read(self, kernel, reset=False):
        """(launches, total_ms) of kernel PROF_PASS or PROF_APPLY."""
        n = _i64()
        ms = _f64()
        self.check(lib().sap_profile_read(self._ptr, kernel, ctypes.byref(n), ctypes.byref(ms), 1 if reset else 0))
        return n.value, ms.value

    def close(self):
        if self._ptr:
            lib().sap_destroy(self._ptr)
            self._ptr = _vp()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


_default = {}


def default_context(device: int = 0) -> Context:
    if device not in _default:
        _default[device] = Context(device)
    return _default[device]


def _sketch_struct(m, d, zeta, seed, stream_id, idx, sign):
    return SpsSketch(m, d, zeta, seed, stream_id, _dev(idx, name="idx"), _dev(sign, name="sign"))


def sps_generate(m, d, zeta, seed, stream_id=0, ctx=None, idx=None, sign=None):
    """Sparse sign sketch on the GPU: returns (idx int32 (m, zeta), sign int64 (m,)) tensors;
    sign holds the uint64 words bit for bit."""
    torch = _torch()
    ctx = ctx or default_context()
    dev = torch.device("cuda", ctx.device)
    idx = idx if idx is not None else torch.empty((m, zeta), dtype=torch.int32, device=dev)
    sign = sign if sign is not None else torch.empty((m,), dtype=torch.int64, device=dev)
    S = _sketch_struct(m, d, zeta, seed, stream_id, idx, sign)
    ctx.check(lib().sps_generate(ctx.handle, ctypes.byref(S), _vp(_stream())))
    return idx, sign


def sps_apply(idx, sign, d, zeta, A, b=None, y_dtype=None, ctx=None, seed=0, stream_id=0, Y=None):
    """Y = S [A b] with S given by (idx, sign).  Returns Y as a (ncols, d)
    tensor whose rows are the columns of the column-major d x ncols result."""
    torch = _torch()
    ctx = ctx or default_context()
    m, n = A.shape
    y_dtype = y_dtype or (torch.float64 if A.dtype == torch.float64 else torch.float32)
    ncols = n + (1 if b is not None else 0)
    Y = Y if Y is not None else torch.empty((ncols, d), dtype=y_dtype, device=A.device)
    S = _sketch_struct(m, d, zeta, seed, stream_id, idx, sign)
    bptr = _dev(b, torch.float64, "b") if b is not None else None
    ctx.check(lib().sps_apply(ctx.handle, ctypes.byref(S), _dev(A, name="A"), _ld(A), _dtype_code(A),
                              bptr, n, _dev(Y, y_dtype, "Y"), _ld(Y), _dtype_code(Y), _vp(_stream())))
    return Y


def sps_apply_noalloc(idx, sign, d, zeta, A, b=None, y_dtype=None, ctx=None, seed=0, stream_id=0, Y=None):
    """sps_apply through the allocation-free entry point (partial sums in the
    library's static device buffer).  Same arguments and result layout as
    sps_apply."""
    torch = _torch()
    ctx = ctx or default_context()
    m, n = A.shape
    y_dtype = y_dtype or (torch.float64 if A.dtype == torch.float64 else torch.float32)
    ncols = n + (1 if b is not None else 0)
    Y = Y if Y is not None else torch.empty((ncols, d), dtype=y_dtype, device=A.device)
    S = _sketch_struct(m, d, zeta, seed, stream_id, idx, sign)
    bptr = _dev(b, torch.float64, "b") if b is not None else None
    ctx.check(lib().sps_apply_noalloc(ctx.handle, ctypes.byref(S), _dev(A, name="A"), _ld(A), _dtype_code(A),
                                      bptr, n, _dev(Y, y_dtype, "Y"), _ld(Y), _dtype_code(Y), _vp(_stream())))
    return Y


def _csr_struct(indptr, indices, values, shape):
    torch = _torch()
    m, n = shape
    if indptr.dtype != torch.int64 or indices.dtype != torch.int32:
        raise TypeError("CSR indptr must be int64 and indices int32")
    return SapCsr(int(m), int(n), int(indices.numel()), _dev(indptr, name="indptr"),
                  _dev(indices, name="indices") if indices.numel() else None,
                  _dev(values, name="values") if values.numel() else None, _dtype_code(values))


def sps_apply_csr(idx, sign, d, zeta, indptr, indices, values, shape, b=None, ctx=None, seed=0, stream_id=0, Y=None):
    """Y = S [A b] for a CSR A given by device tensors (indptr int64 (m+1),
    indices int32, values F64/F32) and shape (m, n).  Returns a (ncols, d)
    float64 tensor whose rows are the columns of Y."""
    torch = _torch()
    ctx = ctx or default_context()
    m, n = shape
    ncols = n + (1 if b is not None else 0)
    Y = Y if Y is not None else torch.empty((ncols, d), dtype=torch.float64, device=indptr.device)
    S = _sketch_struct(m, d, zeta, seed, stream_id, idx, sign)
    A = _csr_struct(indptr, indices, values, shape)
    bptr = _dev(b, torch.float64, "b") if b is not None else None
    ctx.check(lib().sps_apply_csr(ctx.handle, ctypes.byref(S), ctypes.byref(A), bptr, _dev(Y, torch.float64, "Y"),
                                  _ld(Y), _vp(_stream())))
    return Y


def sap_solve_csr(indptr, indices, values, shape, b, d, zeta=8, seed=1, tol=1e-12, maxiter=200, mode=None,
                  ctx=None, x=None, fixed_iters=0):
    """min ||b - A x|| for a CSR A (sap_solve_csr)."""
    torch = _torch()
    ctx = ctx or default_context()
    if mode is None:
        mode = SAP_MODE_FP64 if values.dtype == torch.float64 else SAP_MODE_MIXED_FP32
    A = _csr_struct(indptr, indices, values, shape)
    par = SapParams(int(d), int(zeta), int(seed), float(tol), int(maxiter), int(mode), 0, int(fixed_iters))
    x = x if x is not None else torch.empty(shape[1], dtype=torch.float64, device=indptr.device)
    info = SapInfo()
    st = lib().sap_solve_csr(ctx.handle, ctypes.byref(A), _vp(_dev(b, torch.float64, "b")), ctypes.byref(par),
                             _vp(_dev(x, torch.float64, "x")), ctypes.byref(info), _vp(_stream()))
    ctx.check(st, (SAP_OK, SAP_NOT_CONVERGED))
    return SolveResult(x, st, info.as_dict())


def sap_qr(Yt, ctx=None):
    """In-place Householder QR of the column-major matrix stored as the rows of
    Yt (shape (cols, ldy), float64).  Returns tau (cols,)."""
    torch = _torch()
    ctx = ctx or default_context()
    cols, ldy = Yt.shape
    tau = torch.empty(cols, dtype=torch.float64, device=Yt.device)
    ctx.check(lib().sap_qr(ctx.handle, _dev(Yt, torch.float64, "Y"), _ld(Yt), ldy, cols,
                           _dev(tau, torch.float64, "tau"), _vp(_stream())))
    return tau


def sap_trsv(Rt, rhs, trans=False, n=None, ctx=None, out=None):
    """Solve R x = rhs (or R^T x = rhs) with R the upper triangle of the
    column-major matrix stored as the rows of Rt (shape (>= n, ldr))."""
    torch = _torch()
    ctx = ctx or default_context()
    n = n or rhs.shape[0]
    out = out if out is not None else torch.empty(n, dtype=torch.float64, device=rhs.device)
    ctx.check(lib().sap_trsv(ctx.handle, _dev(Rt, torch.float64, "R"), _ld(Rt), n, 1 if trans else 0,
                             _dev(rhs, torch.float64, "rhs"), _dev(out, torch.float64, "x"), _vp(_stream())))
    return out


def _problem(A, b):
    torch = _torch()
    m, n = A.shape
    return SapProblem(m, n, _dev(A, name="A"), _ld(A), _dtype_code(A), _dev(b, torch.float64, "b"))


@dataclass
class SolveResult:
    x: object
    status: int
    info: dict


def sap_solve(A, b, d, zeta=8, seed=1, tol=1e-12, maxiter=200, mode=None, ctx=None, x=None,
              allow_not_converged=True, max_refine=0, fixed_iters=0):
    """min ||b - A x|| by sketch-and-precondition (Alg. 1) with LSQR (Alg. 2).
    d = 0 chooses d (sap_choose_d); fixed_iters as in sap_params."""
    torch = _torch()
    ctx = ctx or default_context()
    if mode is None:
        mode = SAP_MODE_FP64 if A.dtype == torch.float64 else SAP_MODE_MIXED_FP32
    prob = _problem(A, b)
    par = SapParams(d, zeta, seed, tol, maxiter, mode, max_refine, fixed_iters)
    x = x if x is not None else torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    info = SapInfo()
    st = lib().sap_solve(ctx.handle, ctypes.byref(prob), ctypes.byref(par), _dev(x, torch.float64, "x"),
                         ctypes.byref(info), _vp(_stream()))
    allow = (SAP_OK, SAP_NOT_CONVERGED) if allow_not_converged else (SAP_OK,)
    ctx.check(st, allow)
    return SolveResult(x, st, info.as_dict())


def sap_solve_hbm(A, b, d, zeta=8, seed=1, tol=1e-12, maxiter=500, mode=None, ctx=None, x=None, alpha=0.0,
                  beta=0.0, eta_scale=1.0, gradient_descent=False, fixed_iters=0):
    """Alg. 1 with heavy-ball momentum (App. D.3) in place of LSQR.  alpha <= 0
    takes the appendix's (alpha, beta) for eta = eta_scale sqrt(n/d)."""
    torch = _torch()
    ctx = ctx or default_context()
    if mode is None:
        mode = SAP_MODE_FP64 if A.dtype == torch.float64 else SAP_MODE_MIXED_FP32
    prob = _problem(A, b)
    par = SapParams(d, zeta, seed, tol, maxiter, mode, 0, fixed_iters)
    hb = SapHbmParams(float(alpha), float(beta), float(eta_scale), 1 if gradient_descent else 0, 0)
    x = x if x is not None else torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    info = SapInfo()
    st = lib().sap_solve_hbm(ctx.handle, ctypes.byref(prob), ctypes.byref(par), ctypes.byref(hb),
                             _dev(x, torch.float64, "x"), ctypes.byref(info), _vp(_stream()))
    ctx.check(st, (SAP_OK, SAP_NOT_CONVERGED))
    return SolveResult(x, st, info.as_dict())


def sap_solve_sstep(A, b, d, zeta=8, seed=1, tol=1e-12, maxiter=500, mode=None, ctx=None, x=None, s=8,
                    eta_scale=1.0, fixed_iters=0):
    """Alg. 1 with the s-step form (App. D.4.2) in place of LSQR: blocks of s
    steps on the Chebyshev basis for eta = eta_scale sqrt(n/d)."""
    torch = _torch()
    ctx = ctx or default_context()
    if mode is None:
        mode = SAP_MODE_FP64 if A.dtype == torch.float64 else SAP_MODE_MIXED_FP32
    prob = _problem(A, b)
    par = SapParams(d, zeta, seed, tol, maxiter, mode, 0, fixed_iters)
    ss = SapSstepParams(int(s), 0, float(eta_scale))
    x = x if x is not None else torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    info = SapInfo()
    st = lib().sap_solve_sstep(ctx.handle, ctypes.byref(prob), ctypes.byref(par), ctypes.byref(ss),
                               _dev(x, torch.float64, "x"), ctypes.byref(info), _vp(_stream()))
    ctx.check(st, (SAP_OK, SAP_NOT_CONVERGED))
    return SolveResult(x, st, info.as_dict())


def sap_lsqr(A, b, Rt, x0, tol=1e-12, maxiter=200, ctx=None, x=None):
    """Alg. 2 alone on A R^-1 from x0 (A in FP64, or FP32 storage with FP64 arithmetic)."""
    torch = _torch()
    ctx = ctx or default_context()
    prob = _problem(A, b)
    x = x if x is not None else torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    info = SapInfo()
    st = lib().sap_lsqr(ctx.handle, ctypes.byref(prob), _dev(Rt, torch.float64, "R"), _ld(Rt),
                        _dev(x0, torch.float64, "x0"), tol, maxiter, _dev(x, torch.float64, "x"),
                        ctypes.byref(info), _vp(_stream()))
    ctx.check(st, (SAP_OK, SAP_NOT_CONVERGED))
    return SolveResult(x, st, info.as_dict())


def sap_solve_batch(As, bs, ds, zetas=8, seeds=1, tol=1e-12, maxiter=200, ctx=None, xs=None, mode=0,
                    max_refine=0, fixed_iters=0):
    """Solve many independent problems together (sap_solve_batch).  As, bs:
    lists of device tensors (A row-major, F32 or F64; b F64).  Returns
    (xs, statuses, infos)."""
    torch = _torch()
    ctx = ctx or default_context()
    count = len(As)
    zetas = zetas if isinstance(zetas, (list, tuple)) else [zetas] * count
    seeds = seeds if isinstance(seeds, (list, tuple)) else [seeds] * count
    ds = ds if isinstance(ds, (list, tuple)) else [ds] * count
    probs = (SapProblem * count)(*[_problem(A, b) for A, b in zip(As, bs)])
    modes = mode if isinstance(mode, (list, tuple)) else [mode] * count
    pars = (SapParams * count)(*[SapParams(int(d), int(z), int(s), tol, maxiter, int(md), int(max_refine),
                                           int(fixed_iters))
                                 for d, z, s, md in zip(ds, zetas, seeds, modes)])
    xs = xs or [torch.empty(A.shape[1], dtype=torch.float64, device=A.device) for A in As]
    xptrs = (_vp * count)(*[_vp(_dev(xx, torch.float64, "x")) for xx in xs])
    infos = (SapInfo * count)()
    st = lib().sap_solve_batch(ctx.handle, count, probs, pars, xptrs, infos, _vp(_stream()))
    ctx.check(st, (SAP_OK, SAP_NOT_CONVERGED))
    return xs, st, [infos[k].as_dict() for k in range(count)]


# ---- served form ---------------------------------------------------------------
SERVE_STATS = ("submitted", "completed", "active", "queued", "rejected", "arena_used", "arena_size")
_inflight = {}  # (context handle, ticket) -> tensors the request reads or writes


def sap_serve_start(arena_bytes=0, max_active=1024, ctx=None):
    """Start the continuous-batching scheduler (optional; sap_submit starts it)."""
    ctx = ctx or default_context()
    ctx.check(lib().sap_serve_start(ctx.handle, int(arena_bytes), int(max_active)))


def sap_submit(A, b, d, zeta=8, seed=1, tol=1e-12, maxiter=200, ctx=None, x=None, mode=0, max_refine=0,
               fixed_iters=0):
    """Queue one problem (sap_submit).  Returns the ticket; the tensors stay
    referenced here until sap_poll reports a terminal status."""
    torch = _torch()
    ctx = ctx or default_context()
    x = x if x is not None else torch.empty(A.shape[1], dtype=torch.float64, device=A.device)
    prob = _problem(A, b)
    par = SapParams(int(d), int(zeta), int(seed), float(tol), int(maxiter), int(mode), int(max_refine),
                    int(fixed_iters))
    ticket = _u64(0)
    st = lib().sap_submit(ctx.handle, ctypes.byref(prob), ctypes.byref(par), _vp(_dev(x, torch.float64, "x")),
                          ctypes.byref(ticket), _vp(_stream()))
    ctx.check(st)
    _inflight[(ctx.handle.value, ticket.value)] = (A, b, x)
    return ticket.value


def sap_poll(ticket, wait=False, ctx=None):
    """State of a request: (status, info dict or None, x or None).  status is
    SAP_PENDING until the request finishes."""
    ctx = ctx or default_context()
    info = SapInfo()
    st = lib().sap_poll(ctx.handle, _u64(ticket), ctypes.byref(info), 1 if wait else 0)
    if st == SAP_PENDING:
        return st, None, None
    if st == SAP_EINVAL and (ctx.handle.value, ticket) not in _inflight:
        ctx.check(st)
    held = _inflight.pop((ctx.handle.value, ticket), None)
    return st, info.as_dict(), (held[2] if held else None)


def sap_cancel(ticket, ctx=None):
    ctx = ctx or default_context()
    ctx.check(lib().sap_cancel(ctx.handle, _u64(ticket)))


def sap_serve_stats(ctx=None):
    ctx = ctx or default_context()
    out = (_i64 * len(SERVE_STATS))()
    ctx.check(lib().sap_serve_stats(ctx.handle, out))
    return dict(zip(SERVE_STATS, list(out)))



def sap_embedding_dim(m, n, eps, cost_ratio=1.0):
    """d from eq. (4.2) (Sec. 4.3); host-only, no context or GPU needed."""
    d = _i32(0)
    st = lib().sap_embedding_dim(int(m), int(n), float(eps), float(cost_ratio), ctypes.byref(d))
    if st != SAP_OK:
        raise SapError(st, "sap_embedding_dim: invalid arguments")
    return d.value


def sap_choose_d(A, b, zeta=8, eps=1e-12, ctx=None):
    """Machine-aware embedding dimension for the problem (A, b) (sap_choose_d)."""
    ctx = ctx or default_context()
    d = _i32(0)
    prob = _problem(A, b)
    ctx.check(lib().sap_choose_d(ctx.handle, ctypes.byref(prob), int(zeta), float(eps), ctypes.byref(d),
                                 _vp(_stream())))
    return d.value


def sap_iteration_estimate(n, d, eps):
    """Iterations for the eq. (4.1) rate estimate to reach eps; host-only."""
    t = _i32(0)
    st = lib().sap_iteration_estimate(int(n), int(d), float(eps), ctypes.byref(t))
    if st != SAP_OK:
        raise SapError(st, "sap_iteration_estimate: invalid arguments")
    return t.value
