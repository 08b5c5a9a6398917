"""CPU oracle for sketch-and-precondition least squares with sparse sign sketches.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the product package.  The arithmetic is
in ``sap_oracle.c`` (plain C, double precision, single thread); this module only
marshals numpy arrays.  Function-by-function citations of the paper are in the
C file; the pins that tie each function to something other than itself are in
``tests/test_oracle_*.py``.

Parity unpinned (no external value exists to compare against):
  * the RNG stream layout (which Philox counter feeds which draw) is this
    project's own choice; it is pinned only through NumPy's Philox, the
    statistics of the generated sketch and self-consistency;
  * LSQR iteration counts depend on the stopping-rule reading;
  * mixed-precision iteration and refinement counts.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None

_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u64 = ctypes.c_uint64
_f64 = ctypes.c_double
_vp = ctypes.c_void_p


class LsqrInfo(ctypes.Structure):
    _fields_ = [("iters", _i32), ("converged", _i32), ("resid_est", _f64), ("normar_est", _f64)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", _i32), ("iters", _i32), ("resid_est", _f64), ("normar_est", _f64),
                ("t_generate", _f64), ("t_apply", _f64), ("t_qr", _f64), ("t_iterate", _f64)]


def lib():
    """Load (building on first use if needed) the compiled oracle."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(_build.SRC)):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.orc_philox4x64_10.argtypes = [_vp, _vp, _vp]
        L.orc_word.argtypes = [_u64] * 6
        L.orc_word.restype = _u64
        L.orc_sign_word.argtypes = [_u64] * 3
        L.orc_sign_word.restype = _u64
        L.orc_lemire_step.argtypes = [_u64, _u64, _vp]
        L.orc_lemire_step.restype = ctypes.c_int
        L.orc_bounded.argtypes = [_u64] * 6
        L.orc_bounded.restype = _u64
        L.orc_sketch_column.argtypes = [_u64, _u64, _u64, _i32, _i32, _vp, _vp]
        L.orc_sketch_column.restype = ctypes.c_int
        L.orc_sketch.argtypes = [_u64, _u64, _i64, _i32, _i32, _vp, _vp, _vp]
        L.orc_sketch.restype = ctypes.c_int
        L.orc_apply_sparse.argtypes = [_i64, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _i32, _f64,
                                       _vp, _i64, _vp, _i32]
        L.orc_apply_dense.argtypes = [_i64, _i32, _i32, _vp, _vp, _vp, _i64, _vp, _i32, _f64,
                                      _vp, _i64]
        L.orc_householder_qr.argtypes = [_vp, _i64, _i32, _i32, _vp]
        L.orc_backsub.argtypes = [_vp, _i64, _i32, _vp, _vp]
        L.orc_forwardsub_t.argtypes = [_vp, _i64, _i32, _vp, _vp]
        L.orc_matvec.argtypes = [_i64, _i32, _vp, _i64, _vp, _vp]
        L.orc_matvec_t.argtypes = [_i64, _i32, _vp, _i64, _vp, _vp]
        L.orc_lsqr.argtypes = [_i64, _i32, _vp, _i64, _vp, _vp, _i64, _vp, _f64, _i32, _vp, _vp,
                               ctypes.POINTER(LsqrInfo)]
        L.orc_rank_deficient.argtypes = [_vp, _i64, _i32, _i32]
        L.orc_rank_deficient.restype = ctypes.c_int
        L.orc_solve.argtypes = [_i64, _i32, _vp, _i64, _vp, _i32, _i32, _u64, _u64, _f64, _i32, _vp, _vp,
                                _vp, ctypes.POINTER(SolveInfo)]
        L.orc_direct_solve.argtypes = [_i64, _i32, _vp, _i64, _vp, _vp]
        L.orc_matvec_csr.argtypes = [_i64, _vp, _vp, _vp, _vp, _vp]
        L.orc_matvec_t_csr.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _vp]
        L.orc_apply_csr.argtypes = [_i64, _i32, _i32, _vp, _vp, _vp, _vp, _vp, _vp, _i32, _f64, _vp, _i64]
        L.orc_lsqr_csr.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _vp, _i64, _vp, _f64, _i32, _vp, _vp,
                                   ctypes.POINTER(LsqrInfo)]
        L.orc_solve_csr.argtypes = [_i64, _i32, _vp, _vp, _vp, _vp, _i32, _i32, _u64, _u64, _f64, _i32, _vp, _vp,
                                    _vp, ctypes.POINTER(SolveInfo)]
        L.orc_hbm_params.argtypes = [_i32, _i32, _f64, _i32, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]
        L.orc_hbm_params.restype = ctypes.c_int
        L.orc_hbm.argtypes = [_i64, _i32, _vp, _i64, _vp, _vp, _i64, _vp, _f64, _f64, _f64, _i32, _vp, _vp,
                              ctypes.POINTER(LsqrInfo)]
        L.orc_solve_hbm.argtypes = [_i64, _i32, _vp, _i64, _vp, _i32, _i32, _u64, _u64, _f64, _i32, _f64, _f64,
                                    _vp, _vp, ctypes.POINTER(SolveInfo)]
        L.orc_cheb_basis.argtypes = [_i64, _i32, _vp, _i64, _vp, _i64, _vp, _i32, _f64, _f64, _vp, _vp]
        L.orc_sstep.argtypes = [_i64, _i32, _vp, _i64, _vp, _vp, _i64, _vp, _i32, _f64, _f64, _f64, _i32, _vp,
                                _vp, ctypes.POINTER(LsqrInfo)]
        L.orc_sstep_interval.argtypes = [_f64, ctypes.POINTER(_f64), ctypes.POINTER(_f64)]
        L.orc_solve_sstep.argtypes = [_i64, _i32, _vp, _i64, _vp, _i32, _i32, _u64, _u64, _f64, _i32, _i32, _f64,
                                      _f64, _vp, _vp, ctypes.POINTER(SolveInfo)]
        L.orc_lambert_w0.argtypes = [_f64]
        L.orc_lambert_w0.restype = _f64
        L.orc_embedding_dim.argtypes = [_i64, _i32, _f64, _f64]
        L.orc_embedding_dim.restype = _f64
        L.orc_iteration_estimate.argtypes = [_i32, _i32, _f64]
        L.orc_iteration_estimate.restype = _f64
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_vp) if a is not None else None


def _f64c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------- RNG ----
def philox4x64_10(counter, key):
    """Philox4x64-10 block function (Salmon et al., SC'11)."""
    c = np.asarray(counter, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_p(c), _p(k), _p(out))
    return out


def word(seed, stream, i, r, j, k):
    return int(lib().orc_word(seed, stream, i, r, j, k))


def sign_word(seed, stream, i):
    return int(lib().orc_sign_word(seed, stream, i))


def lemire_step(w, d):
    """Return the bounded value for word w, or None when Lemire's test rejects."""
    out = np.zeros(1, dtype=np.uint64)
    ok = lib().orc_lemire_step(w, d, _p(out))
    return int(out[0]) if ok else None


def bounded(seed, stream, i, r, j, d):
    return int(lib().orc_bounded(seed, stream, i, r, j, d))


# ------------------------------------------------------------- sketch ----
def sketch_column(seed, stream, i, d, zeta):
    idx = np.zeros(zeta, dtype=np.int32)
    sign = np.zeros(1, dtype=np.uint64)
    rounds = lib().orc_sketch_column(seed, stream, i, d, zeta, _p(idx), _p(sign))
    if rounds < 0:
        raise ValueError("invalid sketch parameters")
    return idx, int(sign[0]), rounds


def sketch(seed, stream, m, d, zeta, want_rounds=False):
    """Sparse sign sketch: idx (m, zeta) int32 ascending rows, sign (m,) uint64."""
    idx = np.zeros((m, zeta), dtype=np.int32)
    sign = np.zeros(m, dtype=np.uint64)
    rounds = np.zeros(m, dtype=np.int32) if want_rounds else None
    rc = lib().orc_sketch(seed, stream, m, d, zeta, _p(idx), _p(sign), _p(rounds))
    if rc != 0:
        raise ValueError("invalid sketch parameters")
    return (idx, sign, rounds) if want_rounds else (idx, sign)


def sketch_scale(zeta):
    """h = 1/sqrt(zeta), the magnitude of every nonzero of S (Alg. 3 values)."""
    return 1.0 / np.sqrt(np.float64(zeta))


def sign_values(sign, zeta):
    """(m, zeta) array of +-1 from the sign words (bit k -> sorted position k)."""
    bits = (sign[:, None] >> np.arange(zeta, dtype=np.uint64)[None, :]) & np.uint64(1)
    return np.where(bits == 1, 1.0, -1.0)


def dense_sketch(idx, sign, d, zeta, scaled=True):
    """Explicit d x m matrix S (for tiny m only)."""
    m = idx.shape[0]
    S = np.zeros((d, m))
    vals = sign_values(sign, zeta) * (sketch_scale(zeta) if scaled else 1.0)
    for k in range(zeta):
        S[idx[:, k], np.arange(m)] = vals[:, k]
    return S


def apply_sparse(idx, sign, A, b, d, zeta, cols=None):
    """Y = S [A b] (column-major d x ncols as a numpy (d, ncols) array)."""
    A = _f64c(A)
    m, n = A.shape
    b = None if b is None else _f64c(b)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    sign = np.ascontiguousarray(sign, dtype=np.uint64)
    if cols is not None:
        cols = np.ascontiguousarray(cols, dtype=np.int32)
        ncols = len(cols)
    else:
        ncols = n + 1 if b is not None else n
    Y = np.zeros((ncols, d))  # row c of this array = column c of Y
    lib().orc_apply_sparse(m, d, zeta, _p(idx), _p(sign), _p(A), n, _p(b), n,
                           sketch_scale(zeta), _p(Y), d, _p(cols), ncols)
    return Y.T


def apply_dense(idx, sign, A, b, d, zeta):
    A = _f64c(A)
    m, n = A.shape
    b = None if b is None else _f64c(b)
    ncols = n + 1 if b is not None else n
    Y = np.zeros((ncols, d))
    lib().orc_apply_dense(m, d, zeta, _p(np.ascontiguousarray(idx, dtype=np.int32)),
                          _p(np.ascontiguousarray(sign, dtype=np.uint64)), _p(A), n, _p(b), n,
                          sketch_scale(zeta), _p(Y), d)
    return Y.T


# ------------------------------------------------------------------ QR ----
def householder_qr(Y):
    """In-place-style Householder QR of a (rows, cols) array.

    Returns (F, tau) where F is the factored matrix (R in the upper triangle,
    Householder vectors below) as a (rows, cols) array."""
    rows, cols = Y.shape
    F = np.asfortranarray(np.array(Y, dtype=np.float64))
    tau = np.zeros(cols)
    lib().orc_householder_qr(F.ctypes.data_as(_vp), rows, rows, cols, _p(tau))
    return F, tau


def r_factor(F, n):
    return np.triu(np.asarray(F)[:n, :n])


def q_factor(F, tau):
    """Explicit Q (rows x k) from the stored reflectors (for checks)."""
    rows, cols = F.shape
    k = min(rows, cols)
    Q = np.eye(rows)[:, :k].copy()
    for j in range(k - 1, -1, -1):
        v = np.zeros(rows)
        v[j] = 1.0
        v[j + 1:] = F[j + 1:, j]
        Q -= tau[j] * np.outer(v, v @ Q)
    return Q


def backsub(R, rhs):
    R = np.asfortranarray(R, dtype=np.float64)
    n = R.shape[0]
    x = np.zeros(n)
    lib().orc_backsub(R.ctypes.data_as(_vp), n, n, _p(_f64c(rhs)), _p(x))
    return x


def forwardsub_t(R, rhs):
    R = np.asfortranarray(R, dtype=np.float64)
    n = R.shape[0]
    y = np.zeros(n)
    lib().orc_forwardsub_t(R.ctypes.data_as(_vp), n, n, _p(_f64c(rhs)), _p(y))
    return y


def matvec(A, x):
    A = _f64c(A)
    y = np.zeros(A.shape[0])
    lib().orc_matvec(A.shape[0], A.shape[1], _p(A), A.shape[1], _p(_f64c(x)), _p(y))
    return y


def matvec_t(A, u):
    A = _f64c(A)
    y = np.zeros(A.shape[1])
    lib().orc_matvec_t(A.shape[0], A.shape[1], _p(A), A.shape[1], _p(_f64c(u)), _p(y))
    return y


# ---------------------------------------------------------------- LSQR ----
def lsqr(A, b, R, x0, tol=1e-12, maxiter=200, history=False):
    """Alg. 2 on A R^-1.  Returns (x, info dict[, iterates (t+1, n)])."""
    A = _f64c(A)
    m, n = A.shape
    R = np.asfortranarray(R, dtype=np.float64)
    x = np.zeros(n)
    hist = np.zeros((maxiter + 1, n)) if history else None
    info = LsqrInfo()
    lib().orc_lsqr(m, n, _p(A), n, _p(_f64c(b)), R.ctypes.data_as(_vp), R.shape[0],
                   _p(_f64c(x0)), tol, maxiter, _p(x), _p(hist), ctypes.byref(info))
    d = dict(iters=info.iters, converged=bool(info.converged), resid_est=info.resid_est,
             normar_est=info.normar_est)
    if history:
        return x, d, hist[:info.iters + 1]
    return x, d


def rank_deficient(R, d):
    R = np.asfortranarray(R, dtype=np.float64)
    return bool(lib().orc_rank_deficient(R.ctypes.data_as(_vp), R.shape[0], R.shape[0], d))


STATUS = {0: "ok", 1: "invalid", 3: "rank_deficient", 4: "not_converged"}


def solve(A, b, d, zeta, seed, tol=1e-12, maxiter=200, want_y=False, stream=0):
    """Alg. 1 end to end.  Returns (x, info dict) (+ factored Y if want_y)."""
    A = _f64c(A)
    m, n = A.shape
    x = np.zeros(n)
    x0 = np.zeros(n)
    Y = np.zeros((n + 1, d)) if want_y else None
    info = SolveInfo()
    lib().orc_solve(m, n, _p(A), n, _p(_f64c(b)), d, zeta, seed, stream, tol, maxiter, _p(x), _p(x0),
                    _p(Y), ctypes.byref(info))
    out = dict(status=STATUS.get(info.status, str(info.status)), iters=info.iters,
               resid_est=info.resid_est, normar_est=info.normar_est, x0=x0,
               t_generate=info.t_generate, t_apply=info.t_apply, t_qr=info.t_qr,
               t_iterate=info.t_iterate)
    if want_y:
        return x, out, Y.T
    return x, out


def direct_solve(A, b):
    """Householder QR of [A b] then back substitution (tiny inputs)."""
    A = _f64c(A)
    m, n = A.shape
    x = np.zeros(n)
    lib().orc_direct_solve(m, n, _p(A), n, _p(_f64c(b)), _p(x))
    return x


# ---------------------------------------------------------- sparse (CSR) ----
def _csr(A):
    """(m, n, indptr int64, indices int32, values float64) of a scipy CSR matrix
    (columns sorted within each row), or of a (indptr, indices, values, shape)
    tuple."""
    if isinstance(A, tuple):
        indptr, indices, values, shape = A
    else:
        A = A.tocsr()
        A.sort_indices()
        indptr, indices, values, shape = A.indptr, A.indices, A.data, A.shape
    return (int(shape[0]), int(shape[1]), np.ascontiguousarray(indptr, dtype=np.int64),
            np.ascontiguousarray(indices, dtype=np.int32), np.ascontiguousarray(values, dtype=np.float64))


def matvec_csr(A, x):
    m, n, ip, ix, v = _csr(A)
    y = np.zeros(m)
    lib().orc_matvec_csr(m, _p(ip), _p(ix), _p(v), _p(_f64c(x)), _p(y))
    return y


def matvec_t_csr(A, u):
    m, n, ip, ix, v = _csr(A)
    y = np.zeros(n)
    lib().orc_matvec_t_csr(m, n, _p(ip), _p(ix), _p(v), _p(_f64c(u)), _p(y))
    return y


def apply_csr(idx, sign, A, b, d, zeta):
    """Y = S [A b] for A in CSR form, as a (d, ncols) array."""
    m, n, ip, ix, v = _csr(A)
    b = None if b is None else _f64c(b)
    ncols = n + 1 if b is not None else n
    Y = np.zeros((ncols, d))
    lib().orc_apply_csr(m, d, zeta, _p(np.ascontiguousarray(idx, dtype=np.int32)),
                        _p(np.ascontiguousarray(sign, dtype=np.uint64)), _p(ip), _p(ix), _p(v), _p(b), n,
                        sketch_scale(zeta), _p(Y), d)
    return Y.T


def lsqr_csr(A, b, R, x0, tol=1e-12, maxiter=200, history=False):
    """Alg. 2 on A R^-1 with A in CSR form."""
    m, n, ip, ix, v = _csr(A)
    R = np.asfortranarray(R, dtype=np.float64)
    x = np.zeros(n)
    hist = np.zeros((maxiter + 1, n)) if history else None
    info = LsqrInfo()
    lib().orc_lsqr_csr(m, n, _p(ip), _p(ix), _p(v), _p(_f64c(b)), R.ctypes.data_as(_vp), R.shape[0],
                       _p(_f64c(x0)), tol, maxiter, _p(x), _p(hist), ctypes.byref(info))
    d = dict(iters=info.iters, converged=bool(info.converged), resid_est=info.resid_est,
             normar_est=info.normar_est)
    if history:
        return x, d, hist[:info.iters + 1]
    return x, d


def solve_csr(A, b, d, zeta, seed, tol=1e-12, maxiter=200, stream=0):
    """Alg. 1 end to end with A in CSR form.  Returns (x, info dict)."""
    m, n, ip, ix, v = _csr(A)
    x = np.zeros(n)
    x0 = np.zeros(n)
    info = SolveInfo()
    lib().orc_solve_csr(m, n, _p(ip), _p(ix), _p(v), _p(_f64c(b)), d, zeta, seed, stream, tol, maxiter, _p(x),
                        _p(x0), None, ctypes.byref(info))
    return x, dict(status=STATUS.get(info.status, str(info.status)), iters=info.iters,
                   resid_est=info.resid_est, normar_est=info.normar_est, x0=x0, t_generate=info.t_generate,
                   t_apply=info.t_apply, t_qr=info.t_qr, t_iterate=info.t_iterate)


# ------------------------------------------------- heavy-ball momentum ----
def hbm_params(n, d, c=1.0, gd=False):
    """(alpha, beta) of App. D.3 for eta = c sqrt(n/d): heavy ball, or gradient
    descent when gd."""
    a, b = _f64(0.0), _f64(0.0)
    if lib().orc_hbm_params(int(n), int(d), float(c), 1 if gd else 0, ctypes.byref(a), ctypes.byref(b)) != 0:
        raise ValueError("eta = c sqrt(n/d) must lie in [0, 1)")
    return a.value, b.value


def hbm(A, b, R, x0, alpha, beta, tol=1e-12, maxiter=200, history=False):
    """Heavy-ball momentum (App. D.3) on A with M = R^-1.  Returns (x, info
    dict[, iterates (t+1, n)])."""
    A = _f64c(A)
    m, n = A.shape
    R = np.asfortranarray(R, dtype=np.float64)
    x = np.zeros(n)
    hist = np.zeros((maxiter + 1, n)) if history else None
    info = LsqrInfo()
    lib().orc_hbm(m, n, _p(A), n, _p(_f64c(b)), R.ctypes.data_as(_vp), R.shape[0], _p(_f64c(x0)), alpha, beta,
                  tol, maxiter, _p(x), _p(hist), ctypes.byref(info))
    d = dict(iters=info.iters, converged=bool(info.converged), resid_est=info.resid_est,
             normar_est=info.normar_est)
    if history:
        return x, d, hist[:info.iters + 1]
    return x, d


def solve_hbm(A, b, d, zeta, seed, alpha, beta, tol=1e-12, maxiter=500, stream=0):
    """Alg. 1 with heavy-ball momentum in place of LSQR.  Returns (x, info dict)."""
    A = _f64c(A)
    m, n = A.shape
    x = np.zeros(n)
    x0 = np.zeros(n)
    info = SolveInfo()
    lib().orc_solve_hbm(m, n, _p(A), n, _p(_f64c(b)), d, zeta, seed, stream, tol, maxiter, alpha, beta, _p(x),
                        _p(x0), ctypes.byref(info))
    return x, dict(status=STATUS.get(info.status, str(info.status)), iters=info.iters,
                   resid_est=info.resid_est, normar_est=info.normar_est, x0=x0)


def sstep_interval(eta):
    """Chebyshev interval [(1 - eta)^2, (1 + eta)^2] of the s-step form for a
    distortion estimate eta (App. D.4.2 with the embedding bound)."""
    lo, hi = _f64(0.0), _f64(0.0)
    lib().orc_sstep_interval(float(eta), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def cheb_basis(A, R, r0, s, lo, hi):
    """Chebyshev basis u_0 .. u_{s-1} of K_s(Z, r0), Z = (A R^-1)^T (A R^-1),
    on [lo, hi], and W = Z U.  Returns (U, W), each n x s."""
    A = _f64c(A)
    m, n = A.shape
    R = np.asfortranarray(R, dtype=np.float64)
    U = np.zeros((s, n))
    W = np.zeros((s, n))
    lib().orc_cheb_basis(m, n, _p(A), n, R.ctypes.data_as(_vp), R.shape[0], _p(_f64c(r0)), int(s), float(lo),
                         float(hi), _p(U), _p(W))
    return U.T.copy(), W.T.copy()


def sstep(A, b, R, x0, s, lo, hi, tol=1e-12, maxiter=200, history=False):
    """The s-step form (App. D.4.2) on A with M = R^-1 from x0: blocks of s
    steps, each the CG iterate over its Krylov space in closed form.  Returns
    (x, info dict[, x after each block (blocks, n)])."""
    A = _f64c(A)
    m, n = A.shape
    R = np.asfortranarray(R, dtype=np.float64)
    x = np.zeros(n)
    nb = (max(maxiter, 0) + s - 1) // s
    hist = np.zeros((max(nb, 1), n)) if history else None
    info = LsqrInfo()
    lib().orc_sstep(m, n, _p(A), n, _p(_f64c(b)), R.ctypes.data_as(_vp), R.shape[0], _p(_f64c(x0)), int(s),
                    float(lo), float(hi), tol, int(maxiter), _p(x), _p(hist), ctypes.byref(info))
    d = dict(iters=info.iters, converged=bool(info.converged), resid_est=info.resid_est,
             normar_est=info.normar_est)
    if history:
        return x, d, hist[:info.iters // s]
    return x, d


def solve_sstep(A, b, d, zeta, seed, s, lo, hi, tol=1e-12, maxiter=500, stream=0):
    """Alg. 1 with the s-step form in place of LSQR.  Returns (x, info dict)."""
    A = _f64c(A)
    m, n = A.shape
    x = np.zeros(n)
    x0 = np.zeros(n)
    info = SolveInfo()
    lib().orc_solve_sstep(m, n, _p(A), n, _p(_f64c(b)), d, zeta, seed, stream, tol, maxiter, int(s), float(lo),
                          float(hi), _p(x), _p(x0), ctypes.byref(info))
    return x, dict(status=STATUS.get(info.status, str(info.status)), iters=info.iters,
                   resid_est=info.resid_est, normar_est=info.normar_est, x0=x0)


def lambert_w0(z):
    """Principal branch of the Lambert W function for z >= 0 (Sec. 4.3)."""
    return lib().orc_lambert_w0(float(z))


def embedding_dim(m, n, eps, cost_ratio=1.0):
    """Real d of eq. (4.2), iteration cost weighted by cost_ratio."""
    return lib().orc_embedding_dim(int(m), int(n), float(eps), float(cost_ratio))


def iteration_estimate(n, d, eps):
    """Real t with (n/d)^(t/2) = eps (eq. (4.1))."""
    return lib().orc_iteration_estimate(int(n), int(d), float(eps))
