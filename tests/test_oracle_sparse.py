"""Pins of the oracle's CSR routes (sparse A, Sec. 3 / Table 1's sparse
problems) against its dense routes, which the other pins tie to the paper
and to independent libraries.  Every CSR sum runs in the order of the dense
route and only skips zeros, so the results must agree bit for bit; SciPy's
own sparse products pin the CSR layout itself."""
import numpy as np
import pytest

import inputs


@pytest.fixture(scope="module", params=["sign", "gauss"])
def case(request):
    A, b, _ = inputs.make_sparse_problem(3000, 40, density=0.05, values=request.param, noise=1e-3, seed=12)
    return A, b


def test_csr_products_match_dense_bitwise(orc, case):
    A, b = case
    Ad = A.toarray()
    rng = np.random.default_rng(3)
    x = rng.standard_normal(A.shape[1])
    u = rng.standard_normal(A.shape[0])
    assert np.array_equal(orc.matvec_csr(A, x), orc.matvec(Ad, x))
    assert np.array_equal(orc.matvec_t_csr(A, u), orc.matvec_t(Ad, u))
    # the layout against SciPy's products (rounding order may differ)
    assert np.allclose(orc.matvec_csr(A, x), A @ x, rtol=1e-13, atol=1e-13)
    assert np.allclose(orc.matvec_t_csr(A, u), A.T @ u, rtol=1e-13, atol=1e-12)


def test_csr_apply_matches_dense_bitwise(orc, case):
    A, b = case
    Ad = A.toarray()
    d, zeta = 160, 8
    idx, sign = orc.sketch(5, 0, A.shape[0], d, zeta)
    for bb in (b, None):
        Yc = orc.apply_csr(idx, sign, A, bb, d, zeta)
        Yd = orc.apply_sparse(idx, sign, Ad, bb, d, zeta)
        assert np.array_equal(Yc, Yd)
    # against the explicit d x m sketch times [A b] (NumPy)
    S = orc.dense_sketch(idx, sign, d, zeta)
    Y = S @ np.column_stack([Ad, b])
    assert np.allclose(orc.apply_csr(idx, sign, A, b, d, zeta), Y, rtol=1e-13, atol=1e-12)


def test_csr_lsqr_and_solve_match_dense_bitwise(orc, case):
    A, b = case
    Ad = A.toarray()
    m, n = A.shape
    d, zeta = 4 * n, 8
    idx, sign = orc.sketch(9, 0, m, d, zeta)
    F, _ = orc.householder_qr(orc.apply_csr(idx, sign, A, b, d, zeta))
    R = np.triu(F[:n, :n])
    x0 = orc.backsub(R, F[:n, n])
    xc, ic, hc = orc.lsqr_csr(A, b, R, x0, tol=1e-12, maxiter=100, history=True)
    xd, idd, hd = orc.lsqr(Ad, b, R, x0, tol=1e-12, maxiter=100, history=True)
    assert ic == idd and np.array_equal(hc, hd) and np.array_equal(xc, xd)
    xs_c, sc = orc.solve_csr(A, b, d, zeta, 7, tol=1e-12, maxiter=200)
    xs_d, sd = orc.solve(Ad, b, d, zeta, 7, tol=1e-12, maxiter=200)
    assert sc["status"] == sd["status"] == "ok" and sc["iters"] == sd["iters"]
    assert np.array_equal(xs_c, xs_d)
    # and the least-squares solution itself (LAPACK)
    x_ls = np.linalg.lstsq(Ad, b, rcond=None)[0]
    assert np.linalg.norm(xs_c - x_ls) <= 1e-10 * np.linalg.norm(x_ls)
