"""GPU parity of Alg. 1 with heavy-ball momentum (App. D.3) in place of LSQR,
through the C ABI, against the oracle's momentum iteration.

The GPU forms each step direction from the residual r = b - A x (one fused
pass); the oracle follows the appendix's v - M M^T A^T A x.  In the latter
the two terms cancel as x nears x*, leaving an error of about u kappa(A) ||b||
in A-norm (u the unit roundoff; measured 5e-10 ||b|| at kappa = 1e6, from
the second step on), which the residual form does not have.  Bars derived
from that: fixed-count iterates agree to ||A(x - x_or)|| <= 50 u kappa ||b||
and, for kappa <= 1e3, ||x - x_or|| <= 50 u kappa^2 ||x_or|| (the small
singular directions amplify the A-norm difference by up to kappa);
converged runs to 10 tol ||r*|| in A-norm.  Ill-conditioned accuracy is
checked against LAPACK's solution, which only the residual form reaches."""
import numpy as np
import pytest

import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sap():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03070_amd as sap
    sap.lib()
    return sap


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


U = 2.0 ** -53


@pytest.mark.parametrize("m,n,d,cond,T,gd", [
    (20000, 100, 400, 1e3, 15, False),
    (20000, 100, 400, 1e6, 15, False),
    (9000, 257, 1028, 1e2, 12, False),
    (30000, 40, 400, 1e3, 20, True),     # gradient descent (beta = 0)
    (12000, 1100, 4400, 1e3, 8, False),  # several waves across a row in the pass
])
def test_hbm_fixed_count_parity(sap, orc, m, n, d, cond, T, gd):
    import torch
    print(f"hbm fixed m={m} n={n} d={d} cond={cond:g} T={T} gd={gd}", flush=True)
    p = inputs.make_problem(m, n, kind="svd", cond=cond, noise=1e-6, seed=3 * m + n)
    a, b = orc.hbm_params(n, d, gd=gd)
    res = sap.sap_solve_hbm(_dev(p.A), _dev(p.b), d, 8, 21, tol=1e-12, fixed_iters=T, gradient_descent=gd)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK and res.info["iters"] == T
    x_or, io = orc.solve_hbm(p.A, p.b, d, 8, 21, a, b, tol=0.0, maxiter=T)
    x = res.x.cpu().numpy()
    assert io["iters"] == T
    assert np.linalg.norm(p.A @ (x - x_or)) <= 50 * U * cond * np.linalg.norm(p.b)
    if cond <= 1e3:
        assert np.linalg.norm(x - x_or) <= 50 * U * cond ** 2 * np.linalg.norm(x_or)
    assert res.info["resid_est"] == pytest.approx(io["resid_est"], rel=1e-9)


def test_hbm_converged_parity(sap, orc):
    """A tolerance both forms reach (kappa = 1e2): the same stopping step, to
    two, and solutions within 10 tol ||r*|| of each other in A-norm."""
    import torch
    m, n, d, tol = 40000, 150, 600, 1e-10
    p = inputs.make_problem(m, n, kind="svd", cond=1e2, noise=1e-3, seed=77)
    a, b = orc.hbm_params(n, d, c=np.sqrt(1.1))
    res = sap.sap_solve_hbm(_dev(p.A), _dev(p.b), d, 8, 4, tol=tol, maxiter=400, eta_scale=np.sqrt(1.1))
    torch.cuda.synchronize()
    x_or, io = orc.solve_hbm(p.A, p.b, d, 8, 4, a, b, tol=tol, maxiter=400)
    assert res.status == sap.SAP_OK and io["status"] == "ok", (res.info, io)
    xs = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    rs = np.linalg.norm(p.b - p.A @ xs)
    x = res.x.cpu().numpy()
    assert np.linalg.norm(p.A @ (x - x_or)) <= 10 * tol * rs
    assert abs(res.info["iters"] - io["iters"]) <= 2


def test_hbm_inconsistent_meets_lapack(sap, orc):
    """Residual-form steps reach the 1e-12 normal-equation test; the result
    matches LAPACK's least-squares solution and the GPU LSQR solve, taking no
    fewer steps than LSQR (optimal over the same Krylov space)."""
    import torch
    m, n, d = 20000, 100, 400
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-4, seed=5)
    A, bv = _dev(p.A), _dev(p.b)
    res = sap.sap_solve_hbm(A, bv, d, 8, 6, tol=1e-12, maxiter=500)
    lsq = sap.sap_solve(A, bv, d, 8, 6, tol=1e-12, maxiter=500)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK, res.info
    assert res.info["normar_est"] <= 1e-12 * res.info["resid_est"]
    xs = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    x = res.x.cpu().numpy()
    assert np.linalg.norm(p.A @ (x - xs)) <= 1e-12 * np.linalg.norm(p.b)
    assert np.linalg.norm(x - xs) <= 1e-8 * np.linalg.norm(xs)
    assert res.info["iters"] >= lsq.info["iters"] - 1


def test_hbm_fp32_storage_and_large_pass(sap, orc):
    """MIXED_FP32 (FP32 A, FP64 arithmetic) against the oracle on the rounded
    A, and an FP64 A over 512 MB (the pass's claimed row tail)."""
    import torch
    m, n, d, T = 30000, 200, 800, 10
    cond = 1e3
    p = inputs.make_problem(m, n, kind="svd", cond=cond, noise=1e-6, seed=8)
    A32 = p.A.astype(np.float32)
    a, b = orc.hbm_params(n, d)
    res = sap.sap_solve_hbm(_dev(A32), _dev(p.b), d, 8, 2, fixed_iters=T)
    torch.cuda.synchronize()
    A64 = A32.astype(np.float64)
    x_or, _ = orc.solve_hbm(A64, p.b, d, 8, 2, a, b, tol=0.0, maxiter=T)
    x = res.x.cpu().numpy()
    assert np.linalg.norm(A64 @ (x - x_or)) <= 50 * U * cond * np.linalg.norm(p.b)
    assert np.linalg.norm(x - x_or) <= 50 * U * cond ** 2 * np.linalg.norm(x_or)
    m, n, d, T = 1 << 18, 300, 1200, 6
    print(f"hbm large m={m} n={n}", flush=True)
    p = inputs.make_problem(m, n, kind="colscale", cond=1e3, noise=1e-6, seed=9)
    res = sap.sap_solve_hbm(_dev(p.A), _dev(p.b), d, 8, 3, fixed_iters=T)
    torch.cuda.synchronize()
    a, b = orc.hbm_params(n, d)
    x_or, _ = orc.solve_hbm(p.A, p.b, d, 8, 3, a, b, tol=0.0, maxiter=T)
    x = res.x.cpu().numpy()
    assert np.linalg.norm(p.A @ (x - x_or)) <= 50 * U * 1e3 * np.linalg.norm(p.b)


def test_hbm_argument_checks(sap):
    import torch
    A = torch.randn(4000, 50, dtype=torch.float64, device="cuda")
    b = torch.randn(4000, dtype=torch.float64, device="cuda")
    with pytest.raises(sap.SapError) as e:   # eta = 1.5 sqrt(50/100) > 1
        sap.sap_solve_hbm(A, b, 100, eta_scale=1.5)
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve_hbm(A, b, 200, alpha=0.5, beta=1.0)
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve_hbm(A, b, 200, mode=sap.SAP_MODE_MIXED_FP32_REFINE)
    assert e.value.status == sap.SAP_EINVAL
    r = sap.sap_solve_hbm(A, b, 200, alpha=0.5, beta=0.2, tol=1e-10, maxiter=400)
    torch.cuda.synchronize()
    assert r.status == sap.SAP_OK
