"""Pins for the oracle's heavy-ball momentum (App. D.3) against facts fixed
outside it: the closed form of the linear recurrence per eigen-direction,
the change of variables x = M y, the one-step exactness of gradient descent
on an exactly orthonormalised operator, the optimal rate sqrt(beta) the
appendix states, and the least-squares solution from LAPACK."""
import numpy as np
import pytest

import oracle as orc


def _orth(rng, m, n):
    Q, _ = np.linalg.qr(rng.standard_normal((m, n)))
    return Q


def test_hbm_params_values():
    a, b = orc.hbm_params(100, 400)          # eta = 1/2
    assert a == pytest.approx(0.5625, rel=1e-15) and b == pytest.approx(0.25, rel=1e-15)
    a, b = orc.hbm_params(100, 400, gd=True)
    assert a == pytest.approx(0.5625 / 1.25, rel=1e-15) and b == 0.0
    a, b = orc.hbm_params(100, 400, c=np.sqrt(1.1))
    assert b == pytest.approx(0.275, rel=1e-14)
    with pytest.raises(ValueError):
        orc.hbm_params(100, 100)             # eta = 1


@pytest.mark.parametrize("alpha,beta", [(0.55, 0.3), (0.9, 0.0), (0.3, 0.6)])
def test_hbm_matches_eigen_closed_form(alpha, beta):
    """R = I and A = Q diag(sigma): A^T A = diag(sigma^2), so each coordinate
    of e_t = x_t - x* follows e_t = (1 + beta - alpha l) e_{t-1} - beta e_{t-2}
    with e_{-1} = e_0; its closed form comes from the two roots of
    z^2 - (1 + beta - alpha l) z + beta."""
    rng = np.random.default_rng(1)
    m, n, T = 60, 5, 25
    sig = np.array([0.7, 0.85, 1.0, 1.2, 1.35])
    A = _orth(rng, m, n) * sig
    b = rng.standard_normal(m)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    x0 = rng.standard_normal(n)
    _, info, hist = orc.hbm(A, b, np.eye(n), x0, alpha, beta, tol=0.0, maxiter=T, history=True)
    assert info["iters"] == T and not info["converged"]
    lam = sig ** 2
    p = 1 + beta - alpha * lam
    disc = np.sqrt((p * p - 4 * beta).astype(complex))
    z1, z2 = (p + disc) / 2, (p - disc) / 2
    e0 = x0 - xs
    e1 = (1 - alpha * lam) * e0
    c1 = (e1 - z2 * e0) / (z1 - z2)
    c2 = e0 - c1
    for t in range(T + 1):
        et = (c1 * z1 ** t + c2 * z2 ** t).real
        assert np.allclose(hist[t] - xs, et, rtol=1e-9, atol=1e-12 * np.linalg.norm(e0)), t


def test_hbm_change_of_variables():
    """With B = A M, running on (A, M) from x0 = M y0 gives x_t = M y_t where
    y_t runs on (B, I): this fixes where M and M^T enter."""
    rng = np.random.default_rng(2)
    m, n, T = 80, 7, 15
    A = rng.standard_normal((m, n))
    R = np.triu(rng.uniform(-0.3, 0.3, (n, n)), 1) + np.diag(rng.uniform(1.0, 2.5, n))
    B = np.linalg.solve(R.T, A.T).T          # B = A R^-1
    b = rng.standard_normal(m)
    y0 = rng.standard_normal(n)
    x0 = np.linalg.solve(R, y0)
    alpha, beta = 0.02, 0.4
    _, _, hx = orc.hbm(A, b, R, x0, alpha, beta, tol=0.0, maxiter=T, history=True)
    _, _, hy = orc.hbm(B, b, np.eye(n), y0, alpha, beta, tol=0.0, maxiter=T, history=True)
    for t in range(T + 1):
        assert np.allclose(hx[t], np.linalg.solve(R, hy[t]), rtol=1e-10, atol=1e-12)


def test_gradient_step_exact_with_exact_factor():
    """R from the exact QR of A makes A M orthonormal: M M^T A^T (b - A x) =
    x* - x, so alpha = 1 lands on x* in one step from any x0, and the next
    step adds only the momentum term beta (x_1 - x_0)."""
    rng = np.random.default_rng(3)
    m, n = 40, 6
    A = rng.standard_normal((m, n)) * np.logspace(0, -3, n)
    b = rng.standard_normal(m)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    R = np.linalg.qr(A, mode="r")
    x0 = rng.standard_normal(n)
    beta = 0.37
    _, _, h = orc.hbm(A, b, R, x0, 1.0, beta, tol=0.0, maxiter=2, history=True)
    assert np.allclose(h[1], xs, rtol=1e-10, atol=1e-10 * np.linalg.norm(xs))
    assert np.allclose(h[2], xs + beta * (xs - x0), rtol=1e-9, atol=1e-9 * np.linalg.norm(xs))


def test_optimal_rate_is_sqrt_beta():
    """App. D.3: with the optimal pair for cond(AM) = (1 + eta)/(1 - eta), the
    error ||A(x* - x_t)|| shrinks like sqrt(beta) = eta per step (here with
    singular values of A M spread over the whole allowed range, so the two
    extreme modes carry a factor t); gradient descent is slower."""
    rng = np.random.default_rng(4)
    n, d = 8, 32                              # eta = 1/2
    eta = np.sqrt(n / d)
    # cond(AM) = (1 + eta)/(1 - eta): the range [1/(1+eta), 1/(1-eta)] of Sec. 2
    sig = np.linspace(1 / (1 + eta), 1 / (1 - eta), n)
    A = _orth(rng, 200, n) * sig
    b = rng.standard_normal(200)
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    x0 = xs + rng.standard_normal(n)

    def rate(gd):
        a, bb = orc.hbm_params(n, d, gd=gd)
        _, _, h = orc.hbm(A, b, np.eye(n), x0, a, bb, tol=0.0, maxiter=40, history=True)
        err = [np.linalg.norm(A @ (xs - x)) for x in h]
        return (err[35] / err[20]) ** (1 / 15)

    r_hb, r_gd = rate(False), rate(True)
    assert 0.45 <= r_hb <= 0.56, r_hb         # eta (1 + O(1/t)): the double root at the ends
    kappa2 = ((1 + eta) / (1 - eta)) ** 2     # cond of (AM)^T AM
    assert r_gd == pytest.approx((kappa2 - 1) / (kappa2 + 1), rel=0.03)


def test_hbm_solve_end_to_end():
    """Alg. 1 with momentum reaches the LAPACK solution.  On a consistent
    system the paper's form of the gradient, v - M M^T A^T A x, can meet a
    1e-12 residual test; on an inconsistent one its two terms cancel near
    x*, which floors ||M^T A^T r|| / ||r|| far above 1e-12 (so a looser test
    is used there, and LSQR, forming r itself, goes lower)."""
    rng = np.random.default_rng(5)
    m, n, d = 3000, 40, 160
    U = _orth(rng, m, n)
    A = (U * np.logspace(0, -4, n)) @ _orth(rng, n, n).T
    xt = rng.standard_normal(n)
    a, bb = orc.hbm_params(n, d, c=np.sqrt(1.1))
    b0 = A @ xt                                   # consistent
    x, info = orc.solve_hbm(A, b0, d, 8, 9, a, bb, tol=1e-12, maxiter=400)
    assert info["status"] == "ok" and info["resid_est"] <= 1e-12 * np.linalg.norm(b0)
    assert np.linalg.norm(x - xt) <= 1e-9 * np.linalg.norm(xt)
    b = b0 + 1e-6 * rng.standard_normal(m)         # inconsistent
    xs = np.linalg.lstsq(A, b, rcond=None)[0]
    x, info = orc.solve_hbm(A, b, d, 8, 9, a, bb, tol=1e-6, maxiter=400)
    assert info["status"] == "ok" and info["normar_est"] <= 1e-6 * info["resid_est"]
    assert np.linalg.norm(A @ (x - xs)) <= 1e-6 * np.linalg.norm(b - A @ xs)
    x_l, il = orc.solve(A, b, d, 8, 9, tol=1e-6, maxiter=400)
    # LSQR is optimal over the same Krylov space: momentum takes no fewer steps
    assert info["iters"] >= il["iters"] - 1
    # a cap below the needed count: not converged, the capped iterate returned
    x3, i3 = orc.solve_hbm(A, b, d, 8, 9, a, bb, tol=1e-12, maxiter=3)
    assert i3["status"] == "not_converged" and i3["iters"] == 3
    # the paper's form stalls on the inconsistent system at a 1e-12 test
    _, i4 = orc.solve_hbm(A, b, d, 8, 9, a, bb, tol=1e-12, maxiter=300)
    assert i4["status"] == "not_converged" and i4["normar_est"] > 1e-10 * i4["resid_est"]
