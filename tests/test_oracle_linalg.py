"""Pins for the oracle's sketch apply, Householder QR, triangular solves and
preconditioned LSQR (Alg. 1, Alg. 2, Lemma 2.4, Prop. 2.7, App. A)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.linalg as sla
from scipy.sparse.linalg import LinearOperator, lsqr as scipy_lsqr

import inputs

EPS = np.finfo(float).eps


# ------------------------------------------------------------------ apply --
def test_apply_routes_agree(orc):
    p = inputs.make_problem(3000, 12, kind="svd", cond=1e3, seed=1)
    idx, sign = orc.sketch(9, 0, 3000, 60, 8)
    Ys = orc.apply_sparse(idx, sign, p.A, p.b, 60, 8)
    Yd = orc.apply_dense(idx, sign, p.A, p.b, 60, 8)
    S = orc.dense_sketch(idx, sign, 60, 8)
    Ynp = S @ np.column_stack([p.A, p.b])
    assert Ys.shape == (60, 13)
    scale = np.abs(Ynp).max()
    assert np.abs(Ys - Yd).max() <= 1e-13 * scale
    assert np.abs(Ys - Ynp).max() <= 1e-13 * scale


def test_apply_integer_exact(orc):
    """Integer A, b: the +-1 sums are exact integers; Y = h * sum must equal the
    correctly rounded product bit for bit."""
    m, n, d, zeta = 5000, 7, 50, 8
    p = inputs.make_problem(m, n, kind="integer", seed=3)
    idx, sign = orc.sketch(4, 0, m, d, zeta)
    Y = orc.apply_sparse(idx, sign, p.A, p.b, d, zeta)
    s = orc.sign_values(sign, zeta).astype(np.int64)
    Ab = np.column_stack([p.A, p.b]).astype(np.int64)
    exact = np.zeros((d, n + 1), dtype=np.int64)
    for k in range(zeta):
        np.add.at(exact, idx[:, k], s[:, k:k + 1] * Ab)
    assert (Y == exact.astype(np.float64) * orc.sketch_scale(zeta)).all()
    Yd = orc.apply_dense(idx, sign, p.A, p.b, d, zeta)
    assert (Yd == Y).all()


def test_apply_selected_columns(orc):
    p = inputs.make_problem(2000, 9, kind="colscale", cond=1e3, seed=2)
    idx, sign = orc.sketch(4, 0, 2000, 40, 8)
    Y = orc.apply_sparse(idx, sign, p.A, p.b, 40, 8)
    cols = [9, 0, 4]
    Yc = orc.apply_sparse(idx, sign, p.A, p.b, 40, 8, cols=cols)
    assert (Yc == Y[:, cols]).all()


def test_subspace_embedding_distortion(orc):
    """Def. 2.3: sigma(S U) lies in [1-eta, 1+eta].  For a dense, incoherent
    range the paper observes eta close to sqrt(n/d) (Sec. 4.2, eq. 4.1)."""
    m, n, d, zeta = 20000, 40, 400, 8
    p = inputs.make_problem(m, n, kind="svd", cond=1e4, seed=5)
    U, _ = np.linalg.qr(p.A)
    idx, sign = orc.sketch(6, 0, m, d, zeta)
    SU = orc.apply_sparse(idx, sign, U, None, d, zeta)
    sv = np.linalg.svd(SU, compute_uv=False)
    eta = max(sv.max() - 1, 1 - sv.min())
    assert 0.6 * np.sqrt(n / d) < eta < 1.5 * np.sqrt(n / d)


# --------------------------------------------------------------------- QR --
def test_qr_matches_lapack(orc):
    rng = np.random.default_rng(0)
    Y = rng.standard_normal((300, 41)) * np.logspace(0, -3, 41)
    F, tau = orc.householder_qr(Y)
    Fl, taul = sla.qr(Y, mode="raw")[0]
    R = np.triu(F[:41])
    Rl = np.triu(Fl[:41])
    kappa = np.linalg.cond(Y)
    assert np.abs(R - Rl).max() <= 100 * kappa * EPS * np.abs(Rl).max()
    assert np.abs(tau - taul).max() <= 1e-10
    Q = orc.q_factor(F, tau)
    assert np.linalg.norm(Q @ R - Y) <= 50 * 300 * EPS * np.linalg.norm(Y)
    assert np.abs(Q.T @ Q - np.eye(41)).max() <= 50 * 300 * EPS
    assert np.linalg.norm(R.T @ R - Y.T @ Y) <= 50 * 300 * EPS * np.linalg.norm(Y) ** 2


def test_qr_zero_column_and_wide(orc):
    Y = np.zeros((5, 3))
    Y[:, 1] = [1.0, 2.0, 2.0, 0.0, 0.0]
    F, tau = orc.householder_qr(Y)
    assert tau[0] == 0.0
    assert abs(abs(F[1, 1]) - 2.0) < 1e-15 or abs(abs(F[0, 1]) - 1.0) < 1e-15
    F2, tau2 = orc.householder_qr(np.arange(12.0).reshape(3, 4) + 1)
    assert F2.shape == (3, 4)


def test_qr_integer_exact_cholesky(orc):
    """R^T R = Y^T Y exactly in rationals: compare |R| with a rational Cholesky
    of Y^T Y (diagonal made positive)."""
    Y = np.array([[2, -1, 3], [1, 4, -2], [0, 1, 5], [3, 0, 1], [-1, 2, 2]], dtype=float)
    F, _ = orc.householder_qr(Y)
    R = np.triu(F[:3])
    R = R * np.sign(np.diag(R))[:, None]
    G = [[sum(Fraction(int(Y[k, i])) * Fraction(int(Y[k, j])) for k in range(5)) for j in range(3)]
         for i in range(3)]
    # rational LDL^T gives R_ij^2-free quantities: check squares of the diagonal
    # and the products R_ii R_ij exactly
    L = [[Fraction(0)] * 3 for _ in range(3)]
    D = [Fraction(0)] * 3
    for j in range(3):
        D[j] = G[j][j] - sum(L[j][k] ** 2 * D[k] for k in range(j))
        for i in range(j + 1, 3):
            L[i][j] = (G[i][j] - sum(L[i][k] * L[j][k] * D[k] for k in range(j))) / D[j]
    for j in range(3):
        assert abs(R[j, j] ** 2 - float(D[j])) <= 1e-13 * float(D[j])
        for i in range(j + 1, 3):
            # R_ji = L_ij * R_jj
            assert abs(R[j, i] - float(L[i][j]) * R[j, j]) <= 1e-13 * abs(R[j, j]) * 10


def test_triangular_solves(orc):
    rng = np.random.default_rng(1)
    n = 60
    R = np.triu(rng.standard_normal((n, n))) + 5 * np.eye(n)
    v = rng.standard_normal(n)
    x = orc.backsub(R, v)
    assert np.allclose(x, sla.solve_triangular(R, v, lower=False), rtol=1e-13, atol=1e-13)
    y = orc.forwardsub_t(R, v)
    assert np.allclose(y, sla.solve_triangular(R, v, trans="T", lower=False), rtol=1e-13, atol=1e-13)
    # brute force on a 3x3: substitute back
    R3 = np.array([[2.0, 1.0, -1.0], [0.0, 3.0, 0.5], [0.0, 0.0, 4.0]])
    x3 = orc.backsub(R3, [1.0, 2.0, 3.0])
    assert np.allclose(R3 @ x3, [1.0, 2.0, 3.0], rtol=0, atol=1e-15)
    y3 = orc.forwardsub_t(R3, [1.0, 2.0, 3.0])
    assert np.allclose(R3.T @ y3, [1.0, 2.0, 3.0], rtol=0, atol=1e-15)


def test_matvecs(orc):
    rng = np.random.default_rng(2)
    A = rng.standard_normal((50, 7))
    x = rng.standard_normal(7)
    u = rng.standard_normal(50)
    assert np.allclose(orc.matvec(A, x), A @ x, rtol=1e-14, atol=1e-14)
    assert np.allclose(orc.matvec_t(A, u), A.T @ u, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------------- LSQR --
def _sketched(orc, p, d, zeta, seed):
    m, n = p.A.shape
    idx, sign = orc.sketch(seed, 0, m, d, zeta)
    Y = orc.apply_sparse(idx, sign, p.A, p.b, d, zeta)
    F, tau = orc.householder_qr(Y)
    R = np.triu(F[:n, :n])
    z = F[:n, n]
    return Y, R, z


def test_x0_is_sketch_and_solve(orc):
    """x0 = M Q^T S b (Alg. 1) is the minimiser of ||Sb - SAx||."""
    p = inputs.make_problem(4000, 20, kind="svd", cond=1e5, noise=1e-3, seed=7)
    Y, R, z = _sketched(orc, p, 80, 8, 3)
    x0 = orc.backsub(R, z)
    ref = np.linalg.lstsq(Y[:, :20], Y[:, 20], rcond=None)[0]
    assert np.linalg.norm(p.A @ (x0 - ref)) <= 1e-9 * np.linalg.norm(p.b)


def test_lsqr_iterates_match_scipy(orc):
    """Alg. 2 on A M equals SciPy's LSQR on the LinearOperator A R^-1 (an
    independent implementation) iterate by iterate, mapped back by x = M y."""
    p = inputs.make_problem(3000, 25, kind="svd", cond=1e6, noise=1e-4, seed=8)
    _, R, z = _sketched(orc, p, 100, 8, 5)
    x0 = orc.backsub(R, z)
    x, info, hist = orc.lsqr(p.A, p.b, R, x0, tol=0.0, maxiter=12, history=True)
    A = p.A
    op = LinearOperator((3000, 25), matvec=lambda y: A @ sla.solve_triangular(R, y),
                        rmatvec=lambda u: sla.solve_triangular(R, A.T @ u, trans="T"))
    y0 = R @ x0
    for t in (1, 2, 3, 5, 8, 12):
        y = scipy_lsqr(op, p.b, x0=y0, atol=0, btol=0, conlim=0, iter_lim=t)[0]
        xs = sla.solve_triangular(R, y)
        assert np.linalg.norm(A @ (hist[t] - xs)) <= 1e-9 * np.linalg.norm(p.b), t


def test_lsqr_estimates_and_bounds(orc):
    """Paige-Saunders estimates equal the true residual norms; Prop. 2.7's
    contraction and Lemma 2.4's condition bound hold."""
    m, n, d = 6000, 30, 120
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-2, seed=9)
    _, R, z = _sketched(orc, p, d, 8, 11)
    x0 = orc.backsub(R, z)
    xstar = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    x, info, hist = orc.lsqr(p.A, p.b, R, x0, tol=0.0, maxiter=15, history=True)
    AM = p.A @ np.linalg.inv(R)
    sv = np.linalg.svd(AM, compute_uv=False)
    kappa = sv[0] / sv[-1]
    # Lemma 2.4 with the distortion of S on range([A b]) ... on range(A)
    U, _ = np.linalg.qr(p.A)
    idx, sign = orc.sketch(11, 0, m, d, 8)
    svs = np.linalg.svd(orc.apply_sparse(idx, sign, U, None, d, 8), compute_uv=False)
    eta = max(svs.max() - 1, 1 - svs.min())
    assert kappa <= (1 + eta) / (1 - eta) * (1 + 1e-10)
    e0 = np.linalg.norm(p.A @ (xstar - x0))
    for t in range(1, 16):
        et = np.linalg.norm(p.A @ (xstar - hist[t]))
        assert et <= 2 * ((kappa - 1) / (kappa + 1)) ** t * e0 * (1 + 1e-6) + 1e-12 * np.linalg.norm(p.b)
    # estimates after t iterations (t small, so the quantities are far above
    # the rounding floor and a wrong sign or index in the recurrences shows)
    for t in (1, 2, 4, 6):
        xt, it = orc.lsqr(p.A, p.b, R, x0, tol=0.0, maxiter=t)
        r = p.b - p.A @ xt
        assert abs(it["resid_est"] - np.linalg.norm(r)) <= 1e-9 * np.linalg.norm(r)
        normar = np.linalg.norm(sla.solve_triangular(R, p.A.T @ r, trans="T"))
        assert abs(it["normar_est"] - normar) <= 1e-6 * normar, t


def test_x0_bound_appendix_a(orc):
    """App. A.2: ||b - A x0|| <= (1+eta)/(1-eta) ||b - A x*|| with eta the
    distortion of S on range([A b])."""
    m, n, d = 6000, 30, 150
    p = inputs.make_problem(m, n, kind="svd", cond=1e3, noise=1e-1, seed=10)
    _, R, z = _sketched(orc, p, d, 8, 12)
    x0 = orc.backsub(R, z)
    U, _ = np.linalg.qr(np.column_stack([p.A, p.b]))
    idx, sign = orc.sketch(12, 0, m, d, 8)
    svs = np.linalg.svd(orc.apply_sparse(idx, sign, U, None, d, 8), compute_uv=False)
    eta = max(svs.max() - 1, 1 - svs.min())
    xstar = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    rstar = np.linalg.norm(p.b - p.A @ xstar)
    assert np.linalg.norm(p.b - p.A @ x0) <= (1 + eta) / (1 - eta) * rstar * (1 + 1e-12)
    # App. A.3: ||A(x* - x)||^2 = ||b - Ax||^2 - ||b - Ax*||^2
    lhs = np.linalg.norm(p.A @ (xstar - x0)) ** 2
    rhs = np.linalg.norm(p.b - p.A @ x0) ** 2 - rstar ** 2
    assert abs(lhs - rhs) <= 1e-8 * rstar ** 2


def test_compatible_system_recovers_x(orc):
    p = inputs.make_problem(5000, 20, kind="svd", cond=1e4, noise=0.0, seed=13)
    x, info = orc.solve(p.A, p.b, 80, 8, 21, tol=1e-14, maxiter=100)
    assert info["status"] == "ok"
    assert np.linalg.norm(x - p.x_true) <= 1e4 * 1e-13 * np.linalg.norm(p.x_true)


def test_solve_matches_direct(orc):
    """Alg. 1 end to end vs two direct solvers (LAPACK lstsq and the oracle's
    Householder solve of [A b]) at the paper's metric ||A(x - x_d)|| / ||b||."""
    p = inputs.make_problem(8000, 40, kind="svd", cond=1e6, noise=1e-6, seed=14)
    x, info = orc.solve(p.A, p.b, 160, 8, 22, tol=1e-12, maxiter=200)
    assert info["status"] == "ok" and 5 < info["iters"] < 80
    xd = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    xh = orc.direct_solve(p.A, p.b)
    nb = np.linalg.norm(p.b)
    assert np.linalg.norm(p.A @ (x - xd)) <= 1e-12 * nb
    assert np.linalg.norm(p.A @ (xh - xd)) <= 1e-12 * nb


def test_direct_solve_mpmath_tiny(orc):
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 50
    p = inputs.make_problem(60, 5, kind="svd", cond=1e3, noise=1e-2, seed=15)
    A = mpmath.matrix(p.A.tolist())
    b = mpmath.matrix(p.b.tolist())
    xs = mpmath.lu_solve(A.T * A, A.T * b)
    xs = np.array([float(v) for v in xs])
    xh = orc.direct_solve(p.A, p.b)
    assert np.linalg.norm(xh - xs) <= 1e-12 * np.linalg.norm(xs)
    x, info = orc.solve(p.A, p.b, 24, 8, 3, tol=1e-14, maxiter=100)
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_rank_deficient_flag(orc):
    p = inputs.make_problem(3000, 10, kind="svd", cond=1e2, seed=16)
    A = p.A.copy()
    A[:, 7] = A[:, 2]
    x, info = orc.solve(A, p.b, 40, 8, 1)
    assert info["status"] == "rank_deficient"
    x, info = orc.solve(p.A, p.b, 40, 8, 1, maxiter=1)
    assert info["status"] == "not_converged"
    x, info = orc.solve(p.A, p.b, 10, 8, 1)
    assert info["status"] == "invalid"


def test_identity_hard_case(orc):
    """First n columns of the identity (Sec. 4.1's hard case): S A is just the
    first n columns of S, so columns of Y have exactly zeta nonzeros of size h."""
    m, n, d, zeta = 5000, 20, 80, 4
    p = inputs.make_problem(m, n, kind="identity", seed=0)
    idx, sign = orc.sketch(2, 0, m, d, zeta)
    Y = orc.apply_sparse(idx, sign, p.A, None, d, zeta)
    assert ((Y != 0).sum(axis=0) == zeta).all()
    assert np.allclose(np.abs(Y[Y != 0]), orc.sketch_scale(zeta), rtol=0, atol=0)
