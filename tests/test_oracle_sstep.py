"""Pins for the oracle's s-step form (App. D.4.2) against facts fixed outside
it: the Chebyshev basis against numpy's Chebyshev polynomials evaluated on an
eigen-decomposition of Z, one block of s steps against s iterations of the
oracle's LSQR (Alg. 2, a separate code path: the closed form and LSQR give
the same CG iterate in exact arithmetic), the independence of the result from
the Chebyshev interval (it changes the basis, not the space), exactness once
the block spans the whole space, the CG bound of App. D per block, and the
least-squares solution from LAPACK."""
import numpy as np
import numpy.polynomial.chebyshev as cheb
import pytest

import inputs
import oracle as orc


def _problem(rng, m, n, spread=0.3):
    """A and an upper-triangular R with A R^-1 close to orthonormal: R is the
    triangular factor of a perturbed copy of A (the role the sketch's R plays)."""
    A = rng.standard_normal((m, n)) * np.logspace(0, -2, n)
    E = rng.standard_normal((m, n)) * np.logspace(0, -2, n) * spread / np.sqrt(m)
    R = np.linalg.qr(A + E, mode="r")
    R = R * np.sign(np.diag(R))[:, None]
    return A, R


def _z(A, R):
    B = np.linalg.solve(R.T, A.T).T          # B = A R^-1
    return B.T @ B


def _fitted(A, R, widen=0.05):
    """An interval around Z's spectrum, as the embedding bound supplies one:
    the basis is well conditioned only when the interval fits the spectrum
    (App. D.4.2 names the basis conditioning as the form's weak point)."""
    lam = np.linalg.eigvalsh(_z(A, R))
    return lam[0] * (1 - widen), lam[-1] * (1 + widen)


def test_interval_values():
    lo, hi = orc.sstep_interval(0.5)
    assert lo == 0.25 and hi == 2.25
    lo, hi = orc.sstep_interval(0.0)
    assert lo == 1.0 and hi == 1.0


@pytest.mark.parametrize("lo,hi", [(0.25, 2.25), (0.5, 1.7), (0.05, 4.0)])
def test_cheb_basis_matches_eigen(lo, hi):
    """u_k = T_k((Z - c I)/h) r0 with c, h the centre and half-width of
    [lo, hi]: evaluated independently as V T_k((lam - c)/h) V^T r0."""
    rng = np.random.default_rng(11)
    m, n, s = 90, 7, 6
    A, R = _problem(rng, m, n)
    r0 = rng.standard_normal(n)
    U, W = orc.cheb_basis(A, R, r0, s, lo, hi)
    Z = _z(A, R)
    lam, V = np.linalg.eigh(Z)
    c, h = (hi + lo) / 2, (hi - lo) / 2
    for k in range(s):
        tk = cheb.Chebyshev.basis(k)((lam - c) / h)
        uk = V @ (tk * (V.T @ r0))
        scale = np.linalg.norm(uk) + np.linalg.norm(r0)
        assert np.linalg.norm(U[:, k] - uk) <= 1e-11 * scale, k
        assert np.linalg.norm(W[:, k] - Z @ uk) <= 1e-11 * (np.linalg.norm(Z) * scale), k


@pytest.mark.parametrize("s", [1, 2, 3, 5, 8])
def test_block_equals_lsqr_steps(s):
    """One block of s steps from x0 is the CG iterate over x0 + M K_s(Z, r0),
    which s LSQR iterations from x0 also reach (Alg. 2, fixed count)."""
    rng = np.random.default_rng(20 + s)
    m, n = 150, 12
    A, R = _problem(rng, m, n, spread=4.0)
    b = rng.standard_normal(m)
    x0 = rng.standard_normal(n) * 0.1
    lo, hi = _fitted(A, R)
    xs, info = orc.sstep(A, b, R, x0, s, lo, hi, tol=0.0, maxiter=s)
    assert info["iters"] == s
    xl, _ = orc.lsqr(A, b, R, x0, tol=0.0, maxiter=s)
    assert np.linalg.norm(xs - xl) <= 1e-10 * np.linalg.norm(xl - x0)
    # and the A-norm error is no larger than the LSQR one (both optimal)
    x_star = np.linalg.lstsq(A, b, rcond=None)[0]
    ea = np.linalg.norm(A @ (x_star - xs))
    assert ea <= np.linalg.norm(A @ (x_star - xl)) * (1 + 1e-8) + 1e-14


def test_interval_changes_basis_not_result():
    """Different intervals give different bases of the same Krylov space, so
    the same block result."""
    rng = np.random.default_rng(31)
    m, n, s = 120, 10, 5
    A, R = _problem(rng, m, n, spread=4.0)
    b = rng.standard_normal(m)
    x0 = np.zeros(n)
    lo, hi = _fitted(A, R)
    outs = [orc.sstep(A, b, R, x0, s, a, c, tol=0.0, maxiter=s)[0]
            for a, c in ((lo, hi), (0.8 * lo, 1.2 * hi), (lo + 0.2 * (hi - lo), hi))]
    for x in outs[1:]:
        assert np.linalg.norm(x - outs[0]) <= 1e-9 * np.linalg.norm(outs[0])


@pytest.mark.parametrize("n,s", [(3, 8), (5, 5), (6, 16)])
def test_block_spanning_the_space_is_exact(n, s):
    """With s >= n the block's Krylov space is the whole space (the Gram
    system is truncated where it becomes singular), so one block lands on
    the least-squares solution from any x0."""
    rng = np.random.default_rng(40 + n)
    m = 50
    A, R = _problem(rng, m, n, spread=4.0)
    b = rng.standard_normal(m)
    x0 = rng.standard_normal(n)
    lo, hi = _fitted(A, R)
    x, info = orc.sstep(A, b, R, x0, s, lo, hi, tol=0.0, maxiter=s)
    x_star = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.all(np.isfinite(x))
    assert np.linalg.norm(A @ (x - x_star)) <= 1e-9 * np.linalg.norm(A @ (x0 - x_star))


def test_cg_bound_per_block():
    """Each block is s CG steps from the block's start, so the A-norm error
    drops at least by the Chebyshev factor 2 ((sqrt(k) - 1)/(sqrt(k) + 1))^s,
    k the condition number of Z (App. D, the CG bound)."""
    rng = np.random.default_rng(51)
    m, n, s = 400, 30, 4
    A, R = _problem(rng, m, n, spread=2.0)
    b = rng.standard_normal(m)
    x_star = np.linalg.lstsq(A, b, rcond=None)[0]
    lam = np.linalg.eigvalsh(_z(A, R))
    kap = lam[-1] / lam[0]
    rate = 2 * ((np.sqrt(kap) - 1) / (np.sqrt(kap) + 1)) ** s
    assert rate < 0.5  # the pin is meaningful
    x0 = np.zeros(n)
    lo, hi = orc.sstep_interval(0.6)
    _, info, hist = orc.sstep(A, b, R, x0, s, lo, hi, tol=0.0, maxiter=5 * s, history=True)
    assert info["iters"] == 5 * s and hist.shape[0] == 5
    prev = np.linalg.norm(A @ (x_star - x0))
    for k in range(hist.shape[0]):
        e = np.linalg.norm(A @ (x_star - hist[k]))
        assert e <= rate * prev * (1 + 1e-6) + 1e-13, k
        prev = e


def test_maxiter_rounds_up_to_whole_blocks():
    rng = np.random.default_rng(61)
    A, R = _problem(rng, 100, 8)
    b = rng.standard_normal(100)
    lo, hi = orc.sstep_interval(0.4)
    _, info = orc.sstep(A, b, R, np.zeros(8), 3, lo, hi, tol=0.0, maxiter=7)
    assert info["iters"] == 9 and not info["converged"]
    _, info = orc.sstep(A, b, R, np.zeros(8), 3, lo, hi, tol=0.0, maxiter=0)
    assert info["iters"] == 0


@pytest.mark.parametrize("s", [4, 8])
def test_solve_sstep_matches_lapack(s):
    """Alg. 1 with the s-step form: the sketch, QR and x0 of the LSQR solve,
    then blocks to tol 1e-10 (the true normal-equation residual this test
    measures has a rounding floor near u ||b||, here ~4e-11 ||r||, which LSQR's
    recurrence estimates do not see); the solution meets the least-squares
    perturbation bound against LAPACK and the step count is whole blocks."""
    m, n, d = 3000, 40, 160
    p = inputs.make_problem(m, n, kind="colscale", cond=1e6, noise=1e-6, seed=70 + s)
    eta = np.sqrt(n / d)
    lo, hi = orc.sstep_interval(eta)
    x, info = orc.solve_sstep(p.A, p.b, d, 8, 5, s, lo, hi, tol=1e-10, maxiter=400)
    assert info["status"] == "ok"
    assert info["iters"] % s == 0 and info["iters"] > 0
    x_ref = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    nb = np.linalg.norm(p.b)
    assert np.linalg.norm(p.A @ (x - x_ref)) <= 1e-10 * nb
    # the same sketch and x0 as the LSQR solve
    _, il = orc.solve(p.A, p.b, d, 8, 5, tol=1e-10, maxiter=400)
    assert np.array_equal(info["x0"], il["x0"])


def test_consistent_problem_stops_after_one_block():
    """b in the range of A: the sketch-and-solve x0 is already the solution to
    rounding, the block's Gram system is (numerically) empty and must not
    produce non-finite values; the test after it stops the solve."""
    m, n, d, s = 2000, 20, 80, 4
    rng = np.random.default_rng(81)
    A = rng.standard_normal((m, n))
    b = A @ rng.standard_normal(n)
    lo, hi = orc.sstep_interval(np.sqrt(n / d))
    x, info = orc.solve_sstep(A, b, d, 8, 3, s, lo, hi, tol=1e-12, maxiter=100)
    assert info["status"] == "ok" and info["iters"] == s
    assert np.all(np.isfinite(x))


def test_one_long_block_stalls_restarted_blocks_do_not():
    """One block over a long Krylov space (the closed form with t = 32) stops
    near 1e-11 relative: the Chebyshev basis on the embedding interval turns
    numerically dependent after ~16 steps and the Gram system is truncated.
    Blocks of 8 restarted from each block's residual reach the LSQR accuracy."""
    m, n, d = 3000, 40, 160
    p = inputs.make_problem(m, n, kind="colscale", cond=1e6, noise=1e-6, seed=74)
    xs = np.linalg.lstsq(p.A, p.b, rcond=None)[0]
    nb = np.linalg.norm(p.b)
    lo, hi = orc.sstep_interval(np.sqrt(n / d))
    x1, _ = orc.solve_sstep(p.A, p.b, d, 8, 5, 32, lo, hi, tol=0.0, maxiter=32)
    x8, _ = orc.solve_sstep(p.A, p.b, d, 8, 5, 8, lo, hi, tol=0.0, maxiter=48)
    e1 = np.linalg.norm(p.A @ (x1 - xs)) / nb
    e8 = np.linalg.norm(p.A @ (x8 - xs)) / nb
    assert 1e-13 < e1 < 1e-9
    assert e8 < 1e-13
