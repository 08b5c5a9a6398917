"""GPU parity of LSQR (Alg. 2) and the whole of Alg. 1 through the C ABI.

Bars: the paper's accuracy metric ||A(x - x_or)|| / ||b|| <= 1e-12 in FP64
(Thm. 2.1 measures error as ||A(x* - x)||), and the forward error
||x - x_or|| / ||x_or|| <= 1e-8 where the least-squares perturbation bound
kappa*u + kappa^2*u*||r||/(||A|| ||x||) lies below it.
"""
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


def _note(msg):
    print(msg, flush=True)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


LSQR_CASES = [
    # m, n, d, cond, noise
    (20000, 100, 400, 1e6, 1e-8),
    (9000, 257, 1028, 1e8, 1e-6),
    (3000, 7, 28, 1e3, 1e-2),
    (50000, 520, 2080, 1e6, 1e-4),
]


@pytest.mark.parametrize("m,n,d,cond,noise", LSQR_CASES)
def test_lsqr_parity(sap, orc, m, n, d, cond, noise):
    """Same R and x0 on both sides: the GPU's one-pass reorganisation of the
    iteration (App. D.4.1) must track Alg. 2."""
    import torch
    _note(f"lsqr m={m} n={n} d={d} cond={cond:g}")
    p = inputs.make_problem(m, n, kind="svd", cond=cond, noise=noise, seed=m + n)
    idx, sign = orc.sketch(5, 0, m, d, 8)
    Y = orc.apply_sparse(idx, sign, p.A, p.b, d, 8)
    F, _ = orc.householder_qr(Y)
    R = np.triu(F[:n, :n])
    x0 = orc.backsub(R, F[:n, n])
    x_or, info_or = orc.lsqr(p.A, p.b, R, x0, tol=1e-12, maxiter=300)
    Rt = _dev(np.ascontiguousarray(F[:n, :n].T))
    res = sap.sap_lsqr(_dev(p.A), _dev(p.b), Rt, _dev(x0), tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    x = res.x.cpu().numpy()
    nb = np.linalg.norm(p.b)
    assert res.status == sap.SAP_OK and info_or["converged"]
    assert np.linalg.norm(p.A @ (x - x_or)) <= 1e-12 * nb
    assert abs(res.info["iters"] - info_or["iters"]) <= 2


@pytest.mark.parametrize("m,n,d,cond,noise", [(20000, 100, 400, 1e6, 1e-8), (30000, 300, 1200, 1e4, 1e-4)])
def test_lsqr_fp32_storage_parity(sap, orc, m, n, d, cond, noise):
    """sap_lsqr with A stored in FP32 computes in FP64: the oracle on the
    FP32-rounded A (exact in FP64) is the reference, at the FP64 bar."""
    import torch
    _note(f"lsqr-f32 m={m} n={n} d={d}")
    p = inputs.make_problem(m, n, kind="svd", cond=cond, noise=noise, seed=m + 3 * n, dtype=np.float32)
    A64 = p.A.astype(np.float64)
    idx, sign = orc.sketch(9, 0, m, d, 8)
    Y = orc.apply_sparse(idx, sign, A64, p.b, d, 8)
    F, _ = orc.householder_qr(Y)
    R = np.triu(F[:n, :n])
    x0 = orc.backsub(R, F[:n, n])
    x_or, info_or = orc.lsqr(A64, p.b, R, x0, tol=1e-12, maxiter=300)
    res = sap.sap_lsqr(_dev(p.A), _dev(p.b), _dev(np.ascontiguousarray(F[:n, :n].T)), _dev(x0), tol=1e-12,
                       maxiter=300)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK and info_or["converged"]
    assert np.linalg.norm(A64 @ (res.x.cpu().numpy() - x_or)) <= 1e-12 * np.linalg.norm(p.b)


def test_lsqr_wide_inverse_parity(sap, orc):
    """n = 4100: the explicit inverse M = R^-1 is built two columns per
    workgroup (the LDS holds no more at this width), as for the 2^22 x 4096
    workload.  R comes from LAPACK's QR of an oracle sketch of A (d = 2n);
    it is an input here, the same on both sides, and the iterations of the
    GPU (explicit inverse) and of the oracle (triangular solves, Alg. 2) are
    compared at the FP64 bar."""
    import torch
    m, n, d = 16384, 4100, 8200
    _note(f"lsqr wide inverse m={m} n={n} d={d}")
    p = inputs.make_problem(m, n, kind="colscale", cond=1e4, noise=1e-6, seed=4100)
    idx, sign = orc.sketch(11, 0, m, d, 8)
    Y = orc.apply_sparse(idx, sign, p.A, None, d, 8)
    R = np.linalg.qr(Y, mode="r")
    x0 = np.zeros(n)
    x_or, info_or = orc.lsqr(p.A, p.b, R, x0, tol=1e-12, maxiter=400)
    res = sap.sap_lsqr(_dev(p.A), _dev(p.b), _dev(np.ascontiguousarray(R.T)), _dev(x0), tol=1e-12, maxiter=400)
    torch.cuda.synchronize()
    x = res.x.cpu().numpy()
    assert res.status == sap.SAP_OK and info_or["converged"], res.info
    _note(f"  iterations {res.info['iters']} (oracle {info_or['iters']}), "
          f"forward {np.linalg.norm(x - x_or) / np.linalg.norm(x_or):.2e}")
    assert np.linalg.norm(p.A @ (x - x_or)) <= 1e-12 * np.linalg.norm(p.b)
    assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or)
    assert abs(res.info["iters"] - info_or["iters"]) <= 2


def test_lsqr_maxiter_and_zero(sap, orc):
    import torch
    p = inputs.make_problem(4000, 20, kind="svd", cond=1e4, noise=1e-3, seed=1)
    idx, sign = orc.sketch(5, 0, 4000, 80, 8)
    F, _ = orc.householder_qr(orc.apply_sparse(idx, sign, p.A, p.b, 80, 8))
    R = np.triu(F[:20, :20])
    x0 = orc.backsub(R, F[:20, 20])
    Rt = _dev(np.ascontiguousarray(F[:20, :20].T))
    for t in (0, 1, 3):
        _note(f"lsqr maxiter={t}")
        res = sap.sap_lsqr(_dev(p.A), _dev(p.b), Rt, _dev(x0), tol=1e-14, maxiter=t)
        torch.cuda.synchronize()
        xo, io = orc.lsqr(p.A, p.b, R, x0, tol=0.0, maxiter=t)
        assert res.status == sap.SAP_NOT_CONVERGED
        assert res.info["iters"] == t
        assert np.linalg.norm(p.A @ (res.x.cpu().numpy() - xo)) <= 1e-12 * np.linalg.norm(p.b)
    # b = 0: beta_1 = 0, x0 = 0 is exact
    res = sap.sap_lsqr(_dev(p.A), _dev(np.zeros(4000)), Rt, _dev(np.zeros(20)), tol=1e-12, maxiter=10)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK and np.all(res.x.cpu().numpy() == 0)


SOLVE_CASES = [
    # name, m, n, d, zeta, kind, cond, noise, row_scale
    ("config0", 20000, 100, 400, 8, "svd", 1e6, 1e-8, False),
    ("lev", 30000, 200, 800, 8, "svd", 1e8, 1e-10, True),
    ("colscale", 40000, 300, 1200, 12, "colscale", 1e6, 1e-8, False),
    ("wide-d", 12000, 50, 3000, 4, "svd", 1e3, 1e-4, False),
    ("tiny", 40, 3, 12, 2, "svd", 10.0, 1e-3, False),
    ("sparse", 50000, 120, 480, 8, "sparse_sign", 1.0, 1e-2, False),
    ("odd-n", 25000, 333, 1337, 8, "svd", 1e5, 1e-6, False),
    # degenerate shapes the method allows: the smallest problem (m = 2, n = 1,
    # d = 2, one nonzero per column), the smallest sketch (d = n + 1, slow
    # rate sqrt(n/d) ~ 1), and a dense sign sketch (zeta = d: every column of
    # S holds every row, generation needs the most redraw rounds)
    ("min-m", 2, 1, 2, 1, "svd", 10.0, 1e-3, False),
    ("d-eq-n-plus-1", 5000, 40, 41, 8, "svd", 10.0, 1e-3, False),
    ("zeta-eq-d", 3000, 10, 16, 16, "colscale", 10.0, 1e-3, False),
]


@pytest.mark.parametrize("name,m,n,d,zeta,kind,cond,noise,row_scale", SOLVE_CASES)
def test_solve_parity(sap, orc, name, m, n, d, zeta, kind, cond, noise, row_scale):
    import torch
    _note(f"solve {name} m={m} n={n} d={d} zeta={zeta}")
    if name == "config0":
        p = inputs.config0()
        seed = p.meta["sketch_seed"]
    else:
        p = inputs.make_problem(m, n, kind=kind, cond=cond, noise=noise, seed=m + 3, row_scale=row_scale)
        seed = 99
    res = sap.sap_solve(_dev(p.A), _dev(p.b), d, zeta, seed, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    x = res.x.cpu().numpy()
    x_or, info_or = orc.solve(p.A, p.b, d, zeta, seed, tol=1e-12, maxiter=300)
    nb = np.linalg.norm(p.b)
    assert res.status == sap.SAP_OK, res.info
    assert info_or["status"] == "ok"
    assert np.linalg.norm(p.A @ (x - x_or)) <= 1e-12 * nb
    fwd = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
    _note(f"  forward error {fwd:.2e}, iterations {res.info['iters']} (oracle {info_or['iters']})")
    # The forward bar 1e-8 holds wherever the least-squares perturbation bound
    # kappa u + kappa^2 u ||r|| / (||A|| ||x||) allows it, which it does for
    # every case here.  "lev" is the 1e8-conditioned case with small noise:
    # bound 1.2e-8, and two correct FP64 solvers (the oracle at other sketch
    # seeds, LAPACK's lstsq) differ from the oracle by 1.4e-9 to 1.7e-9 on it.
    assert fwd <= 1e-8, fwd
    # the stopping iteration moves with rounding where the rate is close to 1
    # (d = n + 1: ~80 iterations), by a few percent of the count
    assert abs(res.info["iters"] - info_or["iters"]) <= max(2, 0.05 * info_or["iters"])


def test_solve_claimed_tail_parity(sap, orc):
    """An FP64 solve whose A (2^18 x 300, 629 MB) is past the size at which
    the LSQR pass claims the last eighth of its rows in chunks from a device
    counter (timing-dependent row ownership): against the oracle at the
    paper's metric and the forward bar (bound ~1e-10 here)."""
    import torch
    m, n, d = 1 << 18, 300, 1200
    _note(f"solve claimed-tail m={m} n={n} d={d} ({m * n * 8 / 2**20:.0f} MiB)")
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-8, seed=7)
    res = sap.sap_solve(_dev(p.A), _dev(p.b), d, 8, 5, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    x = res.x.cpu().numpy()
    x_or, info_or = orc.solve(p.A, p.b, d, 8, 5, tol=1e-12, maxiter=300)
    assert res.status == sap.SAP_OK, res.info
    assert info_or["status"] == "ok"
    nb = np.linalg.norm(p.b)
    fwd = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
    _note(f"  forward error {fwd:.2e}, iterations {res.info['iters']} (oracle {info_or['iters']})")
    assert np.linalg.norm(p.A @ (x - x_or)) <= 1e-12 * nb
    assert fwd <= 1e-8
    assert abs(res.info["iters"] - info_or["iters"]) <= 2


def test_solve_errors(sap):
    import torch
    p = inputs.make_problem(3000, 10, kind="svd", cond=1e2, seed=16)
    A = p.A.copy()
    A[:, 7] = A[:, 2]
    _note("solve rank-deficient")
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(A), _dev(p.b), 40, 8, 1)
    assert e.value.status == sap.SAP_RANK_DEFICIENT
    _note("solve maxiter=1")
    res = sap.sap_solve(_dev(p.A), _dev(p.b), 40, 8, 1, maxiter=1)
    assert res.status == sap.SAP_NOT_CONVERGED and res.info["iters"] == 1
    _note("solve invalid d")
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A), _dev(p.b), 10, 8, 1)
    assert e.value.status == sap.SAP_EINVAL
    bad = p.b.copy()
    bad[17] = np.nan
    _note("solve nan b")
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A), _dev(bad), 40, 8, 1)
    assert e.value.status == sap.SAP_EINVAL
    badA = p.A.copy()
    badA[123, 4] = np.inf
    _note("solve inf A")
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(badA), _dev(p.b), 40, 8, 1)
    assert e.value.status == sap.SAP_EINVAL and "not finite" in str(e.value)
    _note("solve dtype mismatch")
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A.astype(np.float32)), _dev(p.b), 40, 8, 1, mode=sap.SAP_MODE_FP64)
    assert e.value.status == sap.SAP_EINVAL
    torch.cuda.synchronize()


def test_solve_deterministic(sap):
    """Fixed reduction orders everywhere except the LDS sketch-apply adds and
    the rows each workgroup of the LSQR pass claims at run time: repeated
    solves agree to the solver tolerance."""
    import torch
    p = inputs.make_problem(20000, 64, kind="svd", cond=1e6, noise=1e-6, seed=5)
    r1 = sap.sap_solve(_dev(p.A), _dev(p.b), 256, 8, 3)
    x1 = r1.x.cpu().numpy()
    r2 = sap.sap_solve(_dev(p.A), _dev(p.b), 256, 8, 3)
    x2 = r2.x.cpu().numpy()
    torch.cuda.synchronize()
    assert np.linalg.norm(p.A @ (x1 - x2)) <= 1e-13 * np.linalg.norm(p.b)


def test_unaligned_wide_rows(sap):
    """n = 4099 in FP64: an odd row length, so the pass reads rows element by
    element, 16 per lane, with all 8 waves of a workgroup across a row (the
    widest element-wise case).  The same matrix stored with lda = n and
    with lda = n + 1 gives the same solution to rounding, and both meet the
    normal-equation bar ||A^T r|| <= 1e-11 ||A||_F (||A||_F ||x|| + ||b||)."""
    import torch
    m, n, d = 20000, 4099, 8200
    _note(f"unaligned wide rows m={m} n={n} d={d}")
    g = torch.Generator(device="cuda")
    g.manual_seed(4099)
    A = torch.randn(m, n, generator=g, device="cuda", dtype=torch.float64)
    A *= torch.logspace(0, -3, n, device="cuda", dtype=torch.float64)[None, :]
    b = torch.randn(m, generator=g, device="cuda", dtype=torch.float64)
    Ap = torch.zeros(m, n + 1, device="cuda", dtype=torch.float64)
    Ap[:, :n] = A
    Aview = Ap[:, :n]  # lda = n + 1
    r1 = sap.sap_solve(A, b, d, 8, 5, tol=1e-12, maxiter=300)
    r2 = sap.sap_solve(Aview, b, d, 8, 5, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    assert r1.status == sap.SAP_OK and r2.status == sap.SAP_OK, (r1.info, r2.info)
    x1, x2 = r1.x, r2.x
    assert float(torch.linalg.vector_norm(x1 - x2)) <= 1e-9 * float(torch.linalg.vector_norm(x2))
    fro = float(torch.linalg.matrix_norm(A))
    for x in (x1, x2):
        r = b - A @ x
        eta = float(torch.linalg.vector_norm(A.T @ r)) / (fro * (fro * float(torch.linalg.vector_norm(x)) +
                                                                 float(torch.linalg.vector_norm(b))))
        assert eta <= 1e-11, eta


def test_adaptive_embedding_dim_solve(sap, orc):
    """A solve at the d that eq. (4.2) picks (Sec. 4.3): parity with the
    oracle at the same d, and the iteration count against the rate estimate
    of eq. (4.1): no more than twice the estimate, and fewer iterations than
    the same problem at d = 4n."""
    import torch
    m, n, eps = 60000, 60, 1e-12
    d = sap.sap_embedding_dim(m, n, eps)
    assert abs(d - orc.embedding_dim(m, n, eps)) <= 1.0
    est = sap.sap_iteration_estimate(n, d, eps)
    _note(f"solve adaptive d m={m} n={n} d={d} estimate={est}")
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-6, seed=6060)
    res = sap.sap_solve(_dev(p.A), _dev(p.b), d, 8, 5, tol=eps, maxiter=300)
    torch.cuda.synchronize()
    x = res.x.cpu().numpy()
    x_or, info_or = orc.solve(p.A, p.b, d, 8, 5, tol=eps, maxiter=300)
    assert res.status == sap.SAP_OK, res.info
    assert info_or["status"] == "ok"
    nb = np.linalg.norm(p.b)
    assert np.linalg.norm(p.A @ (x - x_or)) <= 1e-12 * nb
    assert abs(res.info["iters"] - info_or["iters"]) <= max(2, 0.05 * info_or["iters"])
    assert res.info["iters"] <= 2 * est
    fixed = sap.sap_solve(_dev(p.A), _dev(p.b), 4 * n, 8, 5, tol=eps, maxiter=300)
    torch.cuda.synchronize()
    assert fixed.status == sap.SAP_OK
    assert res.info["iters"] < fixed.info["iters"], (res.info["iters"], fixed.info["iters"])


def test_choose_d_and_auto_d_solve(sap, orc):
    """sap_choose_d (Sec. 4.3 with every phase timed on this GPU) returns one
    of its candidates, k n for k in {1.25 .. 12} or eq. (4.2)'s d, clipped to
    [n + 1, min(m, 16384)]; a solve with d = 0 uses that pick (info d_used)
    and matches the oracle at the same d."""
    import torch
    m, n, eps = 60000, 80, 1e-12
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-6, seed=8080)
    A, b = _dev(p.A), _dev(p.b)
    d = sap.sap_choose_d(A, b, 8, eps)
    cands = {max(n + 1, min(int(np.ceil(k * n)), m, 16384)) for k in (1.25, 1.5, 2, 2.5, 3, 4, 5, 6, 8, 10, 12)}
    cands.add(max(n + 1, min(sap.sap_embedding_dim(m, n, eps), m, 16384)))
    _note(f"choose_d m={m} n={n}: d={d} (candidates {sorted(cands)})")
    assert d in cands
    assert sap.sap_choose_d(A, b, 8, eps) == d  # cached timings: the same pick
    res = sap.sap_solve(A, b, 0, 8, 5, tol=eps, maxiter=300)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK and res.info["d_used"] == d
    x_or, info_or = orc.solve(p.A, p.b, d, 8, 5, tol=eps, maxiter=300)
    assert info_or["status"] == "ok"
    assert np.linalg.norm(p.A @ (res.x.cpu().numpy() - x_or)) <= 1e-12 * np.linalg.norm(p.b)


def test_fixed_count_mode(sap, orc):
    """fixed_iters < 0 runs the eq. (4.1) count for tol (the fixed-count mode
    of Sec. 4.2), > 0 a given count; both report SAP_OK after exactly that many
    iterations and match the oracle run for the same count (tol 0)."""
    import torch
    m, n, d = 30000, 60, 240
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-4, seed=4141)
    A, b = _dev(p.A), _dev(p.b)
    for fixed, tol in ((-1, 1e-6), (7, 1e-12)):
        T = sap.sap_iteration_estimate(n, d, tol) if fixed < 0 else fixed
        _note(f"fixed count m={m} n={n} d={d} fixed_iters={fixed} -> {T}")
        res = sap.sap_solve(A, b, d, 8, 6, tol=tol, maxiter=1000, fixed_iters=fixed)
        torch.cuda.synchronize()
        assert res.status == sap.SAP_OK and res.info["iters"] == T, res.info
        x_or, io = orc.solve(p.A, p.b, d, 8, 6, tol=0.0, maxiter=T)
        assert io["iters"] == T
        assert np.linalg.norm(p.A @ (res.x.cpu().numpy() - x_or)) <= 1e-12 * np.linalg.norm(p.b)
    with pytest.raises(sap.SapError) as e:  # not with the refinement form
        sap.sap_solve(A.float(), b, d, 8, 6, tol=1e-8, mode=sap.SAP_MODE_MIXED_FP32_REFINE, fixed_iters=-1)
    assert e.value.status == sap.SAP_EINVAL
