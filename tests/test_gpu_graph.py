"""The LSQR and momentum iteration batches are captured once into a hipGraph
and replayed (timing mode launches them directly).  Replays must give what
direct launches give: bit for bit where the whole computation is
deterministic (LSQR alone, fixed R and x0, a matrix small enough for static
row splits), to the solver tolerance where the sketch apply's LDS adds make
Y differ in its last bits.  Replays alternate with other work (another
problem's solve, host copies) so that stale cached graphs would show."""
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


def _lsqr_inputs(orc, m, n, d, seed):
    p = inputs.make_problem(m, n, kind="svd", cond=1e6, noise=1e-6, seed=seed)
    idx, sign = orc.sketch(seed, 0, m, d, 8)
    F, _ = orc.householder_qr(orc.apply_sparse(idx, sign, p.A, p.b, d, 8))
    R = np.triu(F[:n, :n])
    return p, R, orc.backsub(R, F[:n, n])


def test_lsqr_graph_replays_match_direct(sap, orc):
    import torch
    ctx = sap.default_context()
    p, R, x0 = _lsqr_inputs(orc, 20000, 100, 400, 31)
    q, Rq, xq0 = _lsqr_inputs(orc, 9000, 60, 240, 32)
    A, b, Rt, x0d = _dev(p.A), _dev(p.b), _dev(np.ascontiguousarray(R.T)), _dev(x0)
    Aq, bq, Rqt, xq0d = _dev(q.A), _dev(q.b), _dev(np.ascontiguousarray(Rq.T)), _dev(xq0)
    ctx.profile(True)                      # direct launches
    ref = sap.sap_lsqr(A, b, Rt, x0d, tol=1e-12, maxiter=300)
    refq = sap.sap_lsqr(Aq, bq, Rqt, xq0d, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    ctx.profile(False)
    ctx.profile_read(sap.PROF_PASS, reset=True)
    x_ref, xq_ref = ref.x.cpu().numpy(), refq.x.cpu().numpy()
    for rep in range(3):                   # capture, then replays, interleaved with the other problem
        r = sap.sap_lsqr(A, b, Rt, x0d, tol=1e-12, maxiter=300)
        rq = sap.sap_lsqr(Aq, bq, Rqt, xq0d, tol=1e-12, maxiter=300)
        torch.cuda.synchronize()
        assert r.info["iters"] == ref.info["iters"] and rq.info["iters"] == refq.info["iters"]
        assert np.array_equal(r.x.cpu().numpy(), x_ref), rep
        assert np.array_equal(rq.x.cpu().numpy(), xq_ref), rep
        _ = (A[:10] * 2).cpu()             # eager work between replays


def test_solve_forms_graph_vs_direct(sap):
    """FP64 LSQR, momentum and the sparse solve: graph replays against direct
    launches, to the tolerance the sketch apply's LDS adds allow."""
    import torch
    ctx = sap.default_context()
    p = inputs.make_problem(30000, 120, kind="svd", cond=1e6, noise=1e-6, seed=9)
    A, b = _dev(p.A), _dev(p.b)
    As, bs, _ = inputs.make_sparse_problem(40000, 80, 0.02, values="gauss", noise=1e-6, seed=10)
    ip = torch.from_numpy(As.indptr.astype(np.int64)).cuda()
    ix = torch.from_numpy(As.indices.astype(np.int32)).cuda()
    v = torch.from_numpy(As.data).cuda()
    bsd = _dev(bs)

    def run_all():
        out = [sap.sap_solve(A, b, 480, 8, 2).x.cpu().numpy(),
               sap.sap_solve_hbm(A, b, 480, 8, 2, tol=1e-10).x.cpu().numpy(),
               sap.sap_solve_csr(ip, ix, v, (40000, 80), bsd, 320, 8, 2).x.cpu().numpy()]
        torch.cuda.synchronize()
        return out

    ctx.profile(True)
    direct = run_all()
    ctx.profile(False)
    ctx.profile_read(sap.PROF_PASS, reset=True)
    for rep in range(3):
        got = run_all()
        assert np.linalg.norm(p.A @ (got[0] - direct[0])) <= 1e-13 * np.linalg.norm(p.b), rep
        assert np.linalg.norm(p.A @ (got[1] - direct[1])) <= 1e-11 * np.linalg.norm(p.b), rep
        assert np.linalg.norm(As @ (got[2] - direct[2])) <= 1e-13 * np.linalg.norm(bs), rep
