"""GPU parity at the full sizes of the four workloads, in the launch
configuration bench.py times.  The oracle cannot redo these solves in
seconds, so the checks are: outputs the oracle computes one at a time
(sampled columns of the sketch product, a few problems of a batch or of a
request stream), and properties that hold at any size (the normal-equation
residual of the solution, agreement of two precision forms).

Bars: sampled Y columns ||dY|| / ||Y|| <= 1e-12 (FP64 sums of ~m zeta / d
terms); the normal-equation backward error
eta = ||A^T r|| / (||A||_F (||A||_F ||x|| + ||b||)) <= 1e-11, r = b - A x: the
stopping test (alpha |c| <= tol with ||A R^-1|| <= 1 + eta_S, or
||r|| <= tol ||b||) bounds it by about 1.5 tol = 1.5e-12, and the rounding of
r itself stays near 1e-15 in this normalisation (unlike ||A^T r|| / (||A|| ||r||),
which the cancellation in r floors near u ||A|| ||x|| / ||r|| for
near-consistent problems); sampled problems against the oracle at the FP64 bar
of the smaller tests, ||A (x - x_or)|| <= 1e-11 ||b||."""
import time

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


def _ne_residual(A, b, x, chunk=1 << 18):
    """Normal-equation backward error ||A^T r|| / (||A||_F (||A||_F ||x|| +
    ||b||)), r = b - A x, in FP64 with A in row chunks (widened when stored
    FP32)."""
    import torch
    n = A.shape[1]
    atr = torch.zeros(n, dtype=torch.float64, device=A.device)
    fro = 0.0
    for r0 in range(0, A.shape[0], chunk):
        blk = A[r0:r0 + chunk].to(torch.float64)
        r = b[r0:r0 + chunk] - blk @ x
        atr += blk.T @ r
        fro += float((blk * blk).sum())
    fro = np.sqrt(fro)
    return float(torch.linalg.vector_norm(atr)) / (fro * (fro * float(torch.linalg.vector_norm(x)) +
                                                          float(torch.linalg.vector_norm(b))))


def test_fp64_workload_full_size(sap, orc):
    """m = 2^20, n = 1000, d = 4000: sampled sketch columns against the
    oracle, then the solve bench.py times."""
    import torch
    _note("full-size FP64 workload: generating")
    A, b, _, meta = inputs.config1_torch("cuda")
    m, n, d, zeta, seed = meta["m"], meta["n"], meta["d"], meta["zeta"], meta["sketch_seed"]
    idx, sign = sap.sps_generate(m, d, zeta, seed)
    Y = sap.sps_apply(idx, sign, d, zeta, A, b)
    torch.cuda.synchronize()
    sel = [0, 1, 333, 998, 999]
    _note("full-size FP64 workload: oracle on sampled columns")
    A_sub = A[:, sel].cpu().numpy()
    Yo = orc.apply_sparse(idx.cpu().numpy(), sign.cpu().numpy().view(np.uint64), A_sub, b.cpu().numpy(), d, zeta,
                          cols=list(range(len(sel))) + [len(sel)])
    Yg = Y.cpu().numpy().T[:, sel + [n]]
    for k in range(len(sel) + 1):
        assert np.linalg.norm(Yg[:, k] - Yo[:, k]) <= 1e-12 * np.linalg.norm(Yo[:, k]), k
    _note("full-size FP64 workload: solve")
    r = sap.sap_solve(A, b, d, zeta, seed, tol=meta["tol"], maxiter=meta["maxiter"])
    torch.cuda.synchronize()
    assert r.status == sap.SAP_OK, r.info
    ne = _ne_residual(A, b, r.x)
    _note(f"full-size FP64 workload: iters {r.info['iters']}, normal-equation backward error {ne:.2e}")
    assert ne <= 1e-11
    assert np.all(np.isfinite(r.x.cpu().numpy()))


def test_mixed_workload_full_size(sap):
    """m = 2^22, n = 4096, d = 8192, A stored FP32 (64 GiB)."""
    import torch
    _note("full-size mixed workload: generating")
    A, b, _, meta = inputs.config2_torch("cuda")
    t0 = time.perf_counter()
    r = sap.sap_solve(A, b, meta["d"], meta["zeta"], meta["sketch_seed"], tol=meta["tol"], maxiter=meta["maxiter"],
                      mode=sap.SAP_MODE_MIXED_FP32)
    torch.cuda.synchronize()
    _note(f"full-size mixed workload: solve {time.perf_counter() - t0:.2f} s, iters {r.info['iters']}")
    assert r.status == sap.SAP_OK, r.info
    ne = _ne_residual(A, b, r.x)
    _note(f"full-size mixed workload: normal-equation backward error {ne:.2e}")
    assert ne <= 1e-11
    # the FP64 form on the exact FP64 copy of the same matrix (128 GiB)
    A64 = torch.empty(A.shape, dtype=torch.float64, device=A.device)
    for r0 in range(0, A.shape[0], 1 << 18):
        A64[r0:r0 + (1 << 18)] = A[r0:r0 + (1 << 18)].to(torch.float64)
    del A
    torch.cuda.empty_cache()
    r64 = sap.sap_solve(A64, b, meta["d"], meta["zeta"], meta["sketch_seed"], tol=meta["tol"],
                        maxiter=meta["maxiter"])
    torch.cuda.synchronize()
    assert r64.status == sap.SAP_OK, r64.info
    diff = 0.0
    for r0 in range(0, A64.shape[0], 1 << 18):
        e = A64[r0:r0 + (1 << 18)] @ (r.x - r64.x)
        diff += float(e @ e)
    rel = np.sqrt(diff) / float(torch.linalg.vector_norm(b))
    _note(f"full-size mixed workload: ||A (x_mixed - x_fp64)|| / ||b|| = {rel:.2e}")
    assert rel <= 1e-10
    del A64
    torch.cuda.empty_cache()


def test_batched_workload_full_size(sap, orc):
    """512 problems, m ~ U[5000, 200000], n ~ U{32..256}, FP32 A: every
    problem by its normal-equation residual, three against the oracle."""
    import torch
    shapes = inputs.batch_shapes(count=512)
    _note("full-size batched workload: generating 512 problems")
    As, bs = [], []
    for s in shapes:
        A, b, _ = inputs.make_problem_torch(s["m"], s["n"], kind="colscale", cond=s["cond"], noise=1e-8,
                                            seed=s["seed"], device="cuda", dtype=torch.float32)
        As.append(A)
        bs.append(b)
    ds = [s["d"] for s in shapes]
    seeds = [s["seed"] + 1 for s in shapes]
    xs, st, infos = sap.sap_solve_batch(As, bs, ds, 8, seeds, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    assert st == sap.SAP_OK
    worst = max(_ne_residual(As[k], bs[k], xs[k]) for k in range(len(As)))
    _note(f"full-size batched workload: worst normal-equation backward error {worst:.2e}")
    assert worst <= 1e-11
    for k in (0, 255, 511):
        _note(f"full-size batched workload: oracle on problem {k} (m={shapes[k]['m']}, n={shapes[k]['n']})")
        A64 = As[k].cpu().numpy().astype(np.float64)
        bk = bs[k].cpu().numpy()
        x_or, io = orc.solve(A64, bk, ds[k], 8, seeds[k], tol=1e-12, maxiter=300, stream=k)
        assert io["status"] == "ok"
        x = xs[k].cpu().numpy()
        assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-11 * np.linalg.norm(bk), k
    del As
    torch.cuda.empty_cache()


def test_served_workload_sample(sap, orc):
    """The first 0.25 s of the 200 requests/s stream (m up to 2^21, n up to
    512), submitted at their arrival times: every request by its residual,
    two against the oracle."""
    import torch
    reqs = inputs.served_stream(rate=200.0, duration=0.25)
    _note(f"served workload sample: {len(reqs)} requests")
    probs = []
    for k, r in enumerate(reqs):
        A, b, _ = inputs.make_problem_torch(r["m"], r["n"], kind="colscale", cond=1e6, noise=1e-8,
                                            seed=inputs.config_seed(4) + 13 * k, device="cuda",
                                            dtype=torch.float32)
        probs.append((A, b))
    torch.cuda.synchronize()
    ctx = sap.Context(0)
    tickets = []
    t0 = time.perf_counter()
    for k, r in enumerate(reqs):
        delay = t0 + r["t"] - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        tickets.append(sap.sap_submit(probs[k][0], probs[k][1], r["d"], 8, 101 + k, tol=1e-12, maxiter=300,
                                      ctx=ctx))
    xs = []
    for t in tickets:
        st, info, x = sap.sap_poll(t, wait=True, ctx=ctx)
        assert st == sap.SAP_OK, info
        xs.append(x)
    ctx.close()
    worst = max(_ne_residual(probs[k][0], probs[k][1], xs[k]) for k in range(len(reqs)))
    _note(f"served workload sample: worst normal-equation backward error {worst:.2e}")
    assert worst <= 1e-11
    small = sorted(range(len(reqs)), key=lambda k: reqs[k]["m"] * reqs[k]["n"])[:2]
    for k in small:
        _note(f"served workload sample: oracle on request {k} (m={reqs[k]['m']}, n={reqs[k]['n']})")
        A64 = probs[k][0].cpu().numpy().astype(np.float64)
        bk = probs[k][1].cpu().numpy()
        x_or, io = orc.solve(A64, bk, reqs[k]["d"], 8, 101 + k, tol=1e-12, maxiter=300, stream=0)
        assert io["status"] == "ok"
        assert np.linalg.norm(A64 @ (xs[k].cpu().numpy() - x_or)) <= 1e-11 * np.linalg.norm(bk), k
