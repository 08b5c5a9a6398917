"""GPU tests of the served form (sap_submit / sap_poll / sap_cancel): requests
of uneven sizes arrive while others run, are admitted when their workspace
fits in the serving arena, advance together a few LSQR iterations per round
and retire independently.  A served request draws the sketch sap_solve draws
for the same seed (Philox stream word 0), so the oracle reference is Alg. 1
with (seed, stream 0).  The passes accumulate in FP64, so the bars are the
FP64 ones: ||A(x - x_or)|| / ||b|| <= 1e-11 and ||x - x_or|| / ||x_or|| <=
1e-8 (cond <= 1e6 here).  A request's result must not depend on the mix it
ran in beyond the rounding order of the sketch accumulation."""
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


@pytest.fixture
def ctx(sap):
    c = sap.Context(0)
    yield c
    c.close()


def _problem(k, m, n, cond, dtype=np.float64):
    return inputs.make_problem(m, n, kind="colscale", cond=cond, noise=1e-8, seed=4000 + k, dtype=dtype)


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _check(orc, p, x, d, seed, tag):
    A64 = p.A.astype(np.float64)
    x_or, io = orc.solve(A64, p.b, d, 8, seed, tol=1e-12, maxiter=300, stream=0)
    assert io["status"] == "ok"
    nb = np.linalg.norm(p.b)
    assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-11 * nb, tag
    assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or), tag


def test_serve_alone_vs_mix(sap, orc, ctx):
    """One request served alone, then the same request inside a mix of eight
    others submitted in two waves while it runs."""
    import torch
    print("serve alone-vs-mix", flush=True)
    target = _problem(0, 30000, 90, 1e5)
    At, bt = _dev(target.A), _dev(target.b)
    d = 4 * 90
    t = sap.sap_submit(At, bt, d, 8, 77, tol=1e-12, maxiter=300, ctx=ctx)
    st, info, x_alone = sap.sap_poll(t, wait=True, ctx=ctx)
    assert st == sap.SAP_OK, info
    x_alone = x_alone.cpu().numpy()
    _check(orc, target, x_alone, d, 77, "alone")

    others = [_problem(k, int(5000 + 7000 * k), int(17 + 23 * k), 10.0 ** (2 + k % 4)) for k in range(1, 9)]
    tensors = [(_dev(p.A), _dev(p.b)) for p in others]
    tickets = []
    for k in range(4):
        A, b = tensors[k]
        tickets.append(sap.sap_submit(A, b, 4 * others[k].A.shape[1], 8, 100 + k, tol=1e-12, maxiter=300, ctx=ctx))
    t_mix = sap.sap_submit(At, bt, d, 8, 77, tol=1e-12, maxiter=300, ctx=ctx)
    time.sleep(0.002)
    for k in range(4, 8):
        A, b = tensors[k]
        tickets.append(sap.sap_submit(A, b, 4 * others[k].A.shape[1], 8, 100 + k, tol=1e-12, maxiter=300, ctx=ctx))
    st, info, x_mix = sap.sap_poll(t_mix, wait=True, ctx=ctx)
    assert st == sap.SAP_OK, info
    x_mix = x_mix.cpu().numpy()
    assert np.linalg.norm(x_mix - x_alone) <= 1e-9 * np.linalg.norm(x_alone)
    _check(orc, target, x_mix, d, 77, "mix")
    for k, tk in enumerate(tickets):
        st, info, x = sap.sap_poll(tk, wait=True, ctx=ctx)
        assert st == sap.SAP_OK, (k, info)
        assert info["t_total_ms"] >= info["t_queue_ms"] >= 0.0
        _check(orc, others[k], x.cpu().numpy(), 4 * others[k].A.shape[1], 100 + k, f"other {k}")
    torch.cuda.synchronize()
    s = sap.sap_serve_stats(ctx)
    assert s["completed"] == s["submitted"] == 10
    assert s["active"] == 0 and s["queued"] == 0 and s["arena_used"] == 0


def test_serve_admission_by_footprint(sap, orc, ctx):
    """An arena that holds about two requests: later ones wait in the queue
    and are admitted in order as memory comes back; all finish correctly."""
    print("serve admission", flush=True)
    probs = [_problem(20 + k, 40000, 64, 1e4, np.float32) for k in range(6)]
    # footprint of one request: sketch (m*zeta int32 + m uint64), u (m doubles), small parts
    one = 40000 * (8 * 4 + 8 + 8) + (1 << 20)
    sap.sap_serve_start(arena_bytes=int(2.5 * one), max_active=64, ctx=ctx)
    ts = [sap.sap_submit(_dev(p.A), _dev(p.b), 256, 8, 5 + k, tol=1e-12, maxiter=300, ctx=ctx)
          for k, p in enumerate(probs)]
    seen_queued = sap.sap_serve_stats(ctx)["queued"]
    queue_ms = []
    for k, t in enumerate(ts):
        st, info, x = sap.sap_poll(t, wait=True, ctx=ctx)
        assert st == sap.SAP_OK, info
        queue_ms.append(info["t_queue_ms"])
        _check(orc, probs[k], x.cpu().numpy(), 256, 5 + k, f"req {k}")
    assert seen_queued >= 1
    assert max(queue_ms[3:]) > 0.0
    s = sap.sap_serve_stats(ctx)
    assert s["arena_used"] == 0 and s["completed"] == 6


def test_serve_cancel_and_errors(sap, ctx):
    import torch
    print("serve cancel/errors", flush=True)
    p = _problem(50, 60000, 200, 1e6)
    A, b = _dev(p.A), _dev(p.b)
    # tol 0 and a large maxiter: runs until cancelled
    t = sap.sap_submit(A, b, 800, 8, 3, tol=0.0, maxiter=100000, ctx=ctx)
    time.sleep(0.05)
    sap.sap_cancel(t, ctx=ctx)
    st, info, x = sap.sap_poll(t, wait=True, ctx=ctx)
    assert st == sap.SAP_ECANCELED
    assert np.all(np.isfinite(x.cpu().numpy()))
    with pytest.raises(sap.SapError) as e:
        sap.sap_poll(t, ctx=ctx)  # ticket forgotten after its terminal status
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_poll(123456789, ctx=ctx)
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:  # one A dtype per serving context
        sap.sap_submit(A.float(), b, 800, 8, 3, ctx=ctx)
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:  # d >= n + 1
        sap.sap_submit(A, b, 150, 8, 3, ctx=ctx)
    assert e.value.status == sap.SAP_EINVAL
    torch.cuda.synchronize()


def test_serve_request_larger_than_arena(sap, ctx):
    print("serve too large", flush=True)
    sap.sap_serve_start(arena_bytes=1 << 20, max_active=4, ctx=ctx)
    p = _problem(60, 50000, 50, 1e3)
    with pytest.raises(sap.SapError) as e:
        sap.sap_submit(_dev(p.A), _dev(p.b), 200, 8, 3, ctx=ctx)
    assert e.value.status == sap.SAP_ENOMEM
    assert sap.sap_serve_stats(ctx)["rejected"] == 1


def test_serve_rank_deficient(sap, ctx):
    print("serve rank deficient", flush=True)
    p = _problem(70, 20000, 40, 1e3)
    A = p.A.copy()
    A[:, 7] = A[:, 2]
    t_bad = sap.sap_submit(_dev(A), _dev(p.b), 160, 8, 3, ctx=ctx)
    t_ok = sap.sap_submit(_dev(p.A), _dev(p.b), 160, 8, 3, ctx=ctx)
    st, info, _ = sap.sap_poll(t_bad, wait=True, ctx=ctx)
    assert st == sap.SAP_RANK_DEFICIENT
    st, info, _ = sap.sap_poll(t_ok, wait=True, ctx=ctx)
    assert st == sap.SAP_OK


def test_serve_refine_form(sap, orc, ctx):
    """Served requests in the refinement form (FP32 A, FP32 inner solves,
    FP64 residual refinement to a 1e-8 relative correction, the outer loop on
    the device) beside requests in FP64 arithmetic: each refined request
    meets the mixed-form bars against the FP64 oracle on its FP32-rounded A
    (forward <= 1e-8, ||A(x - x_or)|| <= 1e-10 ||b||), alone and in the mix
    alike (alone vs mix within 1e-9)."""
    print("serve refine form", flush=True)
    probs = [_problem(80 + k, int(8000 + 9000 * k), int(40 + 37 * k), 10.0 ** (3 + k % 3), np.float32)
             for k in range(6)]
    tensors = [(_dev(p.A), _dev(p.b)) for p in probs]
    ds = [4 * p.A.shape[1] for p in probs]
    R = sap.SAP_MODE_MIXED_FP32_REFINE
    t = sap.sap_submit(*tensors[0], ds[0], 8, 200, tol=1e-8, maxiter=1000, mode=R, max_refine=12, ctx=ctx)
    st, info, x_alone = sap.sap_poll(t, wait=True, ctx=ctx)
    assert st == sap.SAP_OK, info
    assert info["refinements"] >= 2
    x_alone = x_alone.cpu().numpy()
    tickets = []
    for k, (A, b) in enumerate(tensors):
        mode = R if k % 2 == 0 else sap.SAP_MODE_MIXED_FP32
        tol = 1e-8 if mode == R else 1e-12
        tickets.append(sap.sap_submit(A, b, ds[k], 8, 200 + k, tol=tol, maxiter=1000, mode=mode, max_refine=12,
                                      ctx=ctx))
    for k, tk in enumerate(tickets):
        st, info, x = sap.sap_poll(tk, wait=True, ctx=ctx)
        assert st == sap.SAP_OK, (k, info)
        x = x.cpu().numpy()
        p = probs[k]
        if k % 2:
            _check(orc, p, x, ds[k], 200 + k, f"fp64-arith {k}")
            continue
        A64 = p.A.astype(np.float64)
        x_or, io = orc.solve(A64, p.b, ds[k], 8, 200 + k, tol=1e-12, maxiter=400, stream=0)
        fwd = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
        print(f"  refined k={k} iters={info['iters']} refinements={info['refinements']} forward={fwd:.2e}",
              flush=True)
        assert fwd <= 1e-8, k
        assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-10 * np.linalg.norm(p.b), k
        if k == 0:
            assert np.linalg.norm(x - x_alone) <= 1e-9 * np.linalg.norm(x_alone)


def test_serve_row_slices_fixed_count(sap, orc, ctx):
    """Tall requests whose sketch apply is split over row slices (17 and 31
    of 8192 rows or more, the last ragged) served beside a short one, each run for a
    fixed 8 steps: the iterate still depends on the preconditioner, so the
    FP64 bars against the oracle at the same count hold only if every
    slice's rows enter the sketch exactly once."""
    print("serve row slices", flush=True)
    shapes = [(131073, 32), (250000, 48), (6000, 20)]
    probs = [_problem(50 + k, m, n, 1e4) for k, (m, n) in enumerate(shapes)]
    T = 8
    tickets, keep = [], []
    for k, p in enumerate(probs):
        A, b = _dev(p.A), _dev(p.b)
        keep.append((A, b))
        tickets.append(sap.sap_submit(A, b, 4 * p.A.shape[1], 8, 90 + k, tol=0.0, maxiter=T, ctx=ctx, fixed_iters=T))
    for k, (p, t) in enumerate(zip(probs, tickets)):
        st, info, x = sap.sap_poll(t, wait=True, ctx=ctx)
        assert st == sap.SAP_OK, info
        assert info["iters"] == T, info
        A64 = p.A.astype(np.float64)
        x_or, _ = orc.solve(A64, p.b, 4 * p.A.shape[1], 8, 90 + k, tol=0.0, maxiter=T, stream=0)
        x = x.cpu().numpy()
        assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-11 * np.linalg.norm(p.b), k
        assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or), k
