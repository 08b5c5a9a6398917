"""GPU parity of the mixed-precision forms: A stored in FP32; the sketch of
the FP32 values accumulated in FP64; QR, triangular solves, recurrences and
the passes of MIXED_FP32 (which widen each FP32 element) in FP64; FP32 inner
passes in the refinement forms; a BF16 copy of A for the MIXED_BF16SA sketch.
The reference is the FP64 oracle run on the FP32-rounded A (exactly
representable in FP64), so both sides solve the same problem; the bar is the
forward error ||x - x_or|| / ||x_or|| <= 1e-8 (where the least-squares
perturbation bound allows it) and the paper's metric
||A(x - x_or)|| / ||b|| <= 1e-10.  Where the forms round differently from the
oracle (FP32 inner solves, the BF16 sketch) the iterates differ but not the
limit."""
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


MIXED_CASES = [
    # name, m, n, d, kind, cond, noise
    ("colscale", 200000, 256, 1024, "colscale", 1e6, 1e-8),
    ("svd", 60000, 100, 400, "svd", 1e6, 1e-8),
    ("wide", 120000, 1000, 2000, "colscale", 1e4, 1e-6),
    ("odd-n", 50000, 77, 308, "colscale", 1e5, 1e-8),
    # n > 1024: several waves span a row of the pass
    ("wide-rows", 30000, 1100, 2200, "colscale", 1e5, 1e-8),
]


@pytest.mark.parametrize("name,m,n,d,kind,cond,noise", MIXED_CASES)
def test_mixed_solve_parity(sap, orc, name, m, n, d, kind, cond, noise):
    import torch
    print(f"mixed {name} m={m} n={n} d={d}", flush=True)
    p = inputs.make_problem(m, n, kind=kind, cond=cond, noise=noise, seed=m + 11, dtype=np.float32)
    A64 = p.A.astype(np.float64)
    seed = 321
    res = sap.sap_solve(_dev(p.A), _dev(p.b), d, 8, seed, tol=1e-12, maxiter=400, mode=sap.SAP_MODE_MIXED_FP32)
    torch.cuda.synchronize()
    x = res.x.cpu().numpy()
    x_or, info_or = orc.solve(A64, p.b, d, 8, seed, tol=1e-12, maxiter=400)
    assert info_or["status"] == "ok"
    assert res.status == sap.SAP_OK, res.info
    nb = np.linalg.norm(p.b)
    assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-10 * nb
    assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or)


REFINE_CASES = [
    # name, m, n, d, kind, cond, noise
    ("colscale", 200000, 256, 1024, "colscale", 1e6, 1e-8),
    ("svd", 60000, 100, 400, "svd", 1e6, 1e-8),
    ("odd-n", 50000, 77, 308, "colscale", 1e5, 1e-5),
    ("wide-rows", 30000, 1100, 2200, "colscale", 1e5, 1e-8),
]


@pytest.mark.parametrize("name,m,n,d,kind,cond,noise", REFINE_CASES)
def test_refine_solve_parity(sap, orc, name, m, n, d, kind, cond, noise):
    """Residual refinement around FP32 inner solves to the target relative
    error 1e-8, against the FP64 oracle on the same FP32 A: forward error
    ||x - x_or|| <= 1e-8 ||x_or|| and ||A (x - x_or)|| <= 1e-10 ||b||.  The
    cases keep the form's floor, the FP32 rounding of r seen through the
    least-squares solution (~2^-24 ||r|| sqrt(n/m) / sigma_min relative to
    ||x||), well below 1e-8: at noise 1e-3 the odd-n case would sit near it."""
    import torch
    print(f"refine {name} m={m} n={n} d={d}", flush=True)
    p = inputs.make_problem(m, n, kind=kind, cond=cond, noise=noise, seed=m + 29, dtype=np.float32)
    A64 = p.A.astype(np.float64)
    seed = 77
    res = sap.sap_solve(_dev(p.A), _dev(p.b), d, 8, seed, tol=1e-8, maxiter=1000,
                        mode=sap.SAP_MODE_MIXED_FP32_REFINE, max_refine=12)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK, res.info
    assert res.info["refinements"] >= 1
    x = res.x.cpu().numpy()
    x_or, info_or = orc.solve(A64, p.b, d, 8, seed, tol=1e-12, maxiter=400)
    assert info_or["status"] == "ok"
    assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or)
    assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-10 * np.linalg.norm(p.b)


@pytest.mark.parametrize("name,m,n,d,kind,cond,noise", REFINE_CASES[:1] + REFINE_CASES[2:])
def test_bf16_sketch_solve_parity(sap, orc, name, m, n, d, kind, cond, noise):
    """BF16-input sketch (MIXED_BF16SA): the sketch of a BF16 copy of A only
    preconditions, so the refined solution meets the same bars as the
    refinement form against the FP64 oracle on the FP32 A.  The cases are
    column-scaled (their ill-conditioning commutes with the entrywise BF16
    rounding), so the convergence rate stays that of the sketch, about
    rho = sqrt(n/d) per iteration.  What the BF16 sketch loses is the
    sketch-and-solve initial guess: accurate to ~2^-9 instead of to the
    problem's small residual, which costs up to log(2^-9 / 1e-8) / log(1/rho)
    more iterations than the FP32-input refinement form (~18 at d = 4n, ~37
    at d = 2n); the bound allows 6 more."""
    import torch
    print(f"bf16 sketch {name} m={m} n={n} d={d}", flush=True)
    p = inputs.make_problem(m, n, kind=kind, cond=cond, noise=noise, seed=m + 29, dtype=np.float32)
    A64 = p.A.astype(np.float64)
    seed = 77
    res = sap.sap_solve(_dev(p.A), _dev(p.b), d, 8, seed, tol=1e-8, maxiter=1000,
                        mode=sap.SAP_MODE_MIXED_BF16SA, max_refine=12)
    ref = sap.sap_solve(_dev(p.A), _dev(p.b), d, 8, seed, tol=1e-8, maxiter=1000,
                        mode=sap.SAP_MODE_MIXED_FP32_REFINE, max_refine=12)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK, res.info
    extra = int(np.ceil(np.log(2.0 ** -9 / 1e-8) / -np.log(np.sqrt(n / d)))) + 6
    assert res.info["iters"] <= ref.info["iters"] + extra, (res.info["iters"], ref.info["iters"], extra)
    x = res.x.cpu().numpy()
    x_or, info_or = orc.solve(A64, p.b, d, 8, seed, tol=1e-12, maxiter=400)
    assert info_or["status"] == "ok"
    assert np.linalg.norm(x - x_or) <= 1e-8 * np.linalg.norm(x_or)
    assert np.linalg.norm(A64 @ (x - x_or)) <= 1e-10 * np.linalg.norm(p.b)


def test_mixed_mode_dtype_checks(sap):
    p = inputs.make_problem(4000, 10, kind="colscale", cond=10.0, seed=1)
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A), _dev(p.b), 40, 8, 1, mode=sap.SAP_MODE_MIXED_FP32)  # F64 A
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A.astype(np.float32)), _dev(p.b), 40, 8, 1, mode=7)
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A), _dev(p.b), 40, 8, 1, mode=sap.SAP_MODE_MIXED_FP32_REFINE)  # F64 A
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A), _dev(p.b), 40, 8, 1, mode=sap.SAP_MODE_MIXED_BF16SA)  # F64 A
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve(_dev(p.A.astype(np.float32)), _dev(p.b), 40, 8, 1, mode=sap.SAP_MODE_MIXED_FP32_REFINE,
                      max_refine=-1)
    assert e.value.status == sap.SAP_EINVAL


def test_fp32_apply_then_fp64_qr_is_a_good_preconditioner(sap, orc):
    """The preconditioner only has to be approximate: the FP32 sketch gives an
    R with cond(A R^-1) within the sketch's own distortion bound."""
    import torch
    m, n, d = 40000, 60, 240
    p = inputs.make_problem(m, n, kind="colscale", cond=1e6, seed=3, dtype=np.float32)
    idx, sign = sap.sps_generate(m, d, 8, 5)
    Y = sap.sps_apply(idx, sign, d, 8, _dev(p.A), None, y_dtype=torch.float32)
    torch.cuda.synchronize()
    Yh = Y.cpu().numpy().T.astype(np.float64)
    F, _ = orc.householder_qr(Yh)
    R = np.triu(F[:n, :n])
    AM = p.A.astype(np.float64) @ np.linalg.inv(R)
    sv = np.linalg.svd(AM, compute_uv=False)
    eta = np.sqrt(n / d)
    assert sv[0] / sv[-1] <= 2.0 * (1 + eta) / (1 - eta)


def test_refine_repeatable_wide_rows(sap):
    """Refinement form where several waves span a row of the pass (n = 2048,
    FP32 rows: two waves of 1024 columns).  The pass must not update u in
    place there: a wave that read u_i after another wave of the same row
    stored the new value would use the wrong u_i in A^T u.  The refinement
    still converges then, but the inner FP32 solves do not, so the iteration
    and refinement counts vary from run to run.  Three solves of the same
    problem: equal counts, each within 1e-8 of the FP64-arithmetic solution."""
    import torch
    m, n, d = 1 << 20, 2048, 4096
    print(f"refine repeat m={m} n={n} d={d}", flush=True)
    A, b, _ = inputs.make_problem_torch(m, n, kind="colscale", cond=1e6, noise=1e-8, seed=4242,
                                        device="cuda", dtype=torch.float32)
    ref = sap.sap_solve(A, b, d, 8, 99, tol=1e-12, maxiter=400, mode=sap.SAP_MODE_MIXED_FP32)
    torch.cuda.synchronize()
    assert ref.status == sap.SAP_OK, ref.info
    x_ref = ref.x.clone()
    counts = []
    for rep in range(3):
        r = sap.sap_solve(A, b, d, 8, 99, tol=1e-8, maxiter=1600, mode=sap.SAP_MODE_MIXED_FP32_REFINE)
        torch.cuda.synchronize()
        assert r.status == sap.SAP_OK, r.info
        counts.append((r.info["iters"], r.info["refinements"]))
        rel = float((r.x - x_ref).norm() / x_ref.norm())
        print(f"rep {rep}: iters {counts[-1][0]} refinements {counts[-1][1]} rel {rel:.2e}", flush=True)
        assert rel <= 1e-8
    assert len(set(counts)) == 1, counts


def test_wide_rows_refine_and_mixed_parity(sap, orc):
    """n = 2100 FP32 rows against the oracle: the passes then run four waves
    across a row (the FP32 inner pass and the FP64-accumulating residual pass
    of the refinement form, and the FP64-arithmetic pass of MIXED_FP32), the
    explicit inverse of R takes its 2-level blocked path, and A (2^16 x 2100,
    525 MiB of FP32) is past the size at which the pass claims the last eighth
    of its rows from a device counter.  One oracle solve (FP64 on the
    FP32-rounded A) is the reference for both forms; d = 2n, the ratio of the
    2^22 x 4096 workload.  Bars: forward error <= 1e-8 and the metric
    ||A(x - x_or)|| <= 1e-10 ||b|| (perturbation bound ~1e-10 here)."""
    import torch
    m, n, d = 1 << 16, 2100, 4200
    print(f"wide refine+mixed m={m} n={n} d={d}", flush=True)
    p = inputs.make_problem(m, n, kind="colscale", cond=1e5, noise=1e-8, seed=m + 29, dtype=np.float32)
    A64 = p.A.astype(np.float64)
    seed = 77
    A, b = _dev(p.A), _dev(p.b)
    ref = sap.sap_solve(A, b, d, 8, seed, tol=1e-8, maxiter=1000, mode=sap.SAP_MODE_MIXED_FP32_REFINE,
                        max_refine=12)
    mix = sap.sap_solve(A, b, d, 8, seed, tol=1e-12, maxiter=400, mode=sap.SAP_MODE_MIXED_FP32)
    torch.cuda.synchronize()
    assert ref.status == sap.SAP_OK, ref.info
    assert mix.status == sap.SAP_OK, mix.info
    print(f"  refine: iters {ref.info['iters']} refinements {ref.info['refinements']}; "
          f"mixed: iters {mix.info['iters']}", flush=True)
    x_or, info_or = orc.solve(A64, p.b, d, 8, seed, tol=1e-12, maxiter=400)
    assert info_or["status"] == "ok"
    nb, nx = np.linalg.norm(p.b), np.linalg.norm(x_or)
    for name, r in (("refine", ref), ("mixed", mix)):
        x = r.x.cpu().numpy()
        fwd = np.linalg.norm(x - x_or) / nx
        met = np.linalg.norm(A64 @ (x - x_or)) / nb
        print(f"  {name}: forward {fwd:.2e} metric {met:.2e}", flush=True)
        assert fwd <= 1e-8, (name, fwd)
        assert met <= 1e-10, (name, met)
    assert abs(mix.info["iters"] - info_or["iters"]) <= max(2, 0.05 * info_or["iters"])
