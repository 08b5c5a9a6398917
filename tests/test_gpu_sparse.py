"""GPU parity of the sparse (CSR) path: the sketch apply on the stored
entries and Alg. 1 with the fused sparse LSQR pass, against the oracle's CSR
routes (which are pinned bit for bit to its dense routes).  Table 1's sparse
problems are not available here; Sec. 4.1's synthetic sparse recipe (+-1
entries at density 0.01) stands in for them, plus Gaussian values and FP32
storage.  Bars: the apply within 1e-12 relative (bitwise for +-1 entries
with an integer b, whose sums are exact integers), the solve at the FP64
bars ||A(x - x_or)|| <= 1e-12 ||b||, ||x - x_or|| <= 1e-8 ||x_or||."""
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


def _dev_csr(A, dtype=np.float64):
    import torch
    return (torch.from_numpy(A.indptr.astype(np.int64)).cuda(), torch.from_numpy(A.indices.astype(np.int32)).cuda(),
            torch.from_numpy(A.data.astype(dtype)).cuda())


@pytest.mark.parametrize("m,n,density,values,d,zeta", [
    (20000, 100, 0.01, "sign", 400, 8),
    (30000, 257, 0.02, "gauss", 1028, 8),
    (5000, 3, 0.3, "gauss", 40, 4),
    (40000, 64, 0.005, "sign", 4096, 12),   # long columns of b, short rows
    (25000, 90, 0.02, "gauss", 360, 16),
    (25000, 90, 0.02, "sign", 360, 24),
    (25000, 90, 0.02, "gauss", 360, 5),     # zeta not a multiple of 4
    (1500000, 8, 0.002, "sign", 64, 8),     # more rows than one scatter window per workgroup
])
def test_sparse_apply_parity(sap, orc, m, n, density, values, d, zeta):
    import torch
    print(f"sparse apply m={m} n={n} density={density} {values} d={d}", flush=True)
    A, b, _ = inputs.make_sparse_problem(m, n, density, values=values, seed=m + n)
    if values == "sign":
        b = np.rint(b * 4.0)  # integer b: every sum exact
    ip, ix, v = _dev_csr(A)
    idx_ref, sign_ref = orc.sketch(31, 0, m, d, zeta)
    Y = sap.sps_apply_csr(torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d, zeta,
                          ip, ix, v, (m, n), torch.from_numpy(b).cuda())
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().T
    Yo = orc.apply_csr(idx_ref, sign_ref, A, b, d, zeta)
    if values == "sign":
        assert np.array_equal(Yg, Yo)
    else:
        assert np.linalg.norm(Yg - Yo) <= 1e-12 * np.linalg.norm(Yo)


@pytest.mark.parametrize("m,n,density,values,d", [
    (500000, 500, 0.01, "sign", 2000),   # Sec. 4.1's sparse recipe at Table 1's 5e5 x 500 size
    (60000, 120, 0.03, "gauss", 480),
    (30000, 1100, 0.02, "gauss", 2200),  # wide rows: L = 32 lanes a row
])
def test_sparse_solve_parity(sap, orc, m, n, density, values, d):
    import torch
    print(f"sparse solve m={m} n={n} density={density} {values} d={d}", flush=True)
    A, b, _ = inputs.make_sparse_problem(m, n, density, values=values, noise=1e-6, seed=7 * m + n)
    ip, ix, v = _dev_csr(A)
    res = sap.sap_solve_csr(ip, ix, v, (m, n), torch.from_numpy(b).cuda(), d, 8, 17, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK, res.info
    x = res.x.cpu().numpy()
    x_or, io = orc.solve_csr(A, b, d, 8, 17, tol=1e-12, maxiter=300)
    assert io["status"] == "ok"
    fwd = np.linalg.norm(x - x_or) / np.linalg.norm(x_or)
    print(f"  iters {res.info['iters']} (oracle {io['iters']}), forward {fwd:.2e}, apply {res.info['t_apply_ms']:.2f} ms, "
          f"iterate {res.info['t_iterate_ms']:.2f} ms", flush=True)
    assert np.linalg.norm(A @ (x - x_or)) <= 1e-12 * np.linalg.norm(b)
    assert fwd <= 1e-8
    assert abs(res.info["iters"] - io["iters"]) <= 2


def test_sparse_fp32_values_and_errors(sap, orc):
    """F32 values (MIXED_FP32: FP64 arithmetic) against the oracle on the
    FP32-rounded values; argument checks."""
    import torch
    m, n, d = 40000, 90, 360
    A, b, _ = inputs.make_sparse_problem(m, n, 0.02, values="gauss", noise=1e-6, seed=99)
    A32 = A.astype(np.float32).astype(np.float64)
    ip, ix, v = _dev_csr(A, np.float32)
    res = sap.sap_solve_csr(ip, ix, v, (m, n), torch.from_numpy(b).cuda(), d, 8, 3, tol=1e-12, maxiter=300)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK, res.info
    x_or, io = orc.solve_csr(A32.tocsr(), b, d, 8, 3, tol=1e-12, maxiter=300)
    assert np.linalg.norm(A32 @ (res.x.cpu().numpy() - x_or)) <= 1e-12 * np.linalg.norm(b)
    bdev = torch.from_numpy(b).cuda()
    with pytest.raises(sap.SapError) as e:  # values F32 with the FP64 mode
        sap.sap_solve_csr(ip, ix, v, (m, n), bdev, d, mode=sap.SAP_MODE_FP64)
    assert e.value.status == sap.SAP_EINVAL
    with pytest.raises(sap.SapError) as e:  # d < n + 1
        sap.sap_solve_csr(ip, ix, v, (m, n), bdev, n)
    assert e.value.status == sap.SAP_EINVAL


def test_sparse_apply_long_columns_and_empty(sap, orc):
    """A column dense enough to span several work items, empty rows, empty
    columns, and a matrix with no stored entries at all."""
    import scipy.sparse as sp
    import torch
    m, n, d, zeta = 30000, 40, 300, 8
    rng = np.random.default_rng(5)
    rows = np.concatenate([np.arange(0, m, 2), rng.integers(0, m, 3000)])          # column 0: 15000 + entries
    cols = np.concatenate([np.zeros(m // 2, dtype=np.int64), rng.integers(2, n, 3000)])  # column 1 stays empty
    A = sp.coo_matrix((rng.integers(-3, 4, len(rows)).astype(np.float64), (rows, cols)), shape=(m, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    b = rng.integers(-5, 6, m).astype(np.float64)
    idx_ref, sign_ref = orc.sketch(77, 0, m, d, zeta)
    idx, sign = torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda()
    for mat, bb in ((A, b), (A, None), (sp.csr_matrix((m, n)), b)):
        print(f"sparse apply nnz={mat.nnz} with_b={bb is not None}", flush=True)
        ip, ix, v = _dev_csr(mat)
        Y = sap.sps_apply_csr(idx, sign, d, zeta, ip, ix, v, (m, n), None if bb is None else torch.from_numpy(bb).cuda())
        torch.cuda.synchronize()
        assert np.array_equal(Y.cpu().numpy().T, orc.apply_csr(idx_ref, sign_ref, mat, bb, d, zeta))


def test_sparse_rejects_bad_csr(sap, orc):
    """CSR arrays that fail the device check give SAP_EINVAL (the apply
    kernels clamp every access, so the bad call itself stays in bounds), and
    the next good call is unaffected."""
    import torch
    m, n, d = 20000, 50, 200
    A, b, _ = inputs.make_sparse_problem(m, n, 0.02, values="sign", noise=1e-6, seed=4)
    idx_ref, sign_ref = orc.sketch(3, 0, m, d, 8)
    idx, sign = torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda()
    bdev = torch.from_numpy(b).cuda()
    ip, ix, v = _dev_csr(A)
    bad_ix = ix.clone()
    bad_ix[A.nnz // 2] = n                      # column index out of range
    bad_ip = ip.clone()
    bad_ip[m // 2] = ip[m // 2 + 1] + 7         # indptr decreases after row m/2
    for tag, args in (("index", (ip, bad_ix, v)), ("indptr", (bad_ip, ix, v))):
        print(f"bad csr: {tag}", flush=True)
        with pytest.raises(sap.SapError) as e:
            sap.sps_apply_csr(idx, sign, d, 8, *args, (m, n), bdev)
        assert e.value.status == sap.SAP_EINVAL
        with pytest.raises(sap.SapError) as e:
            sap.sap_solve_csr(*args, (m, n), bdev, d)
        assert e.value.status == sap.SAP_EINVAL
    Y = sap.sps_apply_csr(idx, sign, d, 8, ip, ix, v, (m, n), torch.from_numpy(np.rint(4 * b)).cuda())
    torch.cuda.synchronize()
    assert np.array_equal(Y.cpu().numpy().T, orc.apply_csr(idx_ref, sign_ref, A, np.rint(4 * b), d, 8))


def test_sparse_auto_d_fixed_count_and_rank_deficient(sap, orc):
    import scipy.sparse as sp
    import torch
    m, n = 50000, 80
    A, b, _ = inputs.make_sparse_problem(m, n, 0.02, values="gauss", noise=1e-6, seed=12)
    ip, ix, v = _dev_csr(A)
    bdev = torch.from_numpy(b).cuda()
    print("sparse solve d=0", flush=True)
    res = sap.sap_solve_csr(ip, ix, v, (m, n), bdev, 0, 8, 5, tol=1e-10, maxiter=300)
    torch.cuda.synchronize()
    d_exp = min(int(sap.sap_embedding_dim(m, n, 1e-10)), 16384, m)
    assert res.info["d_used"] == d_exp
    x_or, io = orc.solve_csr(A, b, d_exp, 8, 5, tol=1e-10, maxiter=300)
    assert res.status == sap.SAP_OK
    assert np.linalg.norm(A @ (res.x.cpu().numpy() - x_or)) <= 1e-10 * np.linalg.norm(b)
    print("sparse solve fixed count", flush=True)
    res = sap.sap_solve_csr(ip, ix, v, (m, n), bdev, 4 * n, 8, 5, tol=1e-12, fixed_iters=7)
    torch.cuda.synchronize()
    assert res.status == sap.SAP_OK and res.info["iters"] == 7
    x_or, io = orc.solve_csr(A, b, 4 * n, 8, 5, tol=0.0, maxiter=7)
    assert np.linalg.norm(res.x.cpu().numpy() - x_or) <= 1e-10 * np.linalg.norm(x_or)
    print("sparse solve rank deficient", flush=True)
    Ad = A.tolil()
    Ad[:, 3] = 0.0                              # an empty column: A has rank n - 1
    Ad = Ad.tocsr()
    Ad.eliminate_zeros()
    ip, ix, v = _dev_csr(Ad)
    with pytest.raises(sap.SapError) as e:
        sap.sap_solve_csr(ip, ix, v, (m, n), bdev, 4 * n)
    assert e.value.status == sap.SAP_RANK_DEFICIENT
