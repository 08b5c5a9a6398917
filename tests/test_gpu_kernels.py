"""GPU parity: each step of the hot path through the C ABI against the oracle.

Bars (floating point from the arithmetic; see the tolerance section of the
design notes): sketch indices and signs bit-exact; Y bitwise for integer
inputs, ||dY||_F/||Y||_F <= 1e-12 (FP64) or 1e-5 (FP32) otherwise; R backward
error ||R^T R - R_or^T R_or|| / ||R_or||^2 <= 1e-12; triangular solves within
a small multiple of cond(R) * 2^-53.
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


# ------------------------------------------------------------- sketch -----
SKETCH_CASES = [
    # (m, d, zeta, seed, stream)
    (20000, 400, 8, inputs.config_seed(0) + 1, 0),
    (1 << 20, 4000, 8, inputs.config_seed(1) + 1, 0),
    (50000, 6, 3, 11, 0),          # heavy rejection: p = 0.556 per column
    (3000, 64, 64, 12, 5),          # zeta = d: every row in every column
    (7777, 100, 24, 13, 2),
    (4097, 8192, 8, 14, 511),
    (1000, 1, 1, 15, 0),
    (1, 5, 2, 16, 0),
    (12345, 2**31 - 1, 8, 17, 0),   # largest d
    (2000, 300, 17, 18, 1),         # zeta not a power of two, > 16
    (2000, 300, 33, 18, 1),
]


@pytest.mark.parametrize("m,d,zeta,seed,stream", SKETCH_CASES)
def test_sketch_bit_exact(sap, orc, m, d, zeta, seed, stream):
    import torch
    _note(f"sketch m={m} d={d} zeta={zeta} seed={seed} stream={stream}")
    idx, sign = sap.sps_generate(m, d, zeta, seed, stream)
    torch.cuda.synchronize()
    ref_idx, ref_sign = orc.sketch(seed, stream, m, d, zeta)
    assert np.array_equal(idx.cpu().numpy(), ref_idx)
    assert np.array_equal(sign.cpu().numpy().view(np.uint64), ref_sign)


def test_sketch_invalid_args(sap):
    import torch
    for (m, d, zeta) in [(10, 4, 5), (10, 100, 0), (10, 100, 65), (0, 10, 2)]:
        idx = torch.empty((max(m, 1), max(zeta, 1)), dtype=torch.int32, device="cuda")
        sign = torch.empty(max(m, 1), dtype=torch.int64, device="cuda")
        with pytest.raises(sap.SapError) as e:
            sap.sps_generate(m, d, zeta, 1, 0, idx=idx, sign=sign)
        assert e.value.status == sap.SAP_EINVAL


# -------------------------------------------------------------- apply -----
def _apply_case(sap, orc, m, n, d, zeta, kind, adtype, ydtype, with_b=True, lda_pad=0, seed=3):
    import torch
    p = inputs.make_problem(m, n, kind=kind, cond=1e4, seed=seed)
    A_np = p.A
    if adtype == "f32":
        A_np = A_np.astype(np.float32)
    if lda_pad:
        big = np.zeros((m, n + lda_pad), dtype=A_np.dtype)
        big[:, :n] = A_np
        A_dev = torch.from_numpy(big).cuda()[:, :n]
    else:
        A_dev = torch.from_numpy(np.ascontiguousarray(A_np)).cuda()
    b_dev = torch.from_numpy(p.b).cuda() if with_b else None
    idx_ref, sign_ref = orc.sketch(seed + 100, 0, m, d, zeta)
    idx = torch.from_numpy(idx_ref).cuda()
    sign = torch.from_numpy(sign_ref.view(np.int64)).cuda()
    ydt = torch.float64 if ydtype == "f64" else torch.float32
    Y = sap.sps_apply(idx, sign, d, zeta, A_dev, b_dev, y_dtype=ydt)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().T.astype(np.float64)  # d x ncols
    Yo = orc.apply_sparse(idx_ref, sign_ref, A_np.astype(np.float64), p.b if with_b else None, d, zeta)
    return Yg, Yo, idx_ref, sign_ref, A_np, p.b


APPLY_CASES = [
    # m, n, d, zeta, kind, A dtype, Y dtype, with_b, lda_pad
    (20000, 100, 400, 8, "svd", "f64", "f64", True, 0),      # config 0 shape
    (30000, 257, 1000, 8, "colscale", "f64", "f64", True, 3),
    (5000, 3, 70, 4, "colscale", "f64", "f64", False, 0),
    (9000, 33, 30000, 8, "colscale", "f64", "f64", True, 0),  # d beyond one LDS tile: row ranges
    (40000, 64, 512, 12, "colscale", "f32", "f32", True, 0),
    (40000, 64, 512, 8, "colscale", "f32", "f64", True, 1),
    (100000, 17, 8192, 8, "colscale", "f32", "f32", True, 0),
    (1, 5, 7, 3, "colscale", "f64", "f64", True, 0),
    (70000, 47, 4000, 8, "svd", "f64", "f64", True, 0),        # config 1's d: 4 row ranges, bucketed
    (20000, 200, 2600, 8, "colscale", "f32", "f64", True, 0),  # 3 ranges, ragged last tile
    (30000, 1000, 4000, 8, "colscale", "f64", "f64", True, 0),  # 2^20 x 1000 workload's columns: 8 groups
    (20000, 4096, 8192, 8, "colscale", "f32", "f64", True, 0),  # 2^22 x 4096 workload's columns and d
    (20000, 20, 40000, 8, "colscale", "f64", "f64", True, 0),   # d beyond one LDS strip: two row ranges
    (12000, 300, 1200, 64, "colscale", "f64", "f64", True, 0),  # zeta = 64: one sign bit per nonzero
]


@pytest.mark.parametrize("m,n,d,zeta,kind,adt,ydt,with_b,pad", APPLY_CASES)
def test_apply_parity(sap, orc, m, n, d, zeta, kind, adt, ydt, with_b, pad):
    _note(f"apply m={m} n={n} d={d} zeta={zeta} A={adt} Y={ydt} b={with_b} pad={pad}")
    Yg, Yo, *_ = _apply_case(sap, orc, m, n, d, zeta, kind, adt, ydt, with_b, pad)
    rel = np.linalg.norm(Yg - Yo) / np.linalg.norm(Yo)
    bound = 1e-12 if ydt == "f64" else 1e-5
    assert rel <= bound, rel


@pytest.mark.parametrize("ydt,d", [("f64", 700), ("f32", 700), ("f64", 4000), ("f32", 9000)])
def test_apply_integer_bitwise(sap, orc, ydt, d):
    """Integer A and b: every partial sum is an exact integer in the
    accumulation type, so Y = h * sum is the same bits in any order."""
    import torch
    m, n, zeta = 60000, 31, 8
    _note(f"apply-int m={m} n={n} d={d} Y={ydt}")
    p = inputs.make_problem(m, n, kind="integer", seed=9)
    A_np = p.A if ydt == "f64" else p.A.astype(np.float32)
    idx_ref, sign_ref = orc.sketch(77, 0, m, d, zeta)
    Y = sap.sps_apply(torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d,
                      zeta, torch.from_numpy(np.ascontiguousarray(A_np)).cuda(), torch.from_numpy(p.b).cuda(),
                      y_dtype=torch.float64 if ydt == "f64" else torch.float32)
    torch.cuda.synchronize()
    s = orc.sign_values(sign_ref, zeta).astype(np.int64)
    Ab = np.column_stack([p.A, p.b]).astype(np.int64)
    exact = np.zeros((d, n + 1), dtype=np.int64)
    for k in range(zeta):
        np.add.at(exact, idx_ref[:, k], s[:, k:k + 1] * Ab)
    if ydt == "f64":
        ref = exact.astype(np.float64) * orc.sketch_scale(zeta)
        got = Y.cpu().numpy().T
    else:
        assert np.abs(exact).max() < 2**24
        ref = exact.astype(np.float32) * np.float32(orc.sketch_scale(zeta))
        got = Y.cpu().numpy().T
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("ydt", ["f64", "f32"])
def test_apply_bf16_input(sap, orc, ydt):
    """BF16 A (the reduced-precision input variant): the oracle on the
    BF16-rounded values, which are exact in FP64."""
    import torch
    m, n, d, zeta = 30000, 70, 280, 8
    _note(f"apply-bf16 m={m} n={n} d={d} Y={ydt}")
    p = inputs.make_problem(m, n, kind="colscale", cond=1e3, seed=41)
    A_bf = torch.from_numpy(p.A).to(torch.bfloat16)
    A_ref = A_bf.to(torch.float64).numpy()
    idx_ref, sign_ref = orc.sketch(77, 0, m, d, zeta)
    ydtype = torch.float64 if ydt == "f64" else torch.float32
    Y = sap.sps_apply(torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d, zeta,
                      A_bf.cuda(), torch.from_numpy(p.b).cuda(), y_dtype=ydtype)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().T.astype(np.float64)
    Yo = orc.apply_sparse(idx_ref, sign_ref, A_ref, p.b, d, zeta)
    tol = 1e-12 if ydt == "f64" else 1e-5
    assert np.linalg.norm(Yg - Yo) <= tol * np.linalg.norm(Yo)


def test_apply_bf16_wide(sap, orc):
    """BF16 A, 512 columns: full 4-column strips of BF16 input into FP64 Y."""
    import torch
    m, n, d, zeta = 30000, 512, 2048, 8
    _note(f"apply-bf16 wide m={m} n={n} d={d}")
    p = inputs.make_problem(m, n, kind="colscale", cond=1e3, seed=43)
    A_bf = torch.from_numpy(p.A).to(torch.bfloat16)
    A_ref = A_bf.to(torch.float64).numpy()
    idx_ref, sign_ref = orc.sketch(78, 0, m, d, zeta)
    Y = sap.sps_apply(torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d, zeta,
                      A_bf.cuda(), torch.from_numpy(p.b).cuda(), y_dtype=torch.float64)
    torch.cuda.synchronize()
    Yg = Y.cpu().numpy().T
    Yo = orc.apply_sparse(idx_ref, sign_ref, A_ref, p.b, d, zeta)
    assert np.linalg.norm(Yg - Yo) <= 1e-12 * np.linalg.norm(Yo)


def test_apply_ignores_out_of_range_rows(sap, orc):
    """A caller-supplied sketch with row indices outside [0, d) must not
    fault: those nonzeros are ignored."""
    import torch
    m, n, d, zeta = 5000, 9, 3000, 4
    p = inputs.make_problem(m, n, kind="colscale", cond=10.0, seed=4)
    idx_ref, sign_ref = orc.sketch(8, 0, m, d, zeta)
    bad = idx_ref.copy()
    bad[::7, 1] = d + 5
    bad[::11, 2] = -3
    Y = sap.sps_apply(torch.from_numpy(bad).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d, zeta,
                      torch.from_numpy(p.A).cuda(), torch.from_numpy(p.b).cuda())
    torch.cuda.synchronize()
    keep = (bad >= 0) & (bad < d)
    s = orc.sign_values(sign_ref, zeta) * keep
    Ab = np.column_stack([p.A, p.b])
    ref = np.zeros((d, n + 1))
    for k in range(zeta):
        np.add.at(ref, np.where(keep[:, k], bad[:, k], 0), s[:, k:k + 1] * Ab)
    ref *= orc.sketch_scale(zeta)
    assert np.linalg.norm(Y.cpu().numpy().T - ref) <= 1e-12 * np.linalg.norm(ref)


# ----------------------------------------------------------------- QR -----
# rows > 4096 with cols > 192 takes the two-level (64-column panel, WY trailing update) path
QR_CASES = [(400, 101), (4000, 1001), (1000, 1000), (5, 3), (700, 1), (2500, 64), (8192, 130), (16384, 40),
            (513, 100), (1100, 17), (8192, 600), (5000, 257), (700, 259), (300, 300), (193, 193),
            (6000, 700), (4100, 193), (9000, 130),
            # chained one-level path with more workgroups (one per 4 columns) than compute units
            (1200, 1200)]


@pytest.mark.parametrize("rows,cols", QR_CASES)
def test_qr_parity(sap, orc, rows, cols):
    import torch
    _note(f"qr rows={rows} cols={cols}")
    rng = np.random.default_rng(rows * 7 + cols)
    Y = rng.standard_normal((rows, cols)) * np.logspace(0, -4, cols)[None, :]
    Yt = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()  # rows of Yt = columns of Y
    tau = sap.sap_qr(Yt)
    torch.cuda.synchronize()
    F = Yt.cpu().numpy().T
    Fo, tau_o = orc.householder_qr(Y)
    k = min(rows, cols)
    R = np.triu(F[:k])
    Ro = np.triu(Fo[:k])
    nrm = np.linalg.norm(Ro) ** 2
    assert np.linalg.norm(R.T @ R - Ro.T @ Ro) <= 1e-12 * nrm
    kappa = np.linalg.cond(Ro) if k > 1 else 1.0
    assert np.abs(R - Ro).max() <= 100 * kappa * 2.0 ** -53 * np.abs(Ro).max() * max(1, np.sqrt(rows))
    assert np.allclose(tau.cpu().numpy(), tau_o, rtol=0, atol=1e-10)
    # stored Householder vectors reproduce Q with Q R = Y (small cases: the
    # explicit Q is built with rank-1 updates on the host)
    if rows * cols <= 2_000_000:
        Q = orc.q_factor(F, tau.cpu().numpy())
        assert np.linalg.norm(Q @ R - Y) <= 1e-12 * np.linalg.norm(Y) * max(1, np.sqrt(rows) / 10)


@pytest.mark.parametrize("rows,cols", [(4000, 1001), (2048, 1500), (8192, 700)])
def test_qr_chain_reproducible(sap, rows, cols):
    """The chained QR hands each block to whichever workgroup draws its ticket,
    but no sum crosses workgroups, so repeated factorisations of the same
    matrix must agree bit for bit (here with more blocks than compute units at
    2048 x 1500, and through the two-level path's chained panels at 8192 rows)."""
    import torch
    _note(f"qr-repro rows={rows} cols={cols}")
    g = torch.Generator(device="cuda")
    g.manual_seed(rows + cols)
    Y0 = torch.randn(cols, rows, generator=g, dtype=torch.float64, device="cuda")
    outs = []
    for _ in range(3):
        Y = Y0.clone()
        tau = sap.sap_qr(Y)
        torch.cuda.synchronize()
        outs.append((Y.cpu(), tau.cpu()))
    for Y, tau in outs[1:]:
        assert torch.equal(Y, outs[0][0]) and torch.equal(tau, outs[0][1])


@pytest.mark.parametrize("rows", [5000, 3000])
def test_qr_blocked_zero_reflector(sap, orc, rows):
    """A zero column gives tau = 0 inside a panel; the block reflector must then
    drop that reflector (as LAPACK's T does): the two-level path's compact-WY
    update at 5000 rows, the chained one-level path's T at 3000 rows."""
    import torch
    cols = 300
    rng = np.random.default_rng(11)
    Y = rng.standard_normal((rows, cols))
    Y[:, 100] = 0.0
    Yt = torch.from_numpy(np.ascontiguousarray(Y.T)).cuda()
    tau = sap.sap_qr(Yt)
    torch.cuda.synchronize()
    F = Yt.cpu().numpy().T
    Fo, tau_o = orc.householder_qr(Y)
    assert tau_o[100] == 0.0 and tau.cpu().numpy()[100] == 0.0
    R, Ro = np.triu(F[:cols]), np.triu(Fo[:cols])
    assert np.linalg.norm(R.T @ R - Ro.T @ Ro) <= 1e-12 * np.linalg.norm(Ro) ** 2
    assert np.allclose(R, Ro, rtol=0, atol=1e-10 * np.abs(Ro).max())


def test_qr_invalid(sap):
    import torch
    Yt = torch.zeros((5, 3), dtype=torch.float64, device="cuda")
    with pytest.raises(sap.SapError):
        sap.sap_qr(Yt)  # 3 rows x 5 columns: rows < cols


# --------------------------------------------------------------- TRSV -----
@pytest.mark.parametrize("n", [1, 5, 64, 65, 100, 1000, 1001, 2049])
def test_trsv_parity(sap, orc, n):
    import torch
    _note(f"trsv n={n}")
    rng = np.random.default_rng(n)
    Y = rng.standard_normal((max(2 * n, 8), n))
    F, _ = orc.householder_qr(Y)
    R = np.triu(F[:n, :n])
    rhs = rng.standard_normal(n)
    Rt = torch.from_numpy(np.ascontiguousarray(F[:n, :n].T)).cuda()  # lower part holds junk: ignored
    r = torch.from_numpy(rhs).cuda()
    x = sap.sap_trsv(Rt, r, trans=False).cpu().numpy()
    y = sap.sap_trsv(Rt, r, trans=True).cpu().numpy()
    xo = orc.backsub(R, rhs)
    yo = orc.forwardsub_t(R, rhs)
    kappa = np.linalg.cond(R)
    tol = 50 * kappa * 2.0 ** -53 * np.sqrt(n)
    assert np.linalg.norm(x - xo) <= tol * np.linalg.norm(xo)
    assert np.linalg.norm(y - yo) <= tol * np.linalg.norm(yo)


def test_apply_compact_index_path(sap, orc):
    """A sketch re-read by many strips (here 1024 strips of 2 FP64 columns over
    800000 rows, 33 GB of index re-reads) is applied from a 16-bit copy of its
    row indices.  Integer A and b keep every sum exact, so sampled columns of Y
    must equal the exact integer sums times 1/sqrt(zeta) bit for bit."""
    import torch
    m, n, d, zeta = 800000, 2047, 8192, 8
    _note(f"apply-compact m={m} n={n} d={d}")
    g = torch.Generator(device="cuda")
    g.manual_seed(812)
    A = torch.randint(-8, 9, (m, n), generator=g, device="cuda", dtype=torch.int32).to(torch.float32)
    b = torch.randint(-8, 9, (m,), generator=g, device="cuda", dtype=torch.int32).to(torch.float64)
    idx_ref, sign_ref = orc.sketch(2024, 0, m, d, zeta)
    Y = sap.sps_apply(torch.from_numpy(idx_ref).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d,
                      zeta, A, b, y_dtype=torch.float64)
    torch.cuda.synchronize()
    cols = [0, 1, 2, 3, 1000, 1001, 2045, 2046]
    Ab = np.column_stack([A[:, cols].cpu().numpy().astype(np.int64), b.cpu().numpy().astype(np.int64)])
    s = orc.sign_values(sign_ref, zeta).astype(np.int64)
    exact = np.zeros((d, len(cols) + 1), dtype=np.int64)
    for k in range(zeta):
        np.add.at(exact, idx_ref[:, k], s[:, k:k + 1] * Ab)
    got = Y.cpu().numpy().T[:, cols + [n]]
    assert np.array_equal(got, exact.astype(np.float64) * orc.sketch_scale(zeta))


@pytest.mark.parametrize("m,n,d,ydt", [(800000, 2047, 8192, "f64"), (200000, 2047, 35000, "f32")])
def test_apply_compact_out_of_range(sap, orc, m, n, d, ydt):
    """Both forms of the 16-bit index copy with planted indices outside [0, d):
    d = 8192 packs each nonzero's sign into bit 15 of its index, d = 35000
    (one FP32 column a strip) keeps the sign words.  The planted nonzeros must
    be dropped and every other sum exact (integer A and b), so sampled columns
    of Y equal the exact integer sums times 1/sqrt(zeta) bit for bit."""
    import torch
    zeta = 8
    _note(f"apply-compact-oob m={m} n={n} d={d} Y={ydt}")
    g = torch.Generator(device="cuda")
    g.manual_seed(813)
    A = torch.randint(-8, 9, (m, n), generator=g, device="cuda", dtype=torch.int32).to(torch.float32)
    b = torch.randint(-8, 9, (m,), generator=g, device="cuda", dtype=torch.int32).to(torch.float64)
    idx_ref, sign_ref = orc.sketch(2025, 0, m, d, zeta)
    bad = idx_ref.copy()
    bad[::7, 1] = d + 5
    bad[::11, 6] = -3
    bad[::13, 7] = 70000
    Y = sap.sps_apply(torch.from_numpy(bad).cuda(), torch.from_numpy(sign_ref.view(np.int64)).cuda(), d, zeta, A,
                      b, y_dtype=torch.float64 if ydt == "f64" else torch.float32)
    torch.cuda.synchronize()
    cols = [0, 1, 2, 1023, 1024, 2046]
    Ab = np.column_stack([A[:, cols].cpu().numpy().astype(np.int64), b.cpu().numpy().astype(np.int64)])
    keep = (bad >= 0) & (bad < d)
    s = orc.sign_values(sign_ref, zeta).astype(np.int64) * keep
    exact = np.zeros((d, len(cols) + 1), dtype=np.int64)
    for k in range(zeta):
        np.add.at(exact, np.where(keep[:, k], bad[:, k], 0), s[:, k:k + 1] * Ab)
    got = Y.cpu().numpy().T[:, cols + [n]]
    if ydt == "f64":
        ref = exact.astype(np.float64) * orc.sketch_scale(zeta)
    else:
        assert np.abs(exact).max() < 2**24
        ref = exact.astype(np.float32) * np.float32(orc.sketch_scale(zeta))
    assert np.array_equal(got, ref)
