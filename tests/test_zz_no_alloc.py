"""The allocation-free sketch apply (sps_apply_noalloc) against sps_apply,
through the C ABI: the same result to the apply's bar (FP64: relative
Frobenius difference <= 1e-12, the strip kernel's LDS adds land in a
run-dependent order; integer-valued input: bit for bit), on two calls in a
row whose second input is smaller than the first (the static buffer keeps the
first call's partial sums, which the second must not pick up), and a request
larger than the static buffer is refused with SAP_ENOMEM before any device
work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sap():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2506_03070_amd as sap
    sap.lib()
    return sap


def _case(sap, m, n, d, seed, integer):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    if integer:
        A = torch.randint(-1024, 1025, (m, n), generator=g, device="cuda").to(torch.float64)
        b = torch.randint(-1024, 1025, (m,), generator=g, device="cuda").to(torch.float64)
    else:
        A = torch.randn(m, n, generator=g, device="cuda", dtype=torch.float64)
        b = torch.randn(m, generator=g, device="cuda", dtype=torch.float64)
    idx, sign = sap.sps_generate(m, d, 8, seed)
    return A, b, idx, sign


def test_noalloc_apply_matches_apply(sap):
    import torch
    # first call: the 2^20 x 1000 layout at a quarter of the rows (row slices
    # summed through the static buffer); second call: smaller, integer-valued
    for (m, n, d, seed, integer) in [(1 << 18, 1000, 4000, 11, False), (30000, 77, 600, 12, True)]:
        print(f"noalloc apply m={m} n={n} d={d} integer={integer}", flush=True)
        A, b, idx, sign = _case(sap, m, n, d, seed, integer)
        Y_na = sap.sps_apply_noalloc(idx, sign, d, 8, A, b, y_dtype=torch.float64)
        Y_ref = sap.sps_apply(idx, sign, d, 8, A, b, y_dtype=torch.float64)
        torch.cuda.synchronize()
        if integer:
            assert torch.equal(Y_na, Y_ref)
        else:
            rel = float((Y_na - Y_ref).norm() / Y_ref.norm())
            print(f"  relative difference {rel:.2e}", flush=True)
            assert rel <= 1e-12


def test_noalloc_apply_refuses_oversize(sap):
    """A BF16 apply over 2^23 rows whose 16-bit index copy alone (2^23 x 16
    bytes = 128 MiB) plus alignment exceeds the static buffer: SAP_ENOMEM,
    raised on the host before any kernel runs (A and the sketch are left
    uninitialised on purpose; nothing reads them)."""
    import torch
    m, n, d = 1 << 23, 190, 4000
    print(f"noalloc oversize m={m} n={n} d={d}", flush=True)
    A = torch.empty(m, n, dtype=torch.bfloat16, device="cuda")
    b = torch.empty(m, dtype=torch.float64, device="cuda")
    idx = torch.empty(m, 8, dtype=torch.int32, device="cuda")
    sign = torch.empty(m, dtype=torch.int64, device="cuda")
    with pytest.raises(sap.SapError) as e:
        sap.sps_apply_noalloc(idx, sign, d, 8, A, b, y_dtype=torch.float64)
    assert e.value.status == sap.SAP_ENOMEM
    assert "static buffer" in str(e.value)
