"""The library's host-only embedding-dimension entry points (Sec. 4.3,
eqs. (4.1) and (4.2)) against the oracle: sap_embedding_dim returns the
oracle's real d rounded up and clamped to [n + 1, min(m, INT32_MAX)];
sap_iteration_estimate the oracle's real t rounded up.  No device work."""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def sap():
    import os
    import paper_2506_03070_amd as sap
    if not os.path.exists(sap.LIB_PATH):
        from paper_2506_03070_amd import build
        build.build()
    return sap


def _ceil_ok(got, real):
    # equal to ceil(real); at an exact integer either neighbour is a rounding call
    c = math.ceil(real)
    return got == c or (abs(real - round(real)) <= 1e-9 * max(1.0, real) and got == round(real))


def test_embedding_dim_matches_oracle(sap, orc):
    rng = np.random.default_rng(4501)
    for _ in range(400):
        n = int(rng.integers(1, 20000))
        m = int(n + 1 + 10 ** rng.uniform(0, 8))
        eps = 10 ** rng.uniform(-15, -0.5)
        ratio = 10 ** rng.uniform(-2, 2)
        got = sap.sap_embedding_dim(m, n, eps, ratio)
        real = orc.embedding_dim(m, n, eps, ratio)
        lo, hi = n + 1, min(m, 2 ** 31 - 1)
        if real <= lo:
            assert got == lo
        elif real >= hi:
            assert got == hi
        else:
            assert _ceil_ok(got, real), (m, n, eps, ratio, got, real)


def test_embedding_dim_paper_experiment_range(sap, orc):
    # the Sec. 4.3 experiment: m = 6e5, n from 300 to 5000, eps = 1e-5
    ds = [sap.sap_embedding_dim(600000, n, 1e-5) for n in (300, 1000, 2000, 5000)]
    assert all(d > n for d, n in zip(ds, (300, 1000, 2000, 5000)))
    # d / n falls as n grows (the QR term gains weight)
    ratios = [d / n for d, n in zip(ds, (300, 1000, 2000, 5000))]
    assert all(a > b for a, b in zip(ratios, ratios[1:]))


def test_iteration_estimate_matches_oracle(sap, orc):
    rng = np.random.default_rng(4502)
    for _ in range(400):
        n = int(rng.integers(1, 20000))
        d = int(n + 1 + rng.integers(0, 20 * n + 10))
        eps = 10 ** rng.uniform(-15, -0.5)
        got = sap.sap_iteration_estimate(n, d, eps)
        real = orc.iteration_estimate(n, d, eps)
        if real < 2 ** 31 - 1:
            assert _ceil_ok(got, real), (n, d, eps, got, real)
        else:
            assert got == 2 ** 31 - 1
    assert sap.sap_iteration_estimate(1000, 4000, 1e-12) == 40


@pytest.mark.parametrize("args", [(100, 100, 1e-8, 1.0), (100, 0, 1e-8, 1.0), (1000, 10, 0.0, 1.0),
                                  (1000, 10, 1.0, 1.0), (1000, 10, 1e-8, 0.0), (1000, 10, 1e-8, float("inf")),
                                  (1000, 10, float("nan"), 1.0)])
def test_embedding_dim_errors(sap, args):
    with pytest.raises(sap.SapError) as e:
        sap.sap_embedding_dim(*args)
    assert e.value.status == sap.SAP_EINVAL


@pytest.mark.parametrize("args", [(10, 10, 1e-8), (0, 10, 1e-8), (10, 40, 0.0), (10, 40, 1.5)])
def test_iteration_estimate_errors(sap, args):
    with pytest.raises(sap.SapError) as e:
        sap.sap_iteration_estimate(*args)
    assert e.value.status == sap.SAP_EINVAL
