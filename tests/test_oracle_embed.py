"""Pins for the oracle's embedding-dimension selection (Sec. 4.3): the
Lambert W function against SciPy and its closed forms, eq. (4.2) against the
cost balance the paper states it implies, and eq. (4.1) against its own
condition-number form."""
import math

import numpy as np
import pytest
from scipy.special import lambertw


@pytest.mark.parametrize("z", [0.0, 1e-12, 1e-3, 0.5, 1.0, math.e, 10.0, 138.2, 1e4, 1e8, 1e15])
def test_lambert_w0_matches_scipy(orc, z):
    w = orc.lambert_w0(z)
    ref = float(lambertw(z, 0).real)
    assert abs(w - ref) <= 1e-13 * max(1.0, abs(ref))
    assert abs(w * math.exp(w) - z) <= 1e-12 * max(1.0, z)


def test_lambert_w0_closed_forms(orc):
    # W(0) = 0, W(e) = 1, W(2 e^2) = 2, W(k e^k) = k
    assert abs(orc.lambert_w0(0.0)) <= 1e-15
    for k in (1.0, 2.0, 5.0, 0.25):
        assert abs(orc.lambert_w0(k * math.exp(k)) - k) <= 1e-13 * k
    assert math.isnan(orc.lambert_w0(-0.1))


@pytest.mark.parametrize("m,n,eps,ratio", [(600000, 300, 1e-5, 1.0), (600000, 5000, 1e-5, 1.0),
                                           (1 << 20, 1000, 1e-12, 1.0), (1 << 22, 4096, 1e-8, 0.5),
                                           (20000, 100, 1e-12, 2.0)])
def test_embedding_dim_balances_costs(orc, m, n, eps, ratio):
    """Eq. (4.2) states that its d makes the iteration work
    (log eps / log(n/d)) m n equal to the QR work d n^2; a wrong sign or a
    dropped factor in the W form breaks the equality."""
    d = orc.embedding_dim(m, n, eps, ratio)
    assert d > n
    it_cost = ratio * math.log(eps) / math.log(n / d) * m * n
    qr_cost = d * n * n
    assert abs(it_cost - qr_cost) <= 1e-10 * qr_cost


def test_embedding_dim_special_case(orc):
    # m chosen so that -m log(eps) / n^2 = e: W = 1 and d = e n
    n, eps = 200, 1e-6
    m = n * n * math.e / -math.log(eps)
    mi = int(round(m))
    z = -mi * math.log(eps) / (n * n)
    w = float(lambertw(z, 0).real)
    assert abs(orc.embedding_dim(mi, n, eps) - n * math.exp(w)) <= 1e-11 * n * math.exp(w)
    assert abs(w - 1.0) < 1e-3


def test_embedding_dim_monotone(orc):
    # more rows or a tighter eps make iterations dearer: larger d
    ds_m = [orc.embedding_dim(m, 500, 1e-8) for m in (10000, 100000, 1000000, 10000000)]
    assert all(a < b for a, b in zip(ds_m, ds_m[1:]))
    ds_e = [orc.embedding_dim(10 ** 6, 500, e) for e in (1e-2, 1e-5, 1e-8, 1e-12)]
    assert all(a < b for a, b in zip(ds_e, ds_e[1:]))
    # and a cheaper iteration (ratio < 1) a smaller d
    assert orc.embedding_dim(10 ** 6, 500, 1e-8, 0.5) < orc.embedding_dim(10 ** 6, 500, 1e-8, 1.0)


@pytest.mark.parametrize("n,d,eps", [(1000, 4000, 1e-12), (100, 400, 1e-10), (4096, 8192, 1e-8), (50, 2000, 1e-5)])
def test_iteration_estimate(orc, n, d, eps):
    """Eq. (4.1): (n/d)^(t/2) = ((kappa - 1)/(kappa + 1))^t with
    kappa = (1 + sqrt(n/d)) / (1 - sqrt(n/d)); at the estimate both equal eps."""
    t = orc.iteration_estimate(n, d, eps)
    r = math.sqrt(n / d)
    kappa = (1 + r) / (1 - r)
    assert abs(((kappa - 1) / (kappa + 1)) ** t - eps) <= 1e-9 * eps
    assert abs((n / d) ** (t / 2) - eps) <= 1e-9 * eps


def test_iteration_estimate_closed_form(orc):
    # d = 4n, eps = 1e-12: t = 2 ln(1e-12) / ln(1/4) = 12 ln 10 / ln 2
    assert abs(orc.iteration_estimate(1000, 4000, 1e-12) - 12 * math.log(10) / math.log(2)) <= 1e-12
