"""Pins for the oracle's sparse sign sketch (Def. 2.2, Sec. 3.1.2, Alg. 3):
exact structural invariants, uniformity over all zeta-subsets (chi-square on
tiny d), marginal and pairwise inclusion probabilities, the round-0
acceptance probability of eq. (3.2), and the moments of S^T S and S S^T."""
import itertools
import math

import numpy as np
import pytest
from scipy import stats


def _columns(orc, seed, m, d, zeta, stream=0):
    idx, sign, rounds = orc.sketch(seed, stream, m, d, zeta, want_rounds=True)
    return idx, sign, rounds


@pytest.mark.parametrize("d,zeta", [(1, 1), (2, 2), (5, 5), (6, 3), (64, 64), (400, 8), (4000, 8),
                                    (8192, 8), (100, 24), (70, 64), (2**31 - 1, 8)])
def test_structure(orc, d, zeta):
    m = 3000 if d > 64 else 500
    idx, sign, rounds = _columns(orc, 17, m, d, zeta)
    assert idx.shape == (m, zeta)
    assert (idx >= 0).all() and (idx < d).all()
    assert (np.diff(idx.astype(np.int64), axis=1) > 0).all()  # strictly ascending -> distinct
    if zeta < 64:
        assert (sign >> np.uint64(zeta) == 0).all()
    if zeta == d:
        assert (idx == np.arange(d)[None, :]).all()


def test_invalid_parameters(orc):
    for d, zeta in [(3, 4), (100, 0), (100, 65)]:
        with pytest.raises(ValueError):
            orc.sketch_column(1, 0, 0, d, zeta)


def test_columns_are_independent_of_m(orc):
    """Column i depends only on (seed, stream, i): a prefix of a longer sketch
    equals a shorter sketch, and single columns match."""
    a, sa = orc.sketch(5, 2, 100, 400, 8)
    b, sb = orc.sketch(5, 2, 300, 400, 8)
    assert (a == b[:100]).all() and (sa == sb[:100]).all()
    for i in (0, 57, 299):
        col, s, _ = orc.sketch_column(5, 2, i, 400, 8)
        assert (col == b[i]).all() and s == int(sb[i])
    c, _ = orc.sketch(5, 3, 100, 400, 8)
    assert (c != a).any()


@pytest.mark.parametrize("d,zeta", [(6, 3), (8, 3), (10, 4)])
def test_uniform_over_subsets(orc, d, zeta):
    """Def. 2.2 asks for zeta distinct rows in uniformly random coordinates:
    every one of the C(d, zeta) subsets must be equally likely."""
    cells = math.comb(d, zeta)
    m = 400 * cells
    idx, _, rounds = _columns(orc, 1234 + d, m, d, zeta)
    index = {c: k for k, c in enumerate(itertools.combinations(range(d), zeta))}
    counts = np.zeros(cells)
    for row in idx:
        counts[index[tuple(int(v) for v in row)]] += 1
    chi2, p = stats.chisquare(counts)
    assert p > 1e-3, (chi2, p)
    # the rejection loop did fire (otherwise the test would be vacuous)
    assert (rounds > 0).mean() > 0.2


def test_marginal_and_pairwise_inclusion(orc):
    d, zeta, m = 40, 8, 60000
    idx, _, _ = _columns(orc, 77, m, d, zeta)
    inc = np.zeros((m, d), dtype=bool)
    inc[np.arange(m)[:, None], idx] = True
    p1 = inc.mean(axis=0)
    se1 = math.sqrt(zeta / d * (1 - zeta / d) / m)
    assert np.abs(p1 - zeta / d).max() < 5 * se1
    pair = (inc[:, :, None] & inc[:, None, :]).mean(axis=0)
    q = zeta * (zeta - 1) / (d * (d - 1))
    off = pair[~np.eye(d, dtype=bool)]
    assert abs(off.mean() - q) < 5 * math.sqrt(q / (m * d * (d - 1) / 2))
    assert np.abs(off - q).max() < 6 * math.sqrt(q * (1 - q) / m)


@pytest.mark.parametrize("d,zeta", [(6, 3), (50, 8), (400, 8), (4000, 8)])
def test_round0_acceptance_eq_3_2(orc, d, zeta):
    """Eq. (3.2): a with-replacement draw of zeta values is repeat-free with
    probability p = prod_{k<zeta} (1 - k/d) >= 1 - zeta^2/d."""
    m = 40000 if d < 1000 else 200000
    _, _, rounds = _columns(orc, 4242 + d, m, d, zeta)
    p = float(np.prod(1.0 - np.arange(zeta) / d))
    assert p >= 1.0 - zeta * zeta / d
    accepted = int((rounds == 0).sum())
    res = stats.binomtest(accepted, m, p)
    assert res.pvalue > 1e-3, (accepted / m, p)


def test_signs_fair_and_scaled(orc):
    d, zeta, m = 400, 8, 50000
    idx, sign, _ = _columns(orc, 31, m, d, zeta)
    vals = orc.sign_values(sign, zeta)
    plus = int((vals > 0).sum())
    assert stats.binomtest(plus, m * zeta, 0.5).pvalue > 1e-3
    h = orc.sketch_scale(zeta)
    # diag(S^T S) = zeta * h^2 = 1 up to one rounding per term
    col_sq = np.sum((vals * h) ** 2, axis=1)
    assert np.abs(col_sq - 1.0).max() <= zeta * np.finfo(float).eps


def test_gram_moments(orc):
    """E[S^T S] = I (off-diagonal mean 0, variance 1/d) and E[S S^T] = (m/d) I."""
    d, zeta, m = 200, 8, 4000
    idx, sign, _ = _columns(orc, 8, m, d, zeta)
    S = orc.dense_sketch(idx, sign, d, zeta)
    G = S.T @ S
    off = G[~np.eye(m, dtype=bool)]
    assert abs(off.mean()) < 5 * math.sqrt(1.0 / d / off.size) * 10
    assert abs(off.var() - 1.0 / d) < 0.05 / d
    H = S @ S.T
    assert abs(np.trace(H) - m) < 1e-9 * m  # every column has unit norm
    diag = np.diag(H)
    assert abs(diag.mean() - m / d) < 1e-9 * m
    # row loads are Binomial(m, zeta/d) times h^2
    counts = diag * zeta
    assert abs(counts.var() - m * (zeta / d) * (1 - zeta / d)) < 0.3 * m * zeta / d


def numpy_alg3_twin(rng, d, m, zeta):
    """Alg. 3 run with NumPy's own generator (a distributional twin: same law,
    different stream)."""
    C = rng.integers(0, d, size=(m, zeta))
    C.sort(axis=1)
    bi, bj = np.where(C[:, 1:] == C[:, :-1])
    while len(bj) > 0:
        C[bi, bj] = rng.integers(0, d, size=len(bj))
        bad = np.unique(bi)
        C[bad] = np.sort(C[bad], axis=1)
        bi, bj = np.where(C[bad, 1:] == C[bad, :-1])
        bi = bad[bi]
    return C


def test_same_law_as_alg3_twin(orc):
    d, zeta = 8, 3
    cells = math.comb(d, zeta)
    m = 300 * cells
    idx, _, _ = _columns(orc, 5150, m, d, zeta)
    twin = numpy_alg3_twin(np.random.default_rng(3), d, m, zeta)
    index = {c: k for k, c in enumerate(itertools.combinations(range(d), zeta))}
    a = np.zeros(cells)
    b = np.zeros(cells)
    for row in idx:
        a[index[tuple(int(v) for v in row)]] += 1
    for row in twin:
        b[index[tuple(int(v) for v in row)]] += 1
    _, p, _, _ = stats.chi2_contingency(np.vstack([a, b]))
    assert p > 1e-3
