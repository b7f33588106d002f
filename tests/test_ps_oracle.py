"""Pins of the oracle's Paterson-Stockmeyer comparison method (Sec. 4, eq. poli9, Tables 2-3)
against facts independent of it:

* the truncated series on a diagonal matrix equals the scalar truncated series, summed here in
  exact rational arithmetic;
* on the shift matrix N (N^k has ones on the k-th superdiagonal) the k-th superdiagonal of
  T_m(x N) is x^k / k! for k <= m and exactly zero beyond;
* the paper's T_8 is the degree-8 Taylor polynomial exactly and T_12 up to its printed
  decimals, so the oracle's product-reduced evaluation agrees with the plain series;
* the thresholds of the degrees 6, 9 and 16 reproduce the hidden columns of Table 2;
* hand-worked cases of the cheapest-cost rule over the degrees of Table 3.
"""
from fractions import Fraction

import numpy as np
import pytest


def test_diagonal_equals_scalar_series(orc):
    vals = [-1.5, 1.0 / 3.0, 1.4, 0.0, -0.125]
    d = [Fraction(v) for v in vals]  # the exact values of the doubles
    D = np.diag(vals)
    for m in (1, 2, 4, 6, 9, 12, 16):
        T = orc.taylor_poly(D, m)
        for i, x in enumerate(d):
            want = sum(x ** k / Fraction(_fact(k)) for k in range(m + 1))
            assert abs(float(T[i, i]) - float(want)) <= 1e-17 * max(1.0, abs(float(want)))
        assert np.all(T[~np.eye(5, dtype=bool)] == 0)


def _fact(k):
    f = 1
    for j in range(2, k + 1):
        f *= j
    return f


def test_shift_matrix_gives_the_coefficients(orc):
    n = 20
    N = np.diag(np.ones(n - 1), 1)
    x = 0.75
    for m in (6, 9, 16):
        T = orc.taylor_poly(x * N, m)
        for k in range(n):
            diag = np.diagonal(T, k).astype(np.float64)
            want = float(Fraction(3, 4) ** k / Fraction(_fact(k))) if k <= m else 0.0
            if k <= m:
                assert np.all(np.abs(diag - want) <= 1e-18 + 1e-17 * want), (m, k)
            else:
                assert np.all(diag == 0.0), (m, k)


@pytest.mark.parametrize("m,tol", [(8, 1e-15), (12, 1e-15)])
def test_reduced_sequences_equal_the_plain_series(orc, m, tol):
    g = np.random.default_rng(m)
    X = g.standard_normal((12, 12))
    X *= 0.25 / np.abs(X).sum(0).max()
    R, _ = orc.reduced_Tm(X, m)
    P = orc.taylor_poly(X, m).astype(np.float64)
    assert np.abs(R - P).max() <= tol


def test_thresholds_of_the_hidden_columns(orc):
    from oracle import theta
    # Table 2: u = 2^-53 row, degrees 6, 9, 16: 9.07e-3, 8.96e-2, 7.80e-1; u = 2^-24 row:
    # 2.50e-1 (exponent garbled in the text, reading R3), 7.80e-1, 2.48
    for m, u, printed in ((6, 2.0 ** -53, 9.07e-3), (9, 2.0 ** -53, 8.96e-2), (16, 2.0 ** -53, 7.80e-1),
                          (6, 2.0 ** -24, 2.50e-1), (9, 2.0 ** -24, 7.80e-1), (16, 2.0 ** -24, 2.48)):
        t = theta.taylor_theta(m, u)
        assert abs(t - printed) <= 0.0051 * printed, (m, u, t)


@pytest.mark.parametrize("eta,expect", [
    (1e-17, (1, 0)), (1e-9, (2, 0)), (1e-4, (4, 0)),
    (5e-3, (6, 0)),    # (4, 1) costs 3 as well: the tie goes to s = 0
    (0.05, (9, 0)),
    (0.2, (12, 0)),    # (9, 1) also costs 5
    (0.5, (16, 0)),
    (2.0, (16, 2)),    # (12, 3) also costs 8
    (100.0, (16, 8))])
def test_rule_hand_cases(orc, eta, expect):
    assert orc.select_ps(eta) == expect


def test_method_output_is_squared_series(orc):
    g = np.random.default_rng(4)
    A = g.standard_normal((10, 10))
    A *= 3.0 / np.abs(A).sum(0).max()
    m, s = orc.select_ps(orc.norm1(A))
    E = orc.expm_ps(A, m, s)
    ref, _ = orc.expm_taylor(A)
    assert orc.rel_err_1(E, ref) <= 1e-14
