"""Pins of the oracle's 1-norm and alpha_p selection against values worked out by hand.

The 1-norm (Sec. 1: the norm of A drives the choice of (m, s); reading R1: the exact
1-norm, max over columns of the column sums of |a_ij|) and the alpha_p rule (the power-norm
refinement the paper cites in Sec. 1: alpha_p = max(d_p, d_{p+1}), d_k = ||A^k||_1^(1/k),
admissible when p (p - 1) <= m + 1, then the thresholds of Table 2 with the cheapest
products + s, eq. eq.theta) are checked here on inputs whose every quantity is known in
closed form.  Each case is chosen so that a plausible slip fails it: rows summed instead of
columns, min instead of max, |re| + |im| instead of |z|, d_p alone instead of
max(d_p, d_{p+1}), or the admissibility bound on p ignored.
"""
import math

import numpy as np
import pytest

# Table 2, u = 2^-53 (theta_m for m = 1, 2, 4, 8, 12, 18), to the digits printed there
TH = {1: 2.22e-16, 2: 2.58e-8, 4: 3.40e-4, 8: 4.99e-2, 12: 2.99e-1, 18: 1.09}


def test_norm1_columns_not_rows(orc):
    # column sums |-1| + |-2| = 3 and 8 + 0.5 = 8.5; the row sums would be 9 and 2.5
    A = np.array([[-1.0, 8.0], [-2.0, 0.5]])
    assert orc.norm1(A) == 8.5
    # one full row: column sums 1, 2, 3 (max 3); its row sum would be 6
    B = np.zeros((3, 3))
    B[0] = [1.0, -2.0, 3.0]
    assert orc.norm1(B) == 3.0
    # the largest column, not the smallest
    C = np.diag([0.25, -7.0, 2.0])
    assert orc.norm1(C) == 7.0
    assert orc.norm1(np.zeros((4, 4))) == 0.0


def test_norm1_complex_uses_modulus(orc):
    # |3 + 4i| + |i| = 6 in column 0, 1 in column 1; |re| + |im| would give 8, a row sum 5
    A = np.array([[3 + 4j, 0.0], [1j, 1.0]])
    assert orc.norm1(A) == 6.0
    B = np.array([[0.0, -5 + 12j], [0.0, 0.0]])  # |-5 + 12i| = 13
    assert orc.norm1(B) == 13.0


def test_rel_err_1_by_hand(orc):
    R = np.array([[-1.0, 8.0], [-2.0, 0.5]])
    X = R.copy()
    X[1, 0] += 0.25  # difference: one entry 0.25 in column 0
    assert orc.rel_err_1(X, R) == 0.25 / 8.5


def _hand_s(eta, theta):
    # smallest s >= 0 with eta / 2^s <= theta, counted by halving
    s = 0
    while eta > theta * 2.0 ** s:
        s += 1
    return s


def test_powers_norms_antidiagonal(orc):
    # A = [[0, 8], [1/8, 0]]: A^2 = I, so ||A^k||_1 alternates 8, 1, 8, 1, 8
    A = np.array([[0.0, 8.0], [0.125, 0.0]])
    assert list(orc.powers_norms(A, 5)) == [8.0, 1.0, 8.0, 1.0, 8.0]


def test_alpha_rule_takes_the_max_of_neighbours(orc):
    # d = (8, 1, 2, 1, 8^(1/5)): d_2 < d_3, so alpha_2 = alpha_3 = 2 while d_2 = 1.
    # Admissible for m = 18 (and 12): p <= 4, so eta_18 = min(8, 2, 2, 8^(1/5)) = 8^(1/5) = 1.516,
    # which lies in (theta_18, 2 theta_18]: s = 1, cost 5 + 1 = 6.  m = 12: 1.516 / 0.2996 > 4,
    # s = 3, cost 7.  m = 8 (p <= 3): eta = 2, s = 6, cost 9.  So (18, 1).
    A = np.array([[0.0, 8.0], [0.125, 0.0]])
    nk = orc.powers_norms(A, 5)
    d = [nk[k] ** (1.0 / (k + 1)) for k in range(5)]
    assert d[:4] == [8.0, 1.0, 2.0, 1.0]
    assert _hand_s(8.0 ** 0.2, TH[18]) == 1 and _hand_s(8.0 ** 0.2, TH[12]) == 3
    assert orc.select_alpha(d) == (18, 1)
    # taking min(d_p, d_{p+1}) or d_p alone would give eta_18 = 1 <= theta_18: (18, 0)
    # the plain rule: eta = 8, s = 3 at m = 18
    assert orc.select_plain(8.0) == (18, 3)
    assert _hand_s(8.0, TH[18]) == 3


def test_alpha_rule_respects_admissible_p(orc):
    # N = shift with entries 1 on the superdiagonal of a 3 x 3 block: N^2 != 0, N^3 = 0, so
    # d = (1, 1, 0, 0, 0).  m = 1 admits p <= 2 only (p (p - 1) <= 2): eta_1 = max(d_2, d_3) = 1,
    # far above theta_1.  m = 2 and m = 4 admit p <= 2: eta = 1, s = 26 and 12.  m = 8 admits
    # p = 3: alpha_3 = max(d_3, d_4) = 0, so s = 0 at cost 3.  The choice is (8, 0), and
    # T_8(N) = I + N + N^2 / 2 = e^N exactly.  Ignoring the bound on p would allow (1, 0)
    # (alpha_3 = 0 at m = 1), and T_1(N) = I + N is wrong in its (0, 2) entry.
    N = np.zeros((3, 3))
    N[0, 1] = N[1, 2] = 1.0
    nk = orc.powers_norms(N, 5)
    assert list(nk) == [1.0, 1.0, 0.0, 0.0, 0.0]
    d = [nk[k] ** (1.0 / (k + 1)) for k in range(5)]
    assert _hand_s(1.0, TH[2]) == 26 and _hand_s(1.0, TH[4]) == 12
    assert orc.select_alpha(d) == (8, 0)
    E, _ = orc.expm_taylor(N)
    want = np.eye(3) + N + 0.5 * (N @ N)
    assert np.array_equal(E, want)


@pytest.mark.parametrize("a,b", [(8.0, 0.125), (64.0, 1.0 / 64.0), (2.0, 2.0)])
def test_alpha_bounds_of_known_powers(orc, a, b):
    # A = [[0, a], [b, 0]]: A^2 = ab I, so ||A^2|| = ab and ||A^3|| = ab max(a, b); the
    # submultiplicative bounds of d_4, d_5 are then ||A^4|| <= (ab)^2 and
    # ||A^5|| <= min(ab * ab max(a, b), (ab)^2 max(a, b)) = (ab)^2 max(a, b), both exact here.
    n1, n2, n3 = max(a, b), a * b, a * b * max(a, b)
    d = orc.alpha_bounds(n1, n2, n3)
    assert d[0] == n1
    assert math.isclose(d[1], math.sqrt(a * b), rel_tol=1e-15)
    assert math.isclose(d[2], n3 ** (1 / 3), rel_tol=1e-15)
    assert math.isclose(d[3], math.sqrt(a * b), rel_tol=1e-15)
    assert math.isclose(d[4], ((a * b) ** 2 * max(a, b)) ** 0.2, rel_tol=1e-15)
    A = np.array([[0.0, a], [b, 0.0]])
    nk = orc.powers_norms(A, 5)
    exact = [nk[k] ** (1.0 / (k + 1)) for k in range(5)]
    assert np.allclose(exact, d, rtol=1e-15, atol=0)
