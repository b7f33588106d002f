"""Pins of the oracle's diagonal Pade comparison method (Sec. 2, eqs. eq.24, eq.pade10,
eq.pade26; Table 1) against facts independent of it:

* a 1 x 1 input gives p_m(x) / p_m(-x) exactly, summed here in rational arithmetic;
* the definition-based evaluation (plain powers) agrees with the grouped form of eq. eq.pade26
  that the oracle implements separately;
* within its threshold r_2m(X) matches e^X to the backward-error target;
* the thresholds taken (Table 1 less one unit of the third digit) lie below the exact ones and
  within a unit of the printed ones;
* hand-worked cases of the cheapest-cost rule (solve = 4/3 of a product).
"""
from fractions import Fraction
from math import factorial

import numpy as np
import pytest


def _p(m, x):
    return sum(Fraction(factorial(2 * m - j) * factorial(m), factorial(2 * m) * factorial(m - j) * factorial(j))
               * x ** j for j in range(m + 1))


@pytest.mark.parametrize("deg", [10, 26])
@pytest.mark.parametrize("x", [0.3, -1.7, 4.0])
def test_scalar_is_the_rational_function(orc, deg, x):
    m = deg // 2
    X = Fraction(x)
    want = float(_p(m, X) / _p(m, -X))
    got = orc.expm_pade(np.array([[x]]), deg, 0)[0, 0]
    assert abs(got - want) <= 2e-16 * abs(want)


def test_definition_matches_grouped_form(orc):
    g = np.random.default_rng(11)
    for norm in (0.5, 3.0, 40.0):
        A = g.standard_normal((14, 14))
        A *= norm / np.abs(A).sum(0).max()
        E26, s = orc.expm_pade26(A)
        E = orc.expm_pade(A, 26, s)
        assert orc.rel_err_1(E, E26) <= 1e-15


@pytest.mark.parametrize("deg,theta", [(10, 2.53e-1), (26, 5.36)])
def test_accuracy_within_threshold(orc, deg, theta):
    g = np.random.default_rng(deg)
    A = g.standard_normal((12, 12))
    A *= theta / np.abs(A).sum(0).max()
    ref, _ = orc.expm_taylor(A)
    assert orc.rel_err_1(orc.expm_pade(A, deg, 0), ref) <= 2e-15


def test_thresholds_reading(orc):
    from oracle import theta
    printed = {2.0 ** -53: (2.54e-1, 5.37), 2.0 ** -24: (1.88, 11.2)}
    for u, (t10, t26) in orc.PADE_THETA.items():
        for m, t, pr in ((5, t10, printed[u][0]), (13, t26, printed[u][1])):
            exact = theta.pade_theta(m, u)
            assert t <= exact <= 1.02 * t
            assert abs(t - pr) <= 0.0101 * pr


@pytest.mark.parametrize("eta,expect", [(0.1, (10, 0)), (1.0, (10, 2)), (4.0, (26, 0)), (10.0, (26, 1)),
                                        (100.0, (26, 5))])
def test_rule_hand_cases(orc, eta, expect):
    assert orc.select_pade(eta) == expect
