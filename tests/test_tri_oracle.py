"""Pins of the oracle's triangular refinement (concluding remarks) against facts independent
of it:

* for a 2 x 2 upper triangular A every entry of the result is overwritten, so the refined
  method returns e^A itself, here from mpmath at 40 digits (distinct and equal diagonal
  entries, so both branches of the superdiagonal formula are exercised);
* for a larger triangular A with a wide spread of diagonal entries and many squarings, the
  refined diagonal is e^(a_ii) to rounding, entry by entry, and the result stays within the
  method's error of the long-double direct Taylor reference.
"""
import mpmath
import numpy as np
import pytest


@pytest.mark.parametrize("a,b,c", [(-3.0, 2.5, 1.25), (0.5, -7.0, 0.5), (-20.0, 4.0, -0.001), (12.0, 1.0, -9.0)])
def test_two_by_two_is_exact(orc, a, b, c):
    A = np.array([[a, b], [0.0, c]])
    m, s = orc.select_plain(orc.norm1(A))
    E = orc.expm_reduced_tri(A, m, s)
    with mpmath.workdps(40):
        R = mpmath.expm(mpmath.matrix([[a, b], [0, c]]))
        R = np.array([[float(R[i, j]) for j in range(2)] for i in range(2)])
    assert np.all(np.abs(E - R) <= 2e-16 * np.abs(R) + 1e-300), (E, R)


def test_spread_diagonal(orc):
    g = np.random.default_rng(3)
    n = 24
    A = np.triu(g.standard_normal((n, n)))
    A[np.diag_indices(n)] = -np.linspace(0.0, 30.0, n)
    m, s = orc.select_plain(orc.norm1(A))
    assert s >= 4
    E = orc.expm_reduced_tri(A, m, s)
    d = np.exp(np.diag(A))
    assert np.all(np.abs(np.diag(E) - d) <= 2e-16 * d)
    assert np.all(np.tril(E, -1) == 0.0)
    ref, _ = orc.expm_taylor(A)
    assert orc.rel_err_1(E, ref) <= 1e-13
