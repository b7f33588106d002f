"""Backward-error thresholds theta_m(u) (test infrastructure; see the package docstring).

Definition followed (Sec. 1, eq. eq.theta and the paragraph after it): for an approximant r
of e^x, write rho(x) = log(e^{-x} r(x)) = sum_i c_i x^i; with f(theta) = sum_i |c_i| theta^i
(series cut after 150 terms), theta(u) is the root of f(theta) / theta = u.  Then every A
with ||A|| <= theta has r(A) = e^{A+E} with ||E|| / ||A|| <= u.

The series is computed exactly in rational arithmetic (``fractions.Fraction``): the product
e^{-x} r(x) term by term, then the logarithm of a power series with constant term 1 by the
recurrence obtained from g h' = g' (h = log g).  The root is found by bisection in 60-digit
mpmath arithmetic.  Nothing here is shared with the GPU library, which derives its own
thresholds.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial

import mpmath

NTERMS = 150          # the series is cut after this many terms (Sec. 1)
TAYLOR_DEGREES = (1, 2, 4, 8, 12, 18)


def _exp_neg(K):
    """Coefficients of e^{-x} up to x^K."""
    return [Fraction((-1) ** i, factorial(i)) for i in range(K + 1)]


def _mul(a, b, K):
    out = [Fraction(0)] * (K + 1)
    for i, ai in enumerate(a):
        if ai == 0:
            continue
        for j in range(0, K + 1 - i):
            if j < len(b) and b[j] != 0:
                out[i + j] += ai * b[j]
    return out


def _log1p_series(g, K):
    """log g for a power series g with g[0] = 1: h_n = g_n - (1/n) sum_{k<n} k h_k g_{n-k}."""
    assert g[0] == 1
    h = [Fraction(0)] * (K + 1)
    for n in range(1, K + 1):
        acc = Fraction(0)
        for k in range(1, n):
            if h[k] != 0 and g[n - k] != 0:
                acc += k * h[k] * g[n - k]
        h[n] = g[n] - acc / n
    return h


def _series_div(p, q, K):
    """p / q as a power series (q[0] != 0)."""
    out = [Fraction(0)] * (K + 1)
    for n in range(K + 1):
        acc = p[n] if n < len(p) else Fraction(0)
        for k in range(1, n + 1):
            if k < len(q) and q[k] != 0:
                acc -= q[k] * out[n - k]
        out[n] = acc / q[0]
    return out


@lru_cache(maxsize=None)
def taylor_rho(m):
    """(first, coeffs): c_i of rho for T_m(x) = sum_{k<=m} x^k/k!, i = first .. first+NTERMS-1."""
    first = m + 1
    K = first + NTERMS - 1
    tm = [Fraction(1, factorial(k)) for k in range(m + 1)]
    g = _mul(_exp_neg(K), tm, K)
    h = _log1p_series(g, K)
    assert all(c == 0 for c in h[1:first]), "rho must start at x^(m+1)"
    return first, tuple(h[first:K + 1])


@lru_cache(maxsize=None)
def pade_rho(m):
    """Same for the diagonal Pade r_2m = p_m(x)/p_m(-x), p_m from eq. eq.24; starts at x^(2m+1)."""
    first = 2 * m + 1
    K = first + NTERMS - 1
    p = [Fraction(factorial(2 * m - j) * factorial(m), factorial(2 * m) * factorial(m - j) * factorial(j))
         for j in range(m + 1)]
    pneg = [c * (-1) ** j for j, c in enumerate(p)]
    r = _series_div(p, pneg, K)
    g = _mul(_exp_neg(K), r, K)
    h = _log1p_series(g, K)
    assert all(c == 0 for c in h[1:first]), "rho must start at x^(2m+1)"
    return first, tuple(h[first:K + 1])


def _solve(first, coeffs, u, dps=60):
    with mpmath.workdps(dps):
        ab = [mpmath.mpf(abs(c.numerator)) / abs(c.denominator) for c in coeffs]
        u = mpmath.mpf(u)

        def g(t):  # f(t)/t - u, increasing in t
            return mpmath.fsum(a * t ** (first + i - 1) for i, a in enumerate(ab)) - u

        lo, hi = mpmath.mpf(0), mpmath.mpf(1)
        while g(hi) < 0:
            lo, hi = hi, hi * 2
        for _ in range(200):
            mid = (lo + hi) / 2
            if g(mid) < 0:
                lo = mid
            else:
                hi = mid
        return lo


@lru_cache(maxsize=None)
def taylor_theta(m, u):
    """theta_m(u) for the Taylor polynomial of degree m (a float, rounded toward zero)."""
    first, c = taylor_rho(m)
    t = _solve(first, c, u)
    return float(mpmath.mpf(t) * (1 - mpmath.mpf(2) ** -60))


@lru_cache(maxsize=None)
def pade_theta(m, u):
    """theta_2m(u) for the diagonal Pade approximant r_2m."""
    first, c = pade_rho(m)
    t = _solve(first, c, u)
    return float(mpmath.mpf(t) * (1 - mpmath.mpf(2) ** -60))


def taylor_thetas(u):
    """[theta_m(u) for m in (1, 2, 4, 8, 12, 18)]."""
    return [taylor_theta(m, u) for m in TAYLOR_DEGREES]


def backward_bound(m, x):
    """f(x)/x = sum |c_i| x^(i-1): the relative backward-error bound at ||X|| = x."""
    first, c = taylor_rho(m)
    with mpmath.workdps(40):
        return float(mpmath.fsum(mpmath.mpf(abs(ci.numerator)) / abs(ci.denominator) * mpmath.mpf(x) ** (first + i - 1)
                                 for i, ci in enumerate(c)))
