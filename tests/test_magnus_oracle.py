"""Pins of the oracle's fourth-order Magnus step (exponential integrators of the concluding
remarks) against facts independent of it:

* commuting case F(t) = (1 + u(t)) S with a cubic control: the two-point Gauss rule integrates
  cubics exactly and the commutator vanishes, so one step equals expm((h + int u) S) Y,
  computed here with scipy's Pade-based expm;
* S1 = 0: one step is e^{h S0} Y;
* skew-symmetric S0, S1: the step is orthogonal, so an orthogonal state stays orthogonal;
* global error of order h^4 against scipy's DOP853 integration of the same ODE (a dropped or
  sign-flipped commutator term lowers the order to 2, which this catches).
"""
import numpy as np
import pytest
import scipy.integrate
import scipy.linalg

from paper_1710_10989_amd import workloads as W


def _skew(g, n, norm):
    G = g.standard_normal((n, n))
    S = G - G.T
    return S * (norm / np.abs(S).sum(0).max())


def test_commuting_cubic_control_is_exact(orc):
    g = np.random.default_rng(5)
    n = 9
    S = g.standard_normal((n, n)) * 0.3
    Y = g.standard_normal((n, n))
    c = g.standard_normal(4)  # u(t) = c0 + c1 t + c2 t^2 + c3 t^3
    u = lambda t: c[0] + c[1] * t + c[2] * t ** 2 + c[3] * t ** 3
    U = lambda t: c[0] * t + c[1] * t ** 2 / 2 + c[2] * t ** 3 / 3 + c[3] * t ** 4 / 4
    t0, h = 0.3, 0.4
    r = np.sqrt(3.0) / 6.0
    u1, u2 = u(t0 + (0.5 - r) * h), u(t0 + (0.5 + r) * h)
    got, _ = orc.magnus4_step(S, S, Y, u1, u2, h)
    want = scipy.linalg.expm((h + U(t0 + h) - U(t0)) * S) @ Y
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_no_control_is_one_exponential(orc):
    g = np.random.default_rng(6)
    S0 = g.standard_normal((12, 12))
    Y = g.standard_normal((12, 12))
    got, Om = orc.magnus4_step(S0, np.zeros_like(S0), Y, 0.7, -1.3, 0.25)
    assert np.array_equal(Om, 0.25 * S0)
    want = scipy.linalg.expm(0.25 * S0) @ Y
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()


def test_skew_step_keeps_orthogonality(orc):
    S0, S1, Y0, a, w, phi = W.magnus_systems(count=4, n=16)
    for b in range(4):
        Y = Y0[b]
        for k in range(10):
            u1, u2 = W.control_at_gauss_points(a[b], w[b], phi[b], 0.1 * k, 0.1)
            Y, _ = orc.magnus4_step(S0[b], S1[b], Y, u1, u2, 0.1)
        assert np.abs(Y.T @ Y - np.eye(16)).max() <= 1e-13


def test_fourth_order_convergence(orc):
    g = np.random.default_rng(7)
    n = 6
    S0, S1 = _skew(g, n, 1.5), _skew(g, n, 2.0)
    Y0 = np.eye(n)
    a, w, phi = 1.3, 3.0, 0.4
    u = lambda t: a * np.cos(w * t + phi)

    def rhs(t, y):
        return ((S0 + u(t) * S1) @ y.reshape(n, n)).ravel()

    ref = scipy.integrate.solve_ivp(rhs, (0.0, 1.0), Y0.ravel(), method="DOP853", rtol=1e-13, atol=1e-14)
    Yref = ref.y[:, -1].reshape(n, n)

    def integrate(N):
        h = 1.0 / N
        Y = Y0
        for k in range(N):
            u1, u2 = W.control_at_gauss_points(a, w, phi, k * h, h)
            Y, _ = orc.magnus4_step(S0, S1, Y, u1, u2, h)
        return np.abs(Y - Yref).max()

    e1, e2 = integrate(16), integrate(32)
    assert 1e-12 < e2 < e1
    assert 12.0 <= e1 / e2 <= 20.0, (e1, e2)


@pytest.mark.parametrize("h", [0.05, 0.1, 0.2])
def test_workload_norms_stay_in_the_low_degree_regime(orc, h):
    # the default Magnus workload (||S0|| = 2, ||S1|| = 1, |u| <= 2) keeps ||Omega||_1 small:
    # the plain rule picks a degree <= 18 with no or one squaring
    S0, S1, Y0, a, w, phi = W.magnus_systems(count=64, n=16)
    for b in range(64):
        u1, u2 = W.control_at_gauss_points(a[b], w[b], phi[b], 0.0, h)
        Om = orc.magnus4_omega(S0[b], S1[b], u1, u2, h)
        m, s = orc.select_plain(orc.norm1(Om))
        assert m <= 18 and s <= 1
