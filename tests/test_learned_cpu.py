"""CPU pins of the learned selector's references: the FP64 network gradient against central
finite differences, and the label rule against the plain and alpha rules."""
import numpy as np
import pytest

from oracle import mlp as M


def test_mlp_gradient_finite_differences():
    g = np.random.default_rng(0)
    p = g.standard_normal(M.COUNT) * 0.3
    X = g.standard_normal((12, 8))
    y = g.integers(0, 16, 12)
    _, _, grad = M.loss_and_grad(p, X, y)
    idx = g.choice(M.COUNT, 200, replace=False)
    h = 1e-6
    for i in idx:
        e = np.zeros(M.COUNT)
        e[i] = h
        fd = (M.loss_and_grad(p + e, X, y)[0] - M.loss_and_grad(p - e, X, y)[0]) / (2 * h)
        assert abs(fd - grad[i]) <= 1e-7 + 1e-5 * abs(fd), (i, fd, grad[i])


def test_mlp_loss_is_cross_entropy():
    # zero network: uniform softmax over 16 classes, loss log 16 for every sample
    X = np.ones((5, 8))
    loss, losses, _ = M.loss_and_grad(np.zeros(M.COUNT), X, np.arange(5))
    assert np.allclose(losses, np.log(16.0)) and abs(loss - np.log(16.0)) < 1e-15


COST = {1: 0, 2: 1, 4: 2, 8: 3, 12: 4, 18: 5}


def test_label_never_costlier_than_plain(orc):
    g = np.random.default_rng(1)
    for _ in range(3000):
        n1 = float(np.exp(g.uniform(-8, 8)))
        n2 = n1 * n1 * float(g.uniform(0, 1)) ** 2
        n3 = n1 * n2 * float(g.uniform(0, 1)) ** 3
        lm, ls = orc.learned_label(n1, n2, n3)
        pm, ps = orc.select_plain(n1)
        assert COST[lm] + ls <= COST[pm] + ps
        # the label passes the alpha bound with the information used for its degree
        th = dict(zip((1, 2, 4, 8, 12, 18), orc._theta_row(2.0 ** -53)))
        d = orc.alpha_bounds(n1, n2, n3 if lm >= 12 else None)
        eta = min(max(d[p - 1], d[p]) for p in range(1, 5) if p * (p - 1) <= lm + 1)
        assert eta <= th[lm] * 2.0 ** ls


def test_label_matches_alpha_when_a3_is_formed(orc):
    # when the label's degree is >= 12 the learned rule has the same information as alpha
    g = np.random.default_rng(2)
    for _ in range(2000):
        n1 = float(np.exp(g.uniform(-2, 7)))
        n2 = n1 * n1 * float(g.uniform(0.5, 1))
        n3 = n1 * n2 * float(g.uniform(0.5, 1))
        lm, ls = orc.learned_label(n1, n2, n3)
        am, as_ = orc.select_alpha(orc.alpha_bounds(n1, n2, n3))
        if lm >= 12 and am >= 12:
            assert COST[lm] + ls == COST[am] + as_
