"""Pins of the oracle's e^A applied to sampled columns (the series sum_k A^k e_j / k! of Sec. 1,
no scaling), used at orders where forming e^A on the CPU is too slow: closed forms, and
agreement with the oracle's separately written scaling-and-squaring direct Taylor routine."""
import math

import numpy as np


def test_diagonal_columns(orc):
    d = np.array([-30.0, -2.5, 0.0, 0.7, 12.0])
    C = orc.expm_columns(np.diag(d), [0, 1, 3, 4])
    for c, j in enumerate([0, 1, 3, 4]):
        want = np.zeros(5)
        want[j] = math.exp(d[j])
        assert np.allclose(C[:, c], want, rtol=1e-15, atol=0), j


def test_rotation_generator(orc):
    # e^[[0, -t], [t, 0]] = [[cos t, -sin t], [sin t, cos t]]; a large t needs many terms
    for t in (0.3, 7.0, 40.0):
        C = orc.expm_columns(np.array([[0.0, -t], [t, 0.0]]), [0, 1])
        want = np.array([[math.cos(t), -math.sin(t)], [math.sin(t), math.cos(t)]])
        assert np.allclose(C, want, rtol=0, atol=1e-14), t


def test_nilpotent_terminates_exactly(orc):
    # strictly upper triangular with small integer entries: the series ends at N^(n-1) and
    # every term is a dyadic rational here, so the columns are exact
    N = np.triu(np.array([[0, 2, -1, 4], [0, 0, 2, 1], [0, 0, 0, -2], [0, 0, 0, 0]], dtype=float), 1)
    want = np.eye(4) + N + N @ N / 2 + N @ N @ N / 6
    assert np.array_equal(orc.expm_columns(N, [0, 1, 2, 3]), want)


def test_complex_unitary_columns(orc):
    # -i H t with H Hermitian: the columns of e^(-iHt) are orthonormal
    g = np.random.default_rng(4)
    G = g.standard_normal((12, 12)) + 1j * g.standard_normal((12, 12))
    H = (G + G.conj().T) / 2
    C = orc.expm_columns(-1j * H * 3.0, list(range(12)))
    assert np.abs(C.conj().T @ C - np.eye(12)).max() <= 1e-13


def test_agrees_with_scaling_and_squaring_oracle(orc):
    g = np.random.default_rng(8)
    for n, norm in ((30, 0.5), (50, 20.0), (64, 60.0)):
        A = g.standard_normal((n, n)) / np.sqrt(n)
        A *= norm / np.abs(A).sum(0).max()
        E, _ = orc.expm_taylor(A)
        cols = [0, n // 2, n - 1]
        C = orc.expm_columns(A, cols)
        err = np.abs(C - E[:, cols]).sum(0) / np.abs(E[:, cols]).sum(0)
        assert err.max() <= 1e-15, (n, norm, err)
