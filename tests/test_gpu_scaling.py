"""GPU: inputs of huge norm on every kernel family (the one-wave kernel n <= 16, the 4-wave
on-chip kernel 17..64, the split-row kernel 80..96, the 8-wave on-chip kernel 112..128, the
global-memory kernel 144..256, the tiled path above 256).

The scaling X = 2^-s A (Sec. 1, eq. eses) is applied to the matrix itself when it is loaded,
before any power is formed, so no power of A overflows however large ||A||_1 is: e^(-c I) with
c = 1e60 must come back exactly 0 with status OK (the squarings underflow T_m(X) to 0 and keep
it there), a diagonal of entries in [-1e55, -1e54] likewise, and a nilpotent N with N^2 = 0
and ||N||_1 = 1e60 under the alpha rule must give (1, 0) and exactly I + N (X is rescaled from
2^-sp N back to N without rounding).  A matrix of finite entries whose 1-norm overflows is
refused with EXPM_E_NONFINITE, (m, s) = (-1, -1) and a NaN output.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

ORDERS = [16, 48, 96, 128, 200, 300]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A)).cuda()


@pytest.mark.parametrize("n", ORDERS)
@pytest.mark.parametrize("selector", ["plain", "alpha"])
def test_huge_negative_identity_is_zero(n, selector):
    import paper_1710_10989_amd as P
    say("case -1e60 I", n, selector)
    E, m, s, st = P.taylor(dev(-1e60 * np.eye(n)), selector=selector)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert int(m.item()) == 18 and int(s.item()) >= 195
    assert bool((E == 0).all())


@pytest.mark.parametrize("n", ORDERS)
def test_huge_negative_diagonal_is_zero(orc, n):
    import paper_1710_10989_amd as P
    g = np.random.default_rng(n)
    d = -np.exp(g.uniform(np.log(1e54), np.log(1e55), n))
    say("case huge negative diagonal", n)
    E, m, s, st = P.taylor(dev(np.diag(d)))
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (int(m.item()), int(s.item())) == orc.select_plain(float(np.abs(d).max()))
    assert bool((E == 0).all())  # exp of every entry underflows to 0


@pytest.mark.parametrize("n", ORDERS)
def test_huge_nilpotent_alpha_is_exact(n):
    import paper_1710_10989_amd as P
    N = np.zeros((n, n))
    N[0, n - 1] = 1e60
    N[1, n - 1] = -3e59
    say("case huge nilpotent alpha", n)
    E, m, s, st = P.taylor(dev(N), selector="alpha")
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (int(m.item()), int(s.item())) == (1, 0)
    assert np.array_equal(E.cpu().numpy(), np.eye(n) + N)


@pytest.mark.parametrize("n", ORDERS)
def test_overflowing_norm_is_refused(n):
    import paper_1710_10989_amd as P
    A = np.eye(n)
    A[0, 1] = A[1, 1] = 1.5e308  # finite entries, column sum beyond the double range
    say("case overflowing norm", n)
    E, m, s, st = P.taylor(dev(A))
    torch.cuda.synchronize()
    assert (int(st.item()), int(m.item()), int(s.item())) == (2, -1, -1)
    assert bool(torch.isnan(E).all())


def test_huge_norm_batched_mixed_orders(orc):
    # the same inputs through one expm_batched call (work queue, concurrent sweeps)
    import paper_1710_10989_amd as P
    from paper_1710_10989_amd.expm import Batch
    mats = []
    for n in (16, 48, 96, 128, 200):
        mats.append(-1e60 * np.eye(n))
        mats.append(np.random.default_rng(n).standard_normal((n, n)) / n)
    B = Batch.from_host(mats)
    say("case huge norm batched")
    E, m, s, st = P.batched(B)
    torch.cuda.synchronize()
    outs = B.unpack(E)
    assert np.all(st.cpu().numpy() == 0)
    for i, A in enumerate(mats):
        if i % 2 == 0:
            assert np.all(outs[i] == 0), i
        else:
            R, _ = orc.expm_taylor(A)
            assert orc.rel_err_1(outs[i], R) <= 1e-12, i
