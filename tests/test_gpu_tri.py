"""GPU parity of the triangular refinement (EXPM_FLAG_TRI, tiled path) against the oracle's
refined method output: relative 1-norm error <= max(1e-12, 64 u 2^s); the diagonal equal to
exp(a_ii) within 4 ulps entry by entry (it is computed, not accumulated); non-triangular
inputs unaffected (bitwise equal to the unrefined tiled path)."""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_1710_10989_amd as P
    assert torch.cuda.is_available()
    return P


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A)).cuda()


def tri_input(g, n, spread):
    A = np.triu(g.standard_normal((n, n)))
    A[np.diag_indices(n)] = -np.linspace(0.0, spread, n) + 0.1 * g.standard_normal(n)
    return A


@pytest.mark.parametrize("n,spread", [(1, 3.0), (2, 10.0), (5, 25.0), (37, 30.0), (130, 12.0), (300, 40.0)])
def test_refined_triangular(P, orc, n, spread):
    g = np.random.default_rng(n)
    A = tri_input(g, n, spread)
    say("case tri n=%d" % n)
    E, m, s, st = P.taylor(dev(A), method="tri")
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    m, s = int(m.item()), int(s.item())
    assert (m, s) == orc.select_plain(orc.norm1(A))
    E = E.cpu().numpy()
    own = orc.expm_reduced_tri(A, m, s)
    assert orc.rel_err_1(E, own) <= max(1e-12, 64 * 2.0 ** -53 * (1 << s))
    d = np.exp(np.diag(A))
    assert np.all(np.abs(np.diag(E) - d) <= 4 * 2.0 ** -52 * d)
    assert np.all(np.tril(E, -1) == 0.0)
    if n <= 130:
        ref, _ = orc.expm_taylor(A)
        assert orc.rel_err_1(E, ref) <= 1e-12


def test_uniform_batch_mixed_structure(P, orc):
    # a batch with triangular and dense members: only the triangular ones are refined
    g = np.random.default_rng(8)
    mats = [tri_input(g, 64, 20.0), g.standard_normal((64, 64)) * 0.05, tri_input(g, 64, 5.0)]
    E, m, s, st = P.batched_uniform(dev(np.stack(mats)), method="tri")
    torch.cuda.synchronize()
    E, m, s = E.cpu().numpy(), m.cpu().numpy(), s.cpu().numpy()
    for i, A in enumerate(mats):
        ref, _ = orc.expm_taylor(A)
        assert orc.rel_err_1(E[i], ref) <= 1e-12
    for i in (0, 2):
        assert np.allclose(np.diag(E[i]), np.exp(np.diag(mats[i])), rtol=4 * 2.0 ** -52, atol=0)


def test_dense_input_unchanged(P):
    g = np.random.default_rng(9)
    A = g.standard_normal((300, 300)) * (4.0 / 300 ** 0.5)
    E1, m1, s1, _ = P.taylor(dev(A))
    E2, m2, s2, _ = P.taylor(dev(A), method="tri")
    torch.cuda.synchronize()
    assert torch.equal(E1, E2) and torch.equal(m1, m2) and torch.equal(s1, s2)


def test_rejections(P):
    from paper_1710_10989_amd import _native as N
    g = np.random.default_rng(1)
    Z = g.standard_normal((6, 6)) + 1j * g.standard_normal((6, 6))
    with pytest.raises(N.ExpmError) as e:
        P.taylor(dev(Z), method="tri")
    assert e.value.code == N.EXPM_E_UNSUPPORTED
