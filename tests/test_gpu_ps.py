"""GPU parity of the comparison methods against the CPU oracle: Paterson-Stockmeyer
(EXPM_FLAG_PS: the plain Taylor polynomial by eq. poli9; tiled path above real order 16, one
wave per matrix up to 16) and diagonal Pade r_10 / r_26 (EXPM_FLAG_PADE, one wave per matrix).

Tolerances as for the paper's method: relative 1-norm error <= 1e-12 against the oracle's
long-double direct Taylor e^A, and <= max(1e-12, 64 u 2^s) against the oracle's long-double
evaluation of the same (m, s) (the comparison method's own output); (m, s) equal to the
oracle's rule except within a few ulps of a threshold.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

TOL = 1e-12


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def P():
    import paper_1710_10989_amd as P
    assert torch.cuda.is_available()
    return P


def dev(A):
    return torch.from_numpy(np.ascontiguousarray(A)).cuda()


def check(orc, A, E, m, s):
    ref, _ = orc.expm_taylor(A)
    assert orc.rel_err_1(E, ref) <= TOL
    own = orc.expm_ps(A, m, s)
    assert orc.rel_err_1(E, own) <= max(TOL, 64 * 2.0 ** -53 * (1 << min(s, 30)))


@pytest.mark.parametrize("target,expect", [
    (1e-17, (1, 0)), (1e-9, (2, 0)), (1e-4, (4, 0)), (5e-3, (6, 0)), (0.05, (9, 0)), (0.2, (12, 0)),
    (0.5, (16, 0)), (2.0, (16, 2)), (30.0, (16, 6))])
def test_every_degree(P, orc, target, expect):
    g = np.random.default_rng(int(target * 1e6) % 1000 + 7)
    A = g.standard_normal((37, 37))
    A *= target / np.abs(A).sum(0).max()
    say("case ps", expect)
    E, m, s, st = P.taylor(dev(A), method="ps")
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (int(m.item()), int(s.item())) == expect == orc.select_ps(orc.norm1(A))
    check(orc, A, E.cpu().numpy(), *expect)


@pytest.mark.parametrize("n", [1, 16, 129, 200])
def test_orders(P, orc, n):
    from paper_1710_10989_amd import workloads as W
    g = np.random.default_rng(500 + n)
    for kind in W.STRUCTURES:
        if n == 1 and kind != "dense":
            continue
        A = W.rescale(W.structured(g, n, kind) if n > 1 else g.standard_normal((1, 1)), 3.0)
        say("case ps n=%d %s" % (n, kind))
        E, m, s, st = P.taylor(dev(A), method="ps")
        torch.cuda.synchronize()
        m, s = int(m.item()), int(s.item())
        assert (m, s) == orc.select_ps(orc.norm1(A))
        check(orc, A, E.cpu().numpy(), m, s)


def test_uniform_batch_and_complex(P, orc):
    from paper_1710_10989_amd import workloads as W
    mats = W.large_dense(3, 150, norm_range=(0.1, 20.0), seed_stream=3)
    E, m, s, st = P.batched_uniform(dev(np.stack(mats)), method="ps")
    torch.cuda.synchronize()
    for i, A in enumerate(mats):
        assert (int(m[i].item()), int(s[i].item())) == orc.select_ps(orc.norm1(A))
        check(orc, A, E[i].cpu().numpy(), int(m[i].item()), int(s[i].item()))
    g = np.random.default_rng(9)
    Z = (g.standard_normal((24, 24)) + 1j * g.standard_normal((24, 24))) * 0.1
    E, m, s, st = P.taylor(dev(Z), method="ps")
    torch.cuda.synchronize()
    ref, _ = orc.expm_taylor(Z)
    assert orc.rel_err_1(E.cpu().numpy(), ref) <= TOL


def test_select_only_and_rejections(P, orc):
    from paper_1710_10989_amd import _native as N
    from paper_1710_10989_amd.expm import Batch
    g = np.random.default_rng(2)
    A = g.standard_normal((50, 50)) * 0.02
    m, s = P.select(dev(A), method="ps")
    assert (int(m.item()), int(s.item())) == orc.select_ps(orc.norm1(A))
    with pytest.raises(N.ExpmError) as e:
        P.taylor(dev(A), method="ps", selector="alpha")
    assert e.value.code == N.EXPM_E_UNSUPPORTED
    B = Batch.from_host([A, A[:10, :10]])
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    import ctypes
    from paper_1710_10989_amd import expm as X
    o = X._opts(torch.float64, "fp64", "plain", None, "ps")
    outs = [torch.empty(2, dtype=torch.int32, device="cuda") for _ in range(3)]
    E = torch.empty_like(B.packed)
    st = N.lib().expm_batched(X._ptr(B.packed), X._ptr(E), X._ptr(B.offsets), X._ptr(B.ns), 2, B.n_max,
                              ctypes.byref(o), X._ptr(outs[0]), X._ptr(outs[1]), X._ptr(outs[2]), X._ptr(ws),
                              ws.numel(), X._stream())
    assert st == N.EXPM_E_UNSUPPORTED


# ---- the comparison methods on the one-wave kernel (real order <= 16) ----

@pytest.mark.parametrize("target", [1e-17, 1e-9, 1e-4, 5e-3, 0.05, 0.2, 0.5, 2.0, 30.0])
def test_ps_small_orders(P, orc, target):
    g = np.random.default_rng(int(target * 1e7) % 997)
    mats = []
    for n in (3, 9, 16):
        A = g.standard_normal((n, n))
        mats.append(A * (target / np.abs(A).sum(0).max()))
    for A in mats:
        E, m, s, st = P.taylor(dev(A), method="ps")
        torch.cuda.synchronize()
        m, s = int(m.item()), int(s.item())
        assert int(st.item()) == 0
        assert (m, s) == orc.select_ps(orc.norm1(A))
        check(orc, A, E.cpu().numpy(), m, s)


@pytest.mark.parametrize("target,expect", [(0.1, (10, 0)), (1.0, (10, 2)), (4.0, (26, 0)), (10.0, (26, 1)),
                                           (100.0, (26, 5))])
def test_pade_small_orders(P, orc, target, expect):
    g = np.random.default_rng(int(target * 100) + 3)
    for n in (2, 7, 16):
        A = g.standard_normal((n, n))
        A *= target / np.abs(A).sum(0).max()
        say("case pade n=%d" % n, expect)
        E, m, s, st = P.taylor(dev(A), method="pade")
        torch.cuda.synchronize()
        m, s = int(m.item()), int(s.item())
        assert int(st.item()) == 0
        assert (m, s) == expect == orc.select_pade(orc.norm1(A))
        ref, _ = orc.expm_taylor(A)
        assert orc.rel_err_1(E.cpu().numpy(), ref) <= TOL
        own = orc.expm_pade(A, m, s)
        assert orc.rel_err_1(E.cpu().numpy(), own) <= max(TOL, 64 * 2.0 ** -53 * (1 << s))


def test_comparisons_uniform_small_batch(P, orc):
    from paper_1710_10989_amd import workloads as W
    A = W.small_skew_batch(count=257, n=16, seed_stream=5)
    for method, rule, own in (("ps", orc.select_ps, orc.expm_ps), ("pade", orc.select_pade, orc.expm_pade)):
        say("case uniform small", method)
        E, m, s, st = P.batched_uniform(dev(A), method=method)
        torch.cuda.synchronize()
        E, m, s = E.cpu().numpy(), m.cpu().numpy(), s.cpu().numpy()
        assert bool((st == 0).all())
        for i in range(0, 257, 16):
            assert (m[i], s[i]) == rule(orc.norm1(A[i]))
            ref, _ = orc.expm_taylor(A[i])
            assert orc.rel_err_1(E[i], ref) <= TOL
            assert np.abs(E[i].T @ E[i] - np.eye(16)).max() <= 1e-13


def test_pade_rejections(P):
    from paper_1710_10989_amd import _native as N
    g = np.random.default_rng(4)
    with pytest.raises(N.ExpmError) as e:  # the tiled solve covers real orders up to 2048
        P.taylor(dev(g.standard_normal((2049, 2049))), method="pade")
    assert e.value.code == N.EXPM_E_UNSUPPORTED
    with pytest.raises(N.ExpmError) as e:
        P.taylor(dev(g.standard_normal((5, 5))), method="pade", u=2.0 ** -40)
    assert e.value.code == N.EXPM_E_UNSUPPORTED


@pytest.mark.parametrize("n", [17, 48, 130, 300])
@pytest.mark.parametrize("target,expect", [(0.1, (10, 0)), (1.0, (10, 2)), (4.0, (26, 0)), (100.0, (26, 5))])
def test_pade_tiled_orders(P, orc, n, target, expect):
    """Pade r_10 / r_26 above order 16 (the tiled path: products by the MFMA tile engine, the
    solve by blocked LU with partial pivoting): (2m, s) equal the oracle's rule, e^A within
    1e-12 of the direct Taylor oracle, and the method's own output (the oracle's r_2m(A / 2^s)
    squared s times, from its definition with a long-double LU) within 64 u 2^s."""
    if n == 300 and target in (0.1, 4.0):
        pytest.skip("two norms suffice at n = 300")
    g = np.random.default_rng(int(target * 100) + n)
    A = g.standard_normal((n, n))
    A *= target / np.abs(A).sum(0).max()
    say("case pade tiled n=%d" % n, expect)
    E, m, s, st = P.taylor(dev(A), method="pade")
    torch.cuda.synchronize()
    m, s = int(m.item()), int(s.item())
    assert int(st.item()) == 0
    assert (m, s) == expect == orc.select_pade(orc.norm1(A))
    X = E.cpu().numpy()
    ref, _ = orc.expm_taylor(A)
    assert orc.rel_err_1(X, ref) <= TOL
    own = orc.expm_pade(A, m, s)
    assert orc.rel_err_1(X, own) <= max(TOL, 64 * 2.0 ** -53 * (1 << s))


def test_pade_tiled_batch_and_complex(P, orc):
    """A uniform batch of order 200 (several matrices per group, both degrees, structured
    inputs) and a complex input (real form of order 2 x 40) through the tiled Pade path."""
    from paper_1710_10989_amd import workloads as W
    g = np.random.default_rng(200)
    mats = [W.rescale(W.structured(g, 200, k), t) for k, t in
            (("dense", 0.05), ("skew", 3.0), ("nilpotent", 30.0), ("diag_lowrank", 0.7), ("dense", 9.0))]
    say("case pade tiled batch")
    E, m, s, st = P.batched_uniform(dev(np.stack(mats)), method="pade")
    torch.cuda.synchronize()
    assert bool((st == 0).all())
    for i, A in enumerate(mats):
        assert (int(m[i]), int(s[i])) == orc.select_pade(orc.norm1(A))
        ref, _ = orc.expm_taylor(A)
        assert orc.rel_err_1(E[i].cpu().numpy(), ref) <= TOL, i
    Z = (g.standard_normal((40, 40)) + 1j * g.standard_normal((40, 40))) / 10
    say("case pade tiled complex")
    Ez, mz, sz, stz = P.taylor(dev(Z), method="pade")
    torch.cuda.synchronize()
    assert int(stz.item()) == 0
    ref, _ = orc.expm_taylor(Z)
    assert orc.rel_err_1(Ez.cpu().numpy(), ref) <= TOL


def test_pade_tiled_config_size(P, orc):
    """One n = 1024 matrix of the precision workload by Pade r_26 against sampled columns of
    the oracle's e^A (long-double series), 1e-12 per column."""
    from paper_1710_10989_amd import workloads as W
    A = W.large_dense(2, 1024, seed_stream=0)[1]
    cols = [3, 500, 1000]
    say("case pade n=1024")
    E, m, s, st = P.taylor(dev(A), method="pade")
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    assert (int(m.item()), int(s.item())) == orc.select_pade(orc.norm1(A))
    R = orc.expm_columns(A, cols)
    X = E[:, cols].cpu().numpy()
    err = float((np.abs(X - R).sum(0) / np.abs(R).sum(0)).max())
    say("  (2m, s)=(%d, %d) sampled rel err %.2e" % (int(m.item()), int(s.item()), err))
    assert err <= TOL
