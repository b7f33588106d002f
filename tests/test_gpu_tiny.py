"""GPU parity of the one-wave kernels (real order <= 16): the batched exponential of small
matrices and the fourth-order Magnus step, against the CPU oracle.

Tolerances as for the other kernels: relative 1-norm error <= 1e-12 against the oracle's
long-double direct Taylor result; (m, s) equal to the oracle's rule, except when the norm lies
within a few ulps of a threshold (the two sides form Omega with different rounding).
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


def near_threshold(orc, eta, u=2.0 ** -53):
    from oracle import theta as th
    for t in th.taylor_thetas(u):
        for s in range(0, 64):
            if abs(eta - t * 2.0 ** s) <= 1e-13 * eta:
                return True
    return False


def check_e(orc, A, E, m, s):
    ref, _ = orc.expm_taylor(A)
    err = orc.rel_err_1(E, ref)
    assert err <= TOL, err
    own = orc.expm_reduced(A, m, s)
    assert orc.rel_err_1(E, own) <= max(TOL, 64 * 2.0 ** -53 * (1 << min(s, 30)))
    return err


@pytest.mark.parametrize("n", list(range(1, 17)))
def test_uniform_every_small_order(P, orc, n):
    g = np.random.default_rng(300 + n)
    norms = [1e-17, 1e-9, 1e-4, 0.03, 0.25, 1.0, 2.0, 7.0, 300.0]
    A = np.stack([g.standard_normal((n, n)) for _ in norms])
    for i, t in enumerate(norms):
        A[i] *= t / np.abs(A[i]).sum(0).max()
    say("case tiny uniform n=%d" % n)
    E, m, s, st = P.batched_uniform(dev(A))
    torch.cuda.synchronize()
    E, m, s, st = E.cpu().numpy(), m.cpu().numpy(), s.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    for i in range(len(norms)):
        assert (m[i], s[i]) == orc.select_plain(orc.norm1(A[i])), (n, i)
        check_e(orc, A[i], E[i], int(m[i]), int(s[i]))


def test_ragged_small_orders_in_a_batch(P, orc):
    # orders 1..24: np 16 on the one-wave kernel, np 32 on the 4-wave kernel, in one call
    from paper_1710_10989_amd import workloads as W
    from paper_1710_10989_amd.expm import Batch
    g = np.random.default_rng(31)
    mats, kinds = [], []
    for i in range(300):
        n = int(g.integers(1, 25))
        kind = W.STRUCTURES[i % 4]
        mats.append(W.rescale(W.structured(g, n, kind) if n > 1 else g.standard_normal((1, 1)),
                              10.0 ** g.uniform(-3, 2)))
        kinds.append(kind)
    B = Batch.from_host(mats)
    say("case tiny ragged 300")
    E, m, s, st = P.batched(B)
    torch.cuda.synchronize()
    outs = B.unpack(E)
    m, s, st = m.cpu().numpy(), s.cpu().numpy(), st.cpu().numpy()
    assert np.all(st == 0)
    refs, _ = orc.expm_taylor_batch(mats, prec="ld")
    for i, (A, R, X) in enumerate(zip(mats, refs, outs)):
        assert (m[i], s[i]) == orc.select_plain(orc.norm1(A)), i
        assert orc.rel_err_1(X, R) <= TOL, (i, kinds[i], A.shape[0])


@pytest.mark.parametrize("kind", ["dense", "skew", "nilpotent", "diag_lowrank"])
def test_alpha_small(P, orc, alpha_ref, kind):
    from paper_1710_10989_amd import workloads as W
    g = np.random.default_rng(57)
    for n in (5, 12, 16):
        for norm in (0.02, 0.5, 3.0, 40.0):
            A = W.rescale(W.structured(g, n, kind), norm)
            say("case tiny alpha", kind, n, norm)
            E, m, s, st = P.taylor(dev(A), selector="alpha")
            torch.cuda.synchronize()
            m, s = int(m.item()), int(s.item())
            assert (m, s) == alpha_ref(orc.powers_norms(A, 3))
            check_e(orc, A, E.cpu().numpy(), m, s)


@pytest.mark.parametrize("n", [1, 3, 8])
def test_complex_small(P, orc, n):
    g = np.random.default_rng(80 + n)
    for norm in (0.1, 2.0, 20.0):
        A = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
        A *= norm / orc.norm1(A)
        say("case tiny complex", n, norm)
        E, m, s, st = P.taylor(dev(A))
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        ref, _ = orc.expm_taylor(A)
        assert orc.rel_err_1(E.cpu().numpy(), ref) <= TOL


def test_nonfinite_member_of_a_batch(P):
    from paper_1710_10989_amd.expm import Batch
    g = np.random.default_rng(3)
    mats = [g.standard_normal((n, n)) * 0.1 for n in (4, 9, 16, 2)]
    mats[1][2, 3] = np.inf
    B = Batch.from_host(mats)
    say("case tiny nonfinite")
    E, m, s, st = P.batched(B)
    torch.cuda.synchronize()
    st = st.cpu().numpy()
    assert list(st) == [0, 2, 0, 0]
    outs = B.unpack(E)
    assert np.isnan(outs[1]).all() and np.isfinite(outs[0]).all() and np.isfinite(outs[2]).all()
    assert int(m[1].item()) == -1 and int(s[1].item()) == -1


def test_select_only_small(P, orc):
    g = np.random.default_rng(8)
    for n, norm in ((3, 0.001), (10, 0.7), (16, 50.0)):
        A = g.standard_normal((n, n))
        A *= norm / np.abs(A).sum(0).max()
        m, s = P.select(dev(A))
        assert (int(m.item()), int(s.item())) == orc.select_plain(orc.norm1(A))


# ---- fourth-order Magnus step ----

def _magnus_inputs(count, n, h, t=0.0, seed_stream=0):
    from paper_1710_10989_amd import workloads as W
    S0, S1, Y0, a, w, phi = W.magnus_systems(count=count, n=n, seed_stream=seed_stream)
    u1, u2 = W.control_at_gauss_points(a, w, phi, t, h)
    return S0, S1, Y0, u1, u2, (a, w, phi)


def _check_magnus(orc, S0, S1, Y, u1, u2, h, Yg, m, s, shared=False):
    for b in range(Y.shape[0]):
        s0 = S0 if shared else S0[b]
        s1 = S1 if shared else S1[b]
        want, Om = orc.magnus4_step(s0, s1, Y[b], u1[b], u2[b], h)
        eta = orc.norm1(Om)
        if (m[b], s[b]) != orc.select_plain(eta):
            assert near_threshold(orc, eta), (b, m[b], s[b], eta)
        assert orc.rel_err_1(Yg[b], want) <= TOL, b


@pytest.mark.parametrize("n", [1, 3, 8, 16])
def test_magnus_step_vs_oracle(P, orc, n):
    h = 0.1
    S0, S1, Y0, u1, u2, _ = _magnus_inputs(129, n, h, seed_stream=n)
    say("case magnus n=%d" % n)
    Yg, m, s, st = P.magnus4_step(dev(S0), dev(S1), dev(Y0), dev(u1), dev(u2), h)
    torch.cuda.synchronize()
    assert np.all(st.cpu().numpy() == 0)
    _check_magnus(orc, S0, S1, Y0, u1, u2, h, Yg.cpu().numpy(), m.cpu().numpy(), s.cpu().numpy())


def test_magnus_shared_generators_in_place_alpha(P, orc, alpha_ref):
    h = 0.3
    S0, S1, Y0, u1, u2, _ = _magnus_inputs(70, 11, h, seed_stream=4)
    Yd = dev(Y0)
    say("case magnus shared in place alpha")
    Yo, m, s, st = P.magnus4_step(dev(S0[0]), dev(S1[0]), Yd, dev(u1), dev(u2), h, selector="alpha", out=Yd)
    torch.cuda.synchronize()
    assert Yo.data_ptr() == Yd.data_ptr()
    assert np.all(st.cpu().numpy() == 0)
    Yg = Yd.cpu().numpy()
    for b in range(70):
        want, Om = orc.magnus4_step(S0[0], S1[0], Y0[b], u1[b], u2[b], h)
        assert orc.rel_err_1(Yg[b], want) <= TOL, b
        nk = orc.powers_norms(Om, 3)
        ma, sa = alpha_ref(nk)
        if (int(m[b].item()), int(s[b].item())) != (ma, sa):
            assert near_threshold(orc, nk[0]) or near_threshold(orc, nk[1] ** 0.5), b


def test_magnus_many_steps_stay_orthogonal(P, orc):
    from paper_1710_10989_amd import workloads as W
    h, steps = 0.05, 40
    S0, S1, Y0, _, _, (a, w, phi) = _magnus_inputs(32, 16, h, seed_stream=9)
    Yd = dev(Y0)
    S0d, S1d = dev(S0), dev(S1)
    Y = Y0.copy()
    say("case magnus 40 steps")
    for k in range(steps):
        u1, u2 = W.control_at_gauss_points(a, w, phi, k * h, h)
        P.magnus4_step(S0d, S1d, Yd, dev(u1), dev(u2), h, out=Yd)
        for b in range(32):
            Y[b], _ = orc.magnus4_step(S0[b], S1[b], Y[b], u1[b], u2[b], h)
    torch.cuda.synchronize()
    Yg = Yd.cpu().numpy()
    for b in range(32):
        assert orc.rel_err_1(Yg[b], Y[b]) <= 50 * TOL, b
        assert np.abs(Yg[b].T @ Yg[b] - np.eye(16)).max() <= 1e-12


def test_magnus_full_size_sampled(P, orc):
    # the benchmark's configuration: 65536 systems of order 16, one step
    h = 0.1
    S0, S1, Y0, u1, u2, _ = _magnus_inputs(65536, 16, h)
    say("case magnus 65536")
    Yg, m, s, st = P.magnus4_step(dev(S0), dev(S1), dev(Y0), dev(u1), dev(u2), h)
    torch.cuda.synchronize()
    assert bool((st == 0).all())
    G = Yg.transpose(1, 2) @ Yg
    assert float((G - torch.eye(16, dtype=G.dtype, device=G.device)).abs().max()) <= 1e-12
    idx = np.random.default_rng(2).choice(65536, 48, replace=False)
    Yh, mh, sh = Yg.cpu().numpy(), m.cpu().numpy(), s.cpu().numpy()
    _check_magnus(orc, S0[idx], S1[idx], Y0[idx], u1[idx], u2[idx], h, Yh[idx], mh[idx], sh[idx])


def test_magnus_rejects_what_it_does_not_run(P):
    from paper_1710_10989_amd import _native as N
    g = np.random.default_rng(1)
    S = dev(g.standard_normal((2, 17, 17)))
    u = dev(np.zeros(2))
    with pytest.raises(N.ExpmError) as e:
        P.magnus4_step(S, S, S, u, u, 0.1)
    assert e.value.code == N.EXPM_E_UNSUPPORTED
    S = dev(g.standard_normal((2, 8, 8)))
    with pytest.raises(N.ExpmError) as e:
        P.magnus4_step(S, S, S, u, u, 0.1, selector="learned")
    assert e.value.code == N.EXPM_E_UNSUPPORTED


def test_magnus_nonfinite_system(P):
    g = np.random.default_rng(2)
    S0 = g.standard_normal((3, 5, 5)) * 0.1
    Y = g.standard_normal((3, 5, 5))
    u1 = np.array([0.1, np.nan, 0.3])
    Yg, m, s, st = P.magnus4_step(dev(S0), dev(S0), dev(Y), dev(u1), dev(u1), 0.1)
    torch.cuda.synchronize()
    assert list(st.cpu().numpy()) == [0, 2, 0]
    assert torch.isnan(Yg[1]).all() and torch.isfinite(Yg[0]).all()


def test_graph_capture_of_one_wave_calls(P, orc):
    # both entry points are graph-capturable: every replay must equal the eager result
    from paper_1710_10989_amd import workloads as W
    A = dev(W.small_skew_batch(count=1000, n=16, seed_stream=11))
    ws = torch.empty(P.workspace_bytes(16, 1000), dtype=torch.uint8, device="cuda")
    out = torch.empty_like(A)
    outs = tuple(torch.empty(1000, dtype=torch.int32, device="cuda") for _ in range(3))
    E0 = P.batched_uniform(A, workspace=ws)[0]
    h = 0.1
    S0, S1, Y0, u1, u2, _ = _magnus_inputs(500, 12, h, seed_stream=12)
    S0d, S1d, Y0d, u1d, u2d = dev(S0), dev(S1), dev(Y0), dev(u1), dev(u2)
    Yo = torch.empty_like(Y0d)
    mouts = tuple(torch.empty(500, dtype=torch.int32, device="cuda") for _ in range(3))
    Y1 = P.magnus4_step(S0d, S1d, Y0d, u1d, u2d, h)[0]
    P.batched_uniform(A, workspace=ws, out=out, outs=outs)  # warm-up outside capture
    P.magnus4_step(S0d, S1d, Y0d, u1d, u2d, h, out=Yo, outs=mouts)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        P.batched_uniform(A, workspace=ws, out=out, outs=outs)
        P.magnus4_step(S0d, S1d, Y0d, u1d, u2d, h, out=Yo, outs=mouts)
    for rep in range(3):
        out.fill_(3.0)
        Yo.fill_(3.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, E0) and torch.equal(Yo, Y1), rep
        _ = (A * 2).sum().item()  # eager work between replays


def test_learned_selector_keeps_small_orders_on_workgroup_kernel(P, orc):
    # under the learned rule orders <= 16 run on the 4-wave kernel (the network lives there);
    # with a network that always proposes (1, 0) every choice falls back to the plain rule
    from paper_1710_10989_amd import learned as LS
    from paper_1710_10989_amd.expm import Batch
    net = LS.MLP(batch=8)
    net.params.zero_()
    net.params[5760] = 10.0  # b3[0]: constant logits, the argmax is class 0 = (1, 0)
    net.norm = np.concatenate([np.zeros(8), np.ones(8)])
    LS.install(net)
    g = np.random.default_rng(21)
    mats = [g.standard_normal((n, n)) * (s / n) for n, s in ((4, 0.5), (16, 3.0), (9, 40.0), (30, 2.0), (16, 1e-3))]
    B = Batch.from_host(mats)
    E, m, s, st = P.batched(B, selector="learned")
    torch.cuda.synchronize()
    outs = B.unpack(E)
    m, s = m.cpu().numpy(), s.cpu().numpy()
    assert bool((st == 0).all())
    for i, A in enumerate(mats):
        mp, sp = orc.select_plain(orc.norm1(A))
        assert (m[i], s[i]) == (mp, sp) or (mp, sp) == (1, 0), i
        ref, _ = orc.expm_taylor(A)
        assert orc.rel_err_1(outs[i], ref) <= TOL
