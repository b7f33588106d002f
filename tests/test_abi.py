"""The C-ABI library loads, exports every declared symbol, and its host-only entry points
(thresholds, selection rule, workspace size, argument checks) behave as include/expm.h says.
No GPU call is made here."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import paper_1710_10989_amd as P
from paper_1710_10989_amd import _native as N
from oracle import theta as TH

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "expm.h")).read()
    return sorted(set(re.findall(r"EXPM_API\s+[\w\s\*]*?\b(expm_\w+)\s*\(", text)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(N.EXPORTED)


def test_library_exports_every_declared_symbol():
    L = N.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_library_links_only_hip_runtime():
    # the product path has no dependency on the oracle
    import subprocess
    out = subprocess.run(["ldd", N.LIB_PATH], capture_output=True, text=True).stdout
    assert "oracle" not in out


def test_status_strings():
    for code in range(6):
        assert N.status_string(code)
    assert N.status_string(99) == "unknown status"


@pytest.mark.parametrize("u", [2.0 ** -53, 2.0 ** -24, 2.0 ** -40, 2.0 ** -12])
def test_theta_matches_oracle(u):
    for m in (1, 2, 4, 8, 12, 18):
        got = P.theta(m, u)
        ref = TH.taylor_theta(m, u)
        assert abs(got - ref) <= 4e-15 * ref, (m, u, got, ref)
        assert got <= ref * (1 + 1e-15)


def test_theta_rejects_bad_args():
    out = ctypes.c_double()
    assert N.lib().expm_theta(7, 2.0 ** -53, ctypes.byref(out)) == N.EXPM_E_INVALID_ARG
    assert N.lib().expm_theta(18, 1e-20, ctypes.byref(out)) == N.EXPM_E_INVALID_ARG
    assert N.lib().expm_theta(18, 0.1, ctypes.byref(out)) == N.EXPM_E_INVALID_ARG
    assert N.lib().expm_theta(18, 2.0 ** -53, None) == N.EXPM_E_INVALID_ARG


def test_plain_rule_matches_oracle(orc):
    g = np.random.default_rng(3)
    etas = list(np.exp(g.uniform(np.log(1e-18), np.log(1e4), 4000))) + [0.0]
    th = TH.taylor_thetas(2.0 ** -53)
    etas += [t for t in th] + [np.nextafter(t, np.inf) for t in th]
    etas += [math.ldexp(th[5], s) for s in range(1, 30)]
    lib_th = [P.theta(m) for m in (1, 2, 4, 8, 12, 18)]
    near = lambda x: any(abs(x - math.ldexp(t, s)) <= 4 * np.spacing(x) for t in th + lib_th for s in range(0, 40))
    for eta in etas:
        got, ref = P.select_rule([eta]), orc.select_plain(eta)
        # two independent threshold computations may differ in the last bit: at a boundary
        # either neighbouring choice is correct
        assert got == ref or near(eta), eta


def _bounds(n1, n2, n3):
    # submultiplicative bounds for ||A^4||, ||A^5|| from exact ||A||, ||A^2||, ||A^3||
    n4 = min(n2 * n2, n3 * n1)
    n5 = min(n2 * n3, n4 * n1)
    return [n1, math.sqrt(n2), n3 ** (1 / 3), n4 ** 0.25, n5 ** 0.2]


def test_alpha_rule_matches_oracle(orc):
    from paper_1710_10989_amd import workloads as W
    g = np.random.default_rng(5)
    checked = 0
    for kind in W.STRUCTURES:
        for _ in range(12):
            A = W.rescale(W.structured(g, 12, kind), float(np.exp(g.uniform(np.log(1e-3), np.log(1e3)))))
            nk = orc.powers_norms(A, 3)
            got = P.select_rule(list(nk), "alpha")
            ref = orc.select_alpha(_bounds(*nk))
            assert got == ref, (kind, nk, got, ref)
            checked += 1
    assert checked == 48


def test_alpha_rule_never_costlier_than_plain():
    g = np.random.default_rng(6)
    for _ in range(2000):
        n1 = float(np.exp(g.uniform(-10, 8)))
        n2 = n1 * n1 * float(g.uniform(0, 1))
        n3 = n1 * n2 * float(g.uniform(0, 1))
        mp, sp = P.select_rule([n1])
        ma, sa = P.select_rule([n1, n2, n3], "alpha")
        cost = {1: 0, 2: 1, 4: 2, 8: 3, 12: 4, 18: 5}
        assert cost[ma] + sa <= cost[mp] + sp


def test_workspace_bytes():
    assert P.workspace_bytes(64, 1) > 8 * 64 * 64 * 8
    assert P.workspace_bytes(128, 4096) >= P.workspace_bytes(128, 1)
    o = N.ExpmOpts(0, 0, 0, 0, 0.0)
    assert N.lib().expm_workspace_bytes(0, 1, ctypes.byref(o)) == 0
    assert N.lib().expm_workspace_bytes(64, 0, ctypes.byref(o)) == 0
    bad = N.ExpmOpts(0, 0, 9, 0, 0.0)
    assert N.lib().expm_workspace_bytes(64, 1, ctypes.byref(bad)) == 0


def test_argument_errors_return_before_any_launch():
    L = N.lib()
    o = N.ExpmOpts(0, 0, 0, 0, 0.0)
    v = ctypes.c_void_p(16)  # never dereferenced: argument checks fail first
    assert L.expm_taylor(None, v, 8, ctypes.byref(o), v, v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG
    assert L.expm_taylor(v, v, 8, ctypes.byref(o), v, v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG  # aliasing
    w = ctypes.c_void_p(32)
    assert L.expm_taylor(v, w, 0, ctypes.byref(o), v, v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG
    assert L.expm_taylor(v, w, 8, None, v, v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG
    badu = N.ExpmOpts(0, 0, 0, 0, 1e-30)
    assert L.expm_taylor(v, w, 8, ctypes.byref(badu), v, v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG
    assert L.expm_taylor(v, w, 8, ctypes.byref(o), v, v, v, v, 16, None) == N.EXPM_E_WORKSPACE
    assert L.expm_batched(v, w, None, v, 4, 8, ctypes.byref(o), v, v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG
    assert L.expm_select(None, 8, ctypes.byref(o), v, v, v, 1 << 20, None) == N.EXPM_E_INVALID_ARG


def test_noalloc_limits_return_before_any_launch():
    # the no-allocation variant refuses sizes beyond its fixed scratch with EXPM_E_WORKSPACE
    # and reduced forms with EXPM_E_UNSUPPORTED, before touching any device memory
    L = N.lib()
    o = N.ExpmOpts(0, 0, 0, 0, 0.0)
    v, w = ctypes.c_void_p(16), ctypes.c_void_p(32)
    call = lambda A, E, nb, nmax, opts: L.expm_batched_noalloc(A, E, v, v, nb, nmax, ctypes.byref(opts), v, v, v,
                                                               None)
    assert call(v, w, 4, 129, o) == N.EXPM_E_WORKSPACE
    assert call(v, w, 65537, 128, o) == N.EXPM_E_WORKSPACE
    assert call(v, w, 4, 65, N.ExpmOpts(1, 0, 0, 0, 0.0)) == N.EXPM_E_WORKSPACE  # complex: real order 130
    assert call(v, w, 4, 64, N.ExpmOpts(0, 1, 0, 0, 0.0)) == N.EXPM_E_UNSUPPORTED
    assert call(v, w, 4, 64, N.ExpmOpts(0, 0, 0, N.EXPM_FLAG_PS, 0.0)) == N.EXPM_E_UNSUPPORTED
    assert call(v, v, 4, 64, o) == N.EXPM_E_INVALID_ARG  # output aliases input
    assert call(None, w, 4, 64, o) == N.EXPM_E_INVALID_ARG
    assert call(v, w, 0, 64, o) == N.EXPM_E_INVALID_ARG
