"""CPU oracle for the product-reduced Taylor matrix exponential (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may import this
package.  It shares no code with the GPU library: the arithmetic lives in ``expm_oracle.c``
(plain C loop nests, long double / double) and ``theta.py`` (exact rational series).

Every function takes and returns numpy arrays (row-major, float64 or complex128).
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "expm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force=False):
    """Compile ``liboracle.so`` with gcc (no FMA contraction, OpenMP over batches)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O3", "-fPIC", "-shared", "-ffp-contract=off", "-fopenmp",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
        vp, ip = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int)
        L.or_norm1.argtypes = [i64, vp]; L.or_norm1.restype = dbl
        L.or_norm1_z.argtypes = [i64, vp]; L.or_norm1_z.restype = dbl
        L.or_expm_taylor.argtypes = [i64, vp, vp, i32, ip]; L.or_expm_taylor.restype = i32
        L.or_expm_taylor_z.argtypes = [i64, vp, vp, ip]; L.or_expm_taylor_z.restype = i32
        L.or_expm_taylor_batch.argtypes = [i64, vp, vp, vp, vp, i32, vp]; L.or_expm_taylor_batch.restype = i32
        L.or_expm_pade26.argtypes = [i64, vp, vp, dbl, ip]; L.or_expm_pade26.restype = i32
        L.or_pade_ms.argtypes = [i64, vp, i32, i32, vp]; L.or_pade_ms.restype = i32
        L.or_reduced_Tm.argtypes = [i64, vp, i32, vp]; L.or_reduced_Tm.restype = i32
        L.or_expm_reduced.argtypes = [i64, vp, i32, i32, vp]; L.or_expm_reduced.restype = i32
        L.or_select_plain.argtypes = [dbl, vp, ip, ip]; L.or_select_plain.restype = None
        L.or_select_alpha.argtypes = [vp, vp, ip, ip]; L.or_select_alpha.restype = None
        L.or_powers_norms.argtypes = [i64, vp, i32, vp]; L.or_powers_norms.restype = None
        L.or_select_alpha_split.argtypes = [vp, vp, vp, ip, ip]; L.or_select_alpha_split.restype = None
        L.or_expm_apply.argtypes = [i64, vp, i64, vp, vp]; L.or_expm_apply.restype = i32
        L.or_expm_apply_z.argtypes = [i64, vp, i64, vp, vp]; L.or_expm_apply_z.restype = i32
        L.or_set_threads.argtypes = [i32]; L.or_set_threads.restype = None
        L.or_get_threads.argtypes = []; L.or_get_threads.restype = i32
        _lib = L
    return _lib


def _f64(A):
    A = np.ascontiguousarray(A, dtype=np.float64)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return A


def _c128(A):
    A = np.ascontiguousarray(A, dtype=np.complex128)
    assert A.ndim == 2 and A.shape[0] == A.shape[1]
    return A


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def norm1(A):
    """||A||_1 = max_j sum_i |a_ij|, accumulated in long double."""
    if np.iscomplexobj(A):
        A = _c128(A)
        return lib().or_norm1_z(A.shape[0], _p(A))
    A = _f64(A)
    return lib().or_norm1(A.shape[0], _p(A))


def expm_taylor(A, prec="ld"):
    """e^A by the plain Taylor series with the oracle's own scaling (||X||_1 <= 1/2) and
    squaring.  prec: "ld" (long double) or "d" (double); complex input always uses long
    double complex.  Returns (E, s)."""
    s = ctypes.c_int(0)
    if np.iscomplexobj(A):
        A = _c128(A)
        E = np.empty_like(A)
        rc = lib().or_expm_taylor_z(A.shape[0], _p(A), _p(E), ctypes.byref(s))
    else:
        A = _f64(A)
        E = np.empty_like(A)
        rc = lib().or_expm_taylor(A.shape[0], _p(A), _p(E), 1 if prec == "ld" else 0, ctypes.byref(s))
    if rc < 0:
        raise ValueError("non-finite input")
    return E, s.value


def expm_columns(A, cols):
    """Columns `cols` of e^A, i.e. e^A e_j, from the series of A / q applied q times to e_j in
    long double, q = ceil(||A||_1 / 2) (see or_expm_apply).  Returns an (n, len(cols)) array."""
    cplx = np.iscomplexobj(A)
    A = _c128(A) if cplx else _f64(A)
    n = A.shape[0]
    V = np.zeros((len(cols), n), dtype=A.dtype)
    for c, j in enumerate(cols):
        V[c, j] = 1.0
    out = np.empty_like(V)
    f = lib().or_expm_apply_z if cplx else lib().or_expm_apply
    if f(n, _p(A), len(cols), _p(V), _p(out)) < 0:
        raise ValueError("series did not converge")
    return out.T.copy()


def set_threads(t):
    """OpenMP threads of the batch routines; returns the count a parallel region then uses."""
    lib().or_set_threads(int(t))
    return lib().or_get_threads()


def expm_taylor_batch(mats, prec="d"):
    """Direct-Taylor e^A of a list of real matrices, OpenMP over matrices."""
    ns = np.array([m.shape[0] for m in mats], dtype=np.int64)
    offs = np.zeros(len(mats), dtype=np.int64)
    if len(mats) > 1:
        offs[1:] = np.cumsum(ns[:-1] ** 2)
    packed = np.concatenate([np.ascontiguousarray(m, dtype=np.float64).ravel() for m in mats])
    out = np.empty_like(packed)
    svals = np.zeros(len(mats), dtype=np.int32)
    bad = lib().or_expm_taylor_batch(len(mats), _p(ns), _p(offs), _p(packed), _p(out),
                                     1 if prec == "ld" else 0, _p(svals))
    if bad:
        raise ValueError("non-finite input in %d matrices" % bad)
    return [out[o:o + n * n].reshape(n, n) for o, n in zip(offs, ns)], svals


def expm_pade26(A, theta26=None):
    """Diagonal Pade r_26 with scaling and squaring (long double).  Returns (E, s)."""
    if theta26 is None:
        from . import theta as _theta
        theta26 = _theta.pade_theta(13, 2.0 ** -53)
    A = _f64(A)
    E = np.empty_like(A)
    s = ctypes.c_int(0)
    rc = lib().or_expm_pade26(A.shape[0], _p(A), _p(E), float(theta26), ctypes.byref(s))
    if rc < 0:
        raise ValueError("non-finite input or singular denominator")
    return E, s.value


def reduced_Tm(X, m):
    """T_m(X) by the paper's product-reduced sequence, evaluated in long double.
    Returns (T, number_of_products)."""
    X = _f64(X)
    T = np.empty_like(X)
    p = lib().or_reduced_Tm(X.shape[0], _p(X), int(m), _p(T))
    if p < 0:
        raise ValueError("unsupported degree %r" % (m,))
    return T, p


def expm_reduced(A, m, s):
    """T_m(A/2^s)^(2^s) in long double: the method's output for a given (m, s)."""
    A = _f64(A)
    E = np.empty_like(A)
    p = lib().or_expm_reduced(A.shape[0], _p(A), int(m), int(s), _p(E))
    if p < 0:
        raise ValueError("unsupported degree %r" % (m,))
    return E


def powers_norms(A, kmax=5):
    """[||A^k||_1 for k = 1..kmax] from explicit long-double powers."""
    A = _f64(A)
    out = np.zeros(kmax, dtype=np.float64)
    lib().or_powers_norms(A.shape[0], _p(A), int(kmax), _p(out))
    return out


def _theta_row(u):
    from . import theta as _theta
    return np.array(_theta.taylor_thetas(u), dtype=np.float64)


def select_plain(eta, u=2.0 ** -53):
    """(m, s) of the plain norm rule for ||A||_1 = eta."""
    th = _theta_row(u)
    m, s = ctypes.c_int(0), ctypes.c_int(0)
    lib().or_select_plain(float(eta), _p(th), ctypes.byref(m), ctypes.byref(s))
    return m.value, s.value


def select_alpha(dk, u=2.0 ** -53):
    """(m, s) of the alpha_p rule given d_1..d_5 (exact values or upper bounds)."""
    th = _theta_row(u)
    d = np.ascontiguousarray(dk, dtype=np.float64)
    assert d.shape == (5,)
    m, s = ctypes.c_int(0), ctypes.c_int(0)
    lib().or_select_alpha(_p(d), _p(th), ctypes.byref(m), ctypes.byref(s))
    return m.value, s.value


def rel_err_1(X, R):
    """Relative 1-norm error ||X - R||_1 / ||R||_1 (long double accumulation)."""
    D = np.asarray(X) - np.asarray(R)
    return norm1(D) / norm1(R)


def alpha_bounds(n1, n2, n3=None):
    """[d_1..d_5]: d_k = ||A^k||^(1/k) from ||A||, ||A^2|| and, when given, ||A^3||; the
    missing ones by submultiplicativity (||A^3|| <= ||A|| ||A^2||, ||A^4|| <= min(||A^2||^2,
    ||A^3|| ||A||), ||A^5|| <= min(||A^2|| ||A^3||, ||A^4|| ||A||))."""
    if n3 is None:
        n3 = min(n1 * n2, n1 ** 3)
    n4 = min(n2 * n2, n3 * n1)
    n5 = min(n2 * n3, n4 * n1)
    return [n1, n2 ** 0.5, n3 ** (1.0 / 3.0), n4 ** 0.25, n5 ** 0.2]


def learned_label(n1, n2, n3, u=2.0 ** -53):
    """Cheapest (m, s) passing the alpha bound with ||A^3|| for m >= 12 and its bound for
    m <= 8 (the information the learned selector has)."""
    th = _theta_row(u)
    lo = np.array(alpha_bounds(n1, n2), dtype=np.float64)
    hi = np.array(alpha_bounds(n1, n2, n3), dtype=np.float64)
    m, s = ctypes.c_int(0), ctypes.c_int(0)
    lib().or_select_alpha_split(_p(lo), _p(hi), _p(th), ctypes.byref(m), ctypes.byref(s))
    return m.value, s.value


def learned_features(A):
    """The selector's 8 features of a real matrix: log2 d_1..d_5 (bounds from ||A||, ||A^2||),
    log2 n, |tr A| / ||A||_1, ||A - A^T||_1 / (2 ||A||_1)."""
    A = _f64(A)
    n1, n2 = powers_norms(A, 2)
    d = alpha_bounds(n1, n2)
    f = [np.log2(max(x, 1e-300)) for x in d]
    f.append(np.log2(A.shape[0]))
    f.append(abs(np.trace(A)) / n1 if n1 > 0 else 0.0)
    f.append(norm1(A - A.T) / (2 * n1) if n1 > 0 else 0.0)
    return np.array(f)


def magnus4_omega(S0, S1, u1, u2, h):
    """Exponent of one fourth-order Magnus step for Y' = F(t) Y, F(t) = S0 + u(t) S1, with F
    sampled at the two Gauss points (u1, u2 the control there): (h/2)(F_1 + F_2) plus
    (sqrt(3) h^2 / 12) [F_2, F_1] (the exponential integrators of the concluding remarks; the
    scheme is the standard two-point Gauss truncation of the Magnus expansion).  Double
    precision, plain matrix products."""
    S0 = np.asarray(S0, dtype=np.float64)
    S1 = np.asarray(S1, dtype=np.float64)
    F1 = S0 + u1 * S1
    F2 = S0 + u2 * S1
    return 0.5 * h * (F1 + F2) + (np.sqrt(3.0) * h * h / 12.0) * (F2 @ F1 - F1 @ F2)


def magnus4_step(S0, S1, Y, u1, u2, h, prec="ld"):
    """Y_next = e^Omega Y with Omega = magnus4_omega(...) and e^Omega from the oracle's
    direct Taylor series (long double by default)."""
    Om = magnus4_omega(S0, S1, u1, u2, h)
    E, _ = expm_taylor(Om, prec=prec)
    return E @ np.asarray(Y, dtype=np.float64), Om


# ---- Paterson-Stockmeyer comparison method (Sec. 4, eq. poli9, Table 3) ----

PS_DEGREES = (1, 2, 4, 6, 9, 12, 16)
PS_PRODUCTS = (0, 1, 2, 3, 4, 5, 6)


def taylor_poly(X, m):
    """T_m(X) = sum_{k=0}^{m} X^k / k!, the truncated Taylor series itself (Sec. 1), summed
    term by term in long double.  Returns a long-double array."""
    X = np.asarray(X, dtype=np.longdouble)
    P = np.eye(X.shape[0], dtype=np.longdouble)
    S = P.copy()
    for k in range(1, m + 1):
        P = (P @ X) / k
        S = S + P
    return S


def select_ps(eta, u=2.0 ** -53):
    """(m, s) of the comparison method: over the Paterson-Stockmeyer degrees and their product
    counts (Table 3), s = the smallest s >= 0 with eta <= theta_m 2^s (eq. eq.theta, thresholds
    of Table 2 recomputed by theta.py), the cheapest products + s, ties to the smaller s."""
    from . import theta as _theta
    best = None
    for m, p in zip(PS_DEGREES, PS_PRODUCTS):
        th = float(_theta.taylor_theta(m, u))
        s = 0
        while eta > np.ldexp(th, s):
            s += 1
        if best is None or p + s < best[0] or (p + s == best[0] and s < best[2]):
            best = (p + s, m, s)
    return best[1], best[2]


def expm_ps(A, m, s):
    """T_m(A / 2^s)^(2^s) with the plain truncated series, in long double: the comparison
    method's output for a given (m, s)."""
    X = np.asarray(A, dtype=np.longdouble) * np.ldexp(np.longdouble(1.0), -s)
    T = taylor_poly(X, m)
    for _ in range(s):
        T = T @ T
    return np.asarray(T, dtype=np.float64)


# ---- diagonal Pade comparison method (Sec. 2, eqs. eq.24, eq.pade10, eq.pade26, Table 1) ----

# theta_10 and theta_26 of Table 1, one unit of the third printed digit below the printed
# value (a printed value may be rounded up); only the two printed rows of u
PADE_THETA = {2.0 ** -53: (2.53e-1, 5.36), 2.0 ** -24: (1.87, 11.1)}


def select_pade(eta, u=2.0 ** -53):
    """(2m, s) of the Pade comparison: r_10 (3 products) or r_26 (6 products), one solve costed
    4/3 of a product; s the smallest with eta <= theta_2m 2^s; the cheaper, ties to the smaller s."""
    best = None
    for deg, prods, th in zip((10, 26), (3, 6), PADE_THETA[u]):
        s = 0
        while eta > np.ldexp(th, s):
            s += 1
        cost3 = 3 * prods + 4 + 3 * s
        if best is None or cost3 < best[0] or (cost3 == best[0] and s < best[2]):
            best = (cost3, deg, s)
    return best[1], best[2]


def expm_pade(A, deg, s):
    """r_deg(A / 2^s)^(2^s), deg = 2m, from the definition p_m(X) / p_m(-X) (long double)."""
    A = _f64(A)
    E = np.empty_like(A)
    if lib().or_pade_ms(A.shape[0], _p(A), int(deg) // 2, int(s), _p(E)) < 0:
        raise ValueError("singular denominator")
    return E


# ---- triangular refinement (concluding remarks) ----

def _tri_fix(T, A, f):
    """Replaces the diagonal and first superdiagonal of T (long double, in place) by those of
    e^(f A) for upper triangular A: exp(f a_ii), and for each 2 x 2 diagonal block
    [[x1, y], [0, x2]] of f A the (1, 2) entry y (e^x2 - e^x1) / (x2 - x1), written as
    y e^((x1 + x2) / 2) sinh(d) / d with d = (x2 - x1) / 2 (y e^x1 when x1 = x2)."""
    n = T.shape[0]
    for i in range(n):
        x1 = f * A[i, i]
        T[i, i] = np.exp(x1)
        if i + 1 < n:
            x2, y = f * A[i + 1, i + 1], f * A[i, i + 1]
            d = (x2 - x1) / 2
            T[i, i + 1] = y * np.exp((x1 + x2) / 2) * (np.sinh(d) / d if d != 0 else 1)


def expm_reduced_tri(A, m, s):
    """The method's output with the triangular refinement for an upper triangular A, long
    double: T_m(2^-s A) by the product-reduced sequences, its diagonal and first superdiagonal
    replaced by those of e^(2^-s A), then s squarings, each followed by the same replacement
    for e^(2^(r-s) A)."""
    A = _f64(A)
    Al = A.astype(np.longdouble)
    T, _ = reduced_Tm(np.ldexp(A, -s), m)
    T = T.astype(np.longdouble)
    _tri_fix(T, Al, np.ldexp(np.longdouble(1.0), -s))
    for r in range(1, s + 1):
        T = T @ T
        _tri_fix(T, Al, np.ldexp(np.longdouble(1.0), r - s))
    return np.asarray(T, dtype=np.float64)
