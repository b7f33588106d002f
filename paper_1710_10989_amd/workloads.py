"""Seeded synthetic inputs shaped like the paper's experiments (input generation only).

The paper's stability study uses special matrices from a Matlab test collection and random
matrices spread over a range of norms, 30 x 30 to 60 x 60 (Sec. 4).  That collection is not
available here; these generators stand in for it with dense Gaussian, skew-symmetric,
nilpotent (strictly upper triangular) and diagonal-plus-low-rank matrices rescaled to a target
1-norm.  Every generator takes a seed and returns numpy arrays; nothing here computes any
part of the matrix exponential.
"""
import numpy as np

SEED_BASE = 1710109890
STRUCTURES = ("dense", "skew", "nilpotent", "diag_lowrank")
MIX_WEIGHTS = (0.4, 0.2, 0.2, 0.2)


def rng(config_id, stream=0):
    return np.random.Generator(np.random.PCG64([SEED_BASE + config_id, stream]))


def _norm1(A):
    return float(np.abs(A).sum(axis=0).max())


def rescale(A, target):
    nrm = _norm1(A)
    return A * (target / nrm) if nrm > 0 else A


def structured(g, n, kind):
    if kind == "dense":
        return g.standard_normal((n, n))
    if kind == "skew":
        G = g.standard_normal((n, n))
        return G - G.T
    if kind == "nilpotent":
        return np.triu(g.standard_normal((n, n)), 1)
    if kind == "diag_lowrank":
        U, V = g.standard_normal((n, 4)), g.standard_normal((n, 4))
        return np.diag(g.standard_normal(n)) + U @ V.T
    raise ValueError(kind)


def single_dense(n=64, norm1=2.0, seed_stream=0):
    """One n x n matrix with N(0,1) entries rescaled to ||A||_1 = norm1 (the plain single
    matrix case: n = 64, ||A||_1 = 2)."""
    g = rng(1, seed_stream)
    return rescale(g.standard_normal((n, n)), norm1)


def mixed_batch(count=4096, sizes=(16, 32, 48, 64, 96, 128), norm_range=(1e-3, 1e2), config_id=2,
                seed_stream=0):
    """Batch of matrices of uneven order: n uniform over `sizes`, ||A||_1 log-uniform over
    `norm_range`, structure drawn from STRUCTURES with MIX_WEIGHTS.  Returns (mats, kinds)."""
    g = rng(config_id, seed_stream)
    ns = g.choice(np.asarray(sizes), size=count)
    kinds = g.choice(len(STRUCTURES), size=count, p=np.asarray(MIX_WEIGHTS))
    lo, hi = np.log(norm_range[0]), np.log(norm_range[1])
    norms = np.exp(g.uniform(lo, hi, size=count))
    mats = [rescale(structured(g, int(n), STRUCTURES[k]), float(t)) for n, k, t in zip(ns, kinds, norms)]
    return mats, [STRUCTURES[k] for k in kinds]


def pack(mats):
    """(packed float64 vector, int64 element offsets, int32 orders)."""
    ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
    offs = np.zeros(len(mats), dtype=np.int64)
    if len(mats) > 1:
        offs[1:] = np.cumsum(ns[:-1].astype(np.int64) ** 2)
    packed = np.concatenate([np.ascontiguousarray(m, dtype=np.float64).ravel() for m in mats])
    return packed, offs, ns


def large_dense(count, n, norm_range=(0.5, 50.0), config_id=3, seed_stream=0):
    """Dense matrices with N(0,1)/sqrt(n) entries rescaled to ||A||_1 uniform over norm_range."""
    g = rng(config_id, seed_stream)
    out = []
    for _ in range(count):
        t = g.uniform(*norm_range)
        out.append(rescale(g.standard_normal((n, n)) / np.sqrt(n), t))
    return out


def hermitian_unitary_batch(count=512, n=256, dt_range=(1e-2, 1e2), config_id=5, seed_stream=0):
    """A = -i H dt with H = (G + G^H)/2, G complex Gaussian, H rescaled to spectral radius 1,
    dt log-uniform over dt_range.  Returns (mats, dts)."""
    g = rng(config_id, seed_stream)
    mats, dts = [], []
    for _ in range(count):
        G = g.standard_normal((n, n)) + 1j * g.standard_normal((n, n))
        H = (G + G.conj().T) / 2
        H /= np.max(np.abs(np.linalg.eigvalsh(H)))
        dt = float(np.exp(g.uniform(np.log(dt_range[0]), np.log(dt_range[1]))))
        mats.append(-1j * H * dt)
        dts.append(dt)
    return mats, dts


def magnus_systems(count=65536, n=16, s0_norm=2.0, s1_norm=1.0, config_id=6, seed_stream=0):
    """Linear systems Y' = (S0 + u(t) S1) Y on the orthogonal group, the setting of the
    exponential (Magnus) integrators in the paper's concluding remarks: S0, S1 skew-symmetric
    (G - G^T, G Gaussian) rescaled to the given 1-norms, the state Y0 a random orthogonal
    matrix (QR of a Gaussian), and a control u(t) = a cos(w t + phi) per system with a in
    [0.5, 2], w in [1, 10], phi in [0, 2 pi).  Returns S0, S1, Y0 as (count, n, n) arrays and
    a, w, phi as (count,) arrays."""
    g = rng(config_id, seed_stream)

    def skew(norm):
        G = g.standard_normal((count, n, n))
        S = G - np.transpose(G, (0, 2, 1))
        nr = np.abs(S).sum(axis=1).max(axis=1)
        nr[nr == 0] = 1.0
        return S * (norm / nr)[:, None, None]

    S0 = skew(s0_norm)
    S1 = skew(s1_norm)
    Q, R = np.linalg.qr(g.standard_normal((count, n, n)))
    Y0 = Q * np.sign(np.diagonal(R, axis1=1, axis2=2))[:, None, :]
    a = g.uniform(0.5, 2.0, count)
    w = g.uniform(1.0, 10.0, count)
    phi = g.uniform(0.0, 2 * np.pi, count)
    return S0, S1, np.ascontiguousarray(Y0), a, w, phi


def control_at_gauss_points(a, w, phi, t, h):
    """u = a cos(w t + phi) sampled at the two Gauss-Legendre nodes of [t, t + h],
    t + (1/2 -+ sqrt(3)/6) h; returns (u1, u2)."""
    c = np.sqrt(3.0) / 6.0
    return a * np.cos(w * (t + (0.5 - c) * h) + phi), a * np.cos(w * (t + (0.5 + c) * h) + phi)


def small_skew_batch(count=65536, n=16, norm_range=(0.05, 1.0), config_id=7, seed_stream=0):
    """count skew-symmetric n x n matrices (G - G^T) with ||A||_1 log-uniform in norm_range:
    the small, modest-norm exponents an exponential integrator on the orthogonal group
    produces at each step.  Returns a (count, n, n) array."""
    g = rng(config_id, seed_stream)
    G = g.standard_normal((count, n, n))
    S = G - np.transpose(G, (0, 2, 1))
    nr = np.abs(S).sum(axis=1).max(axis=1)
    nr[nr == 0] = 1.0
    target = np.exp(g.uniform(np.log(norm_range[0]), np.log(norm_range[1]), count))
    return np.ascontiguousarray(S * (target / nr)[:, None, None])


def triangular_batch(count=64, n=512, spread=40.0, config_id=8, seed_stream=0):
    """count upper triangular n x n matrices whose diagonal spreads over [-spread, 0]
    (uniform) with strictly upper entries N(0, 1) / sqrt(n): the inputs where overwriting the
    diagonal of the squared iterates with exact values matters (many squarings, entries of very
    different size).  Returns a (count, n, n) array."""
    g = rng(config_id, seed_stream)
    A = np.triu(g.standard_normal((count, n, n)), 1) / np.sqrt(n)
    idx = np.arange(n)
    A[:, idx, idx] = -g.uniform(0.0, spread, (count, n))
    return np.ascontiguousarray(A)
