"""Python binding of the C ABI: torch tensors in, torch tensors out.

PyTorch supplies device memory and the stream only.  Each function checks the arguments it
forwards, calls the matching ``expm_*`` entry point on the current HIP stream and returns
device tensors; nothing is computed in Python.
"""
import ctypes

import torch

from . import _native as N

_PREC = {"fp64": N.EXPM_PREC_FP64, "fp32": N.EXPM_PREC_FP32, "bf16x3": N.EXPM_PREC_BF16X3,
         "fp32all": N.EXPM_PREC_FP32_ALL}
_SEL = {"plain": N.EXPM_SEL_PLAIN, "alpha": N.EXPM_SEL_ALPHA, "learned": N.EXPM_SEL_LEARNED}


_METHOD = {"reduced": 0, "ps": N.EXPM_FLAG_PS, "pade": N.EXPM_FLAG_PADE, "tri": N.EXPM_FLAG_TRI}


def _opts(dtype, prec, selector, u, method="reduced"):
    """method: "reduced" (the paper's product-reduced T_m), "ps" (the Paterson-Stockmeyer
    comparison, EXPM_FLAG_PS), "pade" (diagonal Pade r_10 / r_26, EXPM_FLAG_PADE) or "tri"
    (the paper's T_m with the triangular refinement, EXPM_FLAG_TRI)."""
    return N.ExpmOpts(N.EXPM_C128 if dtype == torch.complex128 else N.EXPM_F64, _PREC[prec],
                      _SEL[selector], _METHOD[method], 0.0 if u is None else float(u))


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def theta(m, u=2.0 ** -53):
    """theta_m(u) as the library computes it (host only)."""
    out = ctypes.c_double(0.0)
    N.check(N.lib().expm_theta(int(m), float(u), ctypes.byref(out)), "expm_theta")
    return out.value


def select_rule(norms, selector="plain", u=2.0 ** -53):
    """(m, s) of the library's selection rule for ||A||, ||A^2||, ||A^3|| (host only; pass -1
    for a power that is not formed)."""
    arr = (ctypes.c_double * 3)(*[float(x) for x in (list(norms) + [-1.0, -1.0])[:3]])
    m, s = ctypes.c_int32(0), ctypes.c_int32(0)
    N.check(N.lib().expm_select_rule(arr, _SEL[selector], float(u), ctypes.byref(m), ctypes.byref(s)),
            "expm_select_rule")
    return m.value, s.value


def workspace_bytes(n_max, batch=1, dtype=torch.float64, prec="fp64", selector="plain", u=None, method="reduced"):
    """Device workspace in bytes for matrices of order up to n_max (expm_workspace_bytes)."""
    o = _opts(dtype, prec, selector, u, method)
    return N.lib().expm_workspace_bytes(int(n_max), int(batch), ctypes.byref(o))


def _workspace(nbytes, device):
    if nbytes == 0:
        raise N.ExpmError(N.EXPM_E_UNSUPPORTED, "expm_workspace_bytes")
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def _check_square(A):
    if A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square matrix")
    if not A.is_cuda:
        raise ValueError("A must be a device tensor")
    if A.dtype not in (torch.float64, torch.complex128):
        raise ValueError("A must be float64 or complex128")


def taylor(A, u=None, prec="fp64", selector="plain", workspace=None, method="reduced", out=None, outs=None):
    """e^A for one square device matrix.  Returns (E, m, s, status) with m, s, status as
    one-element int32 device tensors.  out: reuse E (shape and dtype of A); outs: reuse a
    three-element int32 device tensor for (m, s, status) (callers that repeat the call)."""
    _check_square(A)
    A = A.contiguous()
    n = A.shape[0]
    o = _opts(A.dtype, prec, selector, u, method)
    ws = workspace if workspace is not None else _workspace(
        N.lib().expm_workspace_bytes(n, 1, ctypes.byref(o)), A.device)
    if out is not None and (out.shape != A.shape or out.dtype != A.dtype or not out.is_contiguous()
                            or out.device != A.device):
        raise ValueError("out must be a contiguous tensor of A's shape, dtype and device")
    if outs is not None and (outs.dtype != torch.int32 or outs.numel() != 3 or outs.device != A.device):
        raise ValueError("outs must be a three-element int32 tensor on A's device")
    E = out if out is not None else torch.empty_like(A)
    ms = outs if outs is not None else torch.empty(3, dtype=torch.int32, device=A.device)
    st = N.lib().expm_taylor(_ptr(A), _ptr(E), n, ctypes.byref(o), _ptr(ms[0:1]), _ptr(ms[1:2]),
                             _ptr(ms[2:3]), _ptr(ws), ws.numel(), _stream())
    N.check(st, "expm_taylor")
    return E, ms[0:1], ms[1:2], ms[2:3]


def select(A, u=None, prec="fp64", selector="plain", method="reduced"):
    """(m, s) chosen for A, as one-element int32 device tensors."""
    _check_square(A)
    A = A.contiguous()
    n = A.shape[0]
    o = _opts(A.dtype, prec, selector, u, method)
    ws = _workspace(N.lib().expm_workspace_bytes(n, 1, ctypes.byref(o)), A.device)
    ms = torch.empty(2, dtype=torch.int32, device=A.device)
    N.check(N.lib().expm_select(_ptr(A), n, ctypes.byref(o), _ptr(ms[0:1]), _ptr(ms[1:2]), _ptr(ws),
                                ws.numel(), _stream()), "expm_select")
    return ms[0:1], ms[1:2]


class Batch:
    """A packed batch of square matrices of uneven order on the device."""

    def __init__(self, packed, offsets, ns, n_max):
        self.packed, self.offsets, self.ns, self.n_max = packed, offsets, ns, int(n_max)

    @classmethod
    def from_host(cls, mats, device="cuda", dtype=torch.float64):
        import numpy as np
        ns = np.array([m.shape[0] for m in mats], dtype=np.int32)
        offs = np.zeros(len(mats), dtype=np.int64)
        if len(mats) > 1:
            offs[1:] = np.cumsum(ns[:-1].astype(np.int64) ** 2)
        packed = np.concatenate([np.ascontiguousarray(m).ravel() for m in mats])
        return cls(torch.from_numpy(packed).to(device=device, dtype=dtype),
                   torch.from_numpy(offs).to(device), torch.from_numpy(ns).to(device), int(ns.max()))

    def unpack(self, flat):
        offs = self.offsets.cpu().numpy()
        ns = self.ns.cpu().numpy()
        host = flat.cpu().numpy()
        return [host[o:o + n * n].reshape(n, n) for o, n in zip(offs, ns)]


def batched(batch, u=None, prec="fp64", selector="plain", workspace=None, out=None, stage=None, outs=None):
    """e^A for every matrix of a Batch.  Returns (E_packed, m, s, status) device tensors.
    stage: None (all phases) or 0..5 (expm_batched_stage); outs: reuse (E, m, s, status)."""
    nb = batch.ns.numel()
    o = _opts(batch.packed.dtype, prec, selector, u)
    ws = workspace if workspace is not None else _workspace(
        N.lib().expm_workspace_bytes(batch.n_max, nb, ctypes.byref(o)), batch.packed.device)
    if outs is not None:
        E, m, s, status = outs
    else:
        E = out if out is not None else torch.empty_like(batch.packed)
        m = torch.empty(nb, dtype=torch.int32, device=batch.packed.device)
        s = torch.empty_like(m)
        status = torch.empty_like(m)
    args = (_ptr(batch.packed), _ptr(E), _ptr(batch.offsets), _ptr(batch.ns), nb, batch.n_max, ctypes.byref(o),
            _ptr(m), _ptr(s), _ptr(status), _ptr(ws), ws.numel(), _stream())
    if stage is None:
        N.check(N.lib().expm_batched(*args), "expm_batched")
    else:
        N.check(N.lib().expm_batched_stage(*args, int(stage)), "expm_batched_stage")
    return E, m, s, status


def batched_noalloc(batch, u=None, prec="fp64", selector="plain", outs=None):
    """e^A for every matrix of a Batch through expm_batched_noalloc (no workspace: the library's
    own device scratch; real order <= 128, at most 65536 matrices).  outs: reuse (E, m, s,
    status).  Returns (E_packed, m, s, status) device tensors."""
    nb = batch.ns.numel()
    o = _opts(batch.packed.dtype, prec, selector, u)
    if outs is not None:
        E, m, s, status = outs
    else:
        E = torch.empty_like(batch.packed)
        m = torch.empty(nb, dtype=torch.int32, device=batch.packed.device)
        s = torch.empty_like(m)
        status = torch.empty_like(m)
    N.check(N.lib().expm_batched_noalloc(_ptr(batch.packed), _ptr(E), _ptr(batch.offsets), _ptr(batch.ns), nb,
                                         batch.n_max, ctypes.byref(o), _ptr(m), _ptr(s), _ptr(status), _stream()),
            "expm_batched_noalloc")
    return E, m, s, status


def batched_uniform(A, u=None, prec="fp64", selector="plain", workspace=None, out=None, outs=None,
                    method="reduced"):
    """e^A for a stack A of shape (batch, n, n) of same-order matrices (float64 or complex128).
    outs reuses (m, s, status).  Returns (E, m, s, status) device tensors."""
    if A.dim() != 3 or A.shape[1] != A.shape[2]:
        raise ValueError("A must have shape (batch, n, n)")
    if not A.is_cuda or A.dtype not in (torch.float64, torch.complex128):
        raise ValueError("A must be a float64 or complex128 device tensor")
    A = A.contiguous()
    nb, n = A.shape[0], A.shape[1]
    o = _opts(A.dtype, prec, selector, u, method)
    ws = workspace if workspace is not None else _workspace(
        N.lib().expm_workspace_bytes(n, nb, ctypes.byref(o)), A.device)
    E = out if out is not None else torch.empty_like(A)
    if outs is not None:
        m, s, status = outs
    else:
        m = torch.empty(nb, dtype=torch.int32, device=A.device)
        s = torch.empty_like(m)
        status = torch.empty_like(m)
    st = N.lib().expm_batched_uniform(_ptr(A), _ptr(E), n, nb, ctypes.byref(o), _ptr(m), _ptr(s), _ptr(status),
                                      _ptr(ws), ws.numel(), _stream())
    N.check(st, "expm_batched_uniform")
    return E, m, s, status


def magnus4_step(S0, S1, Y, u1, u2, h, u=None, selector="plain", out=None, outs=None):
    """One fourth-order Magnus step Y <- e^Omega Y for a batch of systems Y' = (S0 + u(t) S1) Y
    (expm_magnus4_step).  S0, S1: (batch, n, n) or (n, n) shared by all systems; Y: (batch, n, n);
    u1, u2: (batch,) control values at the two Gauss points; h: step.  float64 device tensors,
    n <= 16.  out may be Y itself (in place); outs reuses (m, s, status).  Returns
    (Y_out, m, s, status)."""
    if Y.dim() != 3 or Y.shape[1] != Y.shape[2]:
        raise ValueError("Y must have shape (batch, n, n)")
    nb, n = Y.shape[0], Y.shape[1]
    for t in (S0, S1, Y, u1, u2):
        if not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
            raise ValueError("inputs must be contiguous float64 device tensors")
    if S0.shape != S1.shape or S0.shape[-2:] != (n, n) or S0.dim() not in (2, 3):
        raise ValueError("S0 and S1 must have shape (n, n) or (batch, n, n)")
    if S0.dim() == 3 and S0.shape[0] != nb:
        raise ValueError("per-system S0, S1 need one pair per system")
    if u1.shape != (nb,) or u2.shape != (nb,):
        raise ValueError("u1 and u2 need one value per system")
    stride = 0 if S0.dim() == 2 else n * n
    o = _opts(torch.float64, "fp64", selector, u)
    Yo = out if out is not None else torch.empty_like(Y)
    if outs is not None:
        m, s, status = outs
    else:
        m = torch.empty(nb, dtype=torch.int32, device=Y.device)
        s = torch.empty_like(m)
        status = torch.empty_like(m)
    st = N.lib().expm_magnus4_step(_ptr(S0), _ptr(S1), stride, _ptr(Y), _ptr(Yo), _ptr(u1), _ptr(u2), n, nb,
                                   float(h), ctypes.byref(o), _ptr(m), _ptr(s), _ptr(status), _stream())
    N.check(st, "expm_magnus4_step")
    return Yo, m, s, status
