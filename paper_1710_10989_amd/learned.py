"""Learned (m, s) selector: data generation, training and installation.

Every numerical step runs in the library's HIP kernels: feature rows and labels come from
expm_features (norms of A, A^2, A^3, trace, asymmetry, label rule), training steps from
expm_mlp_grad / expm_mlp_adam, inference inside the fused expm kernels once expm_learned_set
has installed the parameters.  This module only moves tensors and loops over batches.

Training data: the learned workload's matrices (n in {32, 64, 128, 256}, the 40/20/20/20
dense / skew / strictly upper triangular / diagonal + rank-4 mix, ||A||_1 log-uniform in
[1e-2, 1e3]), drawn on the device with a seeded torch generator (input generation only).

Command line:
  python -m paper_1710_10989_amd.learned train --count 200000 --out ckpt.npz [--resume ckpt.npz]
"""
import argparse
import ctypes
import os

import numpy as np
import torch

from . import _native as N
from . import expm as X

SIZES = (32, 64, 128, 256)
NORM_RANGE = (1e-2, 1e3)
MIX = (0.4, 0.2, 0.2, 0.2)
DEFAULT_CKPT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "learned_selector.npz")


def param_count():
    return N.lib().expm_mlp_param_count()


def device_batch(count, n, gen, device="cuda"):
    """`count` matrices of order n with the structure mix, on the device (float64)."""
    kinds = torch.multinomial(torch.tensor(MIX, dtype=torch.float64), count, replacement=True, generator=gen)
    G = torch.randn(count, n, n, dtype=torch.float64, generator=gen).to(device)
    kd = kinds.to(device)
    A = G.clone()
    skew = kd == 1
    A[skew] = G[skew] - G[skew].transpose(1, 2)
    nil = kd == 2
    A[nil] = torch.triu(G[nil], 1)
    dl = kd == 3
    if dl.any():
        k = int(dl.sum())
        U = torch.randn(k, n, 4, dtype=torch.float64, generator=gen).to(device)
        V = torch.randn(k, n, 4, dtype=torch.float64, generator=gen).to(device)
        d = torch.randn(k, n, dtype=torch.float64, generator=gen).to(device)
        A[dl] = torch.diag_embed(d) + torch.matmul(U, V.transpose(1, 2).contiguous())
    lo, hi = np.log(NORM_RANGE[0]), np.log(NORM_RANGE[1])
    target = torch.exp(torch.rand(count, dtype=torch.float64, generator=gen) * (hi - lo) + lo).to(device)
    nrm = A.abs().sum(dim=1).amax(dim=1)
    A = A * (target / torch.clamp(nrm, min=1e-300)).view(-1, 1, 1)
    return A.contiguous()


def features(batch_obj, workspace=None):
    """Feature rows (batch x 16 float64, see expm_features) and label (m, s) for a Batch."""
    nb = batch_obj.ns.numel()
    o = X._opts(torch.float64, "fp64", "plain", None)
    ws = workspace if workspace is not None else X._workspace(
        N.lib().expm_workspace_bytes(batch_obj.n_max, nb, ctypes.byref(o)), batch_obj.packed.device)
    F = torch.empty(nb, 16, dtype=torch.float64, device=batch_obj.packed.device)
    m = torch.empty(nb, dtype=torch.int32, device=batch_obj.packed.device)
    s = torch.empty_like(m)
    N.check(N.lib().expm_features(X._ptr(batch_obj.packed), X._ptr(batch_obj.offsets), X._ptr(batch_obj.ns), nb,
                                  batch_obj.n_max, ctypes.byref(o), X._ptr(F), X._ptr(m), X._ptr(s), X._ptr(ws),
                                  ws.numel(), X._stream()), "expm_features")
    return F, m, s


def stack_to_batch(A):
    """A Batch view of a (count, n, n) device stack."""
    count, n = A.shape[0], A.shape[1]
    offs = torch.arange(count, dtype=torch.int64, device=A.device) * (n * n)
    ns = torch.full((count,), n, dtype=torch.int32, device=A.device)
    return X.Batch(A.reshape(-1), offs, ns, n)


def make_dataset(count, seed=1710, chunk=4096, device="cuda"):
    """(features [count, 16] float64 device tensor) for `count` matrices, sizes cycled."""
    gen = torch.Generator().manual_seed(seed)
    rows = []
    per = chunk
    done = 0
    i = 0
    while done < count:
        n = SIZES[i % len(SIZES)]
        k = min(per if n < 256 else per // 4, count - done)
        A = device_batch(k, n, gen, device)
        F, _, _ = features(stack_to_batch(A))
        rows.append(F)
        done += k
        i += 1
        del A
    return torch.cat(rows)


class MLP:
    """Parameters, Adam state and device scratch of the selector's network."""

    def __init__(self, batch=1024, seed=0, device="cuda"):
        npar = param_count()
        g = torch.Generator().manual_seed(seed)
        p = torch.zeros(npar, dtype=torch.float32)
        # He-style initialisation of the three weight matrices (biases zero)
        layout = [(0, 64, 8), (576, 64, 64), (4736, 16, 64)]
        for off, rows, cols in layout:
            p[off:off + rows * cols] = torch.randn(rows * cols, generator=g) * np.sqrt(2.0 / cols)
        self.params = p.to(device)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grads = torch.zeros_like(self.params)
        self.step = 0
        self.batch = batch
        self.scratch = torch.empty(N.lib().expm_mlp_scratch_bytes(batch), dtype=torch.uint8, device=device)
        self.loss = torch.empty(batch, dtype=torch.float32, device=device)
        self.norm = np.zeros(16)

    def grad(self, x, y):
        B = x.shape[0]
        N.check(N.lib().expm_mlp_grad(X._ptr(self.params), X._ptr(x), X._ptr(y), B, X._ptr(self.grads),
                                      X._ptr(self.loss), X._ptr(self.scratch), self.scratch.numel(), X._stream()),
                "expm_mlp_grad")
        return self.grads, self.loss[:B]

    def train_step(self, x, y, lr):
        self.grad(x, y)
        self.step += 1
        N.check(N.lib().expm_mlp_adam(X._ptr(self.params), X._ptr(self.grads), X._ptr(self.m), X._ptr(self.v),
                                      self.step, ctypes.c_float(lr), X._stream()), "expm_mlp_adam")

    def logits(self, x):
        B = x.shape[0]
        out = torch.empty(B, 16, dtype=torch.float32, device=x.device)
        N.check(N.lib().expm_mlp_forward(X._ptr(self.params), X._ptr(x), B, X._ptr(out), X._ptr(self.scratch),
                                         self.scratch.numel(), X._stream()), "expm_mlp_forward")
        return out

    def save(self, path):
        np.savez(path, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
                 step=np.array(self.step), norm=self.norm)

    def load(self, path):
        z = np.load(path)  # plain arrays, no pickled objects
        dev = self.params.device
        self.params = torch.from_numpy(z["params"]).to(dev)
        self.m = torch.from_numpy(z["m"]).to(dev)
        self.v = torch.from_numpy(z["v"]).to(dev)
        self.step = int(z["step"])
        self.norm = z["norm"]


def normalisation(F):
    f = F[:, :8].cpu().numpy()
    mean = f.mean(axis=0)
    std = f.std(axis=0)
    std[std < 1e-6] = 1.0
    return np.concatenate([mean, std])


def inputs(F, norm):
    mean = torch.from_numpy(norm[:8]).to(F.device)
    std = torch.from_numpy(norm[8:]).to(F.device)
    return ((F[:, :8] - mean) / std).float().contiguous()


def train(F, epochs=20, lr=2e-3, batch=1024, seed=0, mlp=None, log=None):
    """Trains on feature rows F (label in column 11); returns the MLP."""
    if mlp is None:
        mlp = MLP(batch=batch, seed=seed, device=F.device)
        mlp.norm = normalisation(F)
    x_all = inputs(F, mlp.norm)
    y_all = F[:, 11].round().to(torch.int32).contiguous()
    n = x_all.shape[0]
    g = torch.Generator().manual_seed(seed + 1)
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g).to(F.device)
        tot = 0.0
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            mlp.train_step(x_all[idx].contiguous(), y_all[idx].contiguous(), lr * (0.5 ** (ep // 8)))
            tot += float(mlp.loss.sum())
        if log:
            log("epoch %d mean loss %.4f" % (ep, tot / max(1, (n // batch) * batch)))
    return mlp


def accuracy(mlp, F):
    x = inputs(F, mlp.norm)
    hits = 0
    for b0 in range(0, x.shape[0], mlp.batch):
        pred = mlp.logits(x[b0:b0 + mlp.batch].contiguous()).argmax(dim=1)
        hits += int((pred.cpu() == F[b0:b0 + mlp.batch, 11].round().long().cpu()).sum())
    return hits / x.shape[0]


def install(mlp):
    N.check(N.lib().expm_learned_set(X._ptr(mlp.params), mlp.norm.ctypes.data_as(ctypes.c_void_p), X._stream()),
            "expm_learned_set")


def counts():
    a, r = ctypes.c_int64(0), ctypes.c_int64(0)
    N.check(N.lib().expm_learned_counts(ctypes.byref(a), ctypes.byref(r)), "expm_learned_counts")
    return a.value, r.value


def load_installed(path=DEFAULT_CKPT):
    mlp = MLP()
    mlp.load(path)
    install(mlp)
    return mlp


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train"])
    ap.add_argument("--count", type=int, default=200000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--out", default=DEFAULT_CKPT)
    ap.add_argument("--resume", default=None)
    args = ap.parse_args()
    F = make_dataset(args.count)
    mlp = None
    if args.resume:
        mlp = MLP()
        mlp.load(args.resume)
    mlp = train(F, epochs=args.epochs, mlp=mlp, log=lambda s: print(s, flush=True))
    mlp.save(args.out)
    print("train accuracy %.4f" % accuracy(mlp, F), flush=True)


if __name__ == "__main__":
    main()
