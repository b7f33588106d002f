"""FP64 reference of the learned selector's network (test infrastructure).

Network: x (8) -> relu(W1 x + b1) (64) -> relu(W2 h1 + b2) (64) -> W3 h2 + b3 (16 logits);
loss: mean over the batch of the softmax cross-entropy.  Parameters packed as W1[64][8],
b1[64], W2[64][64], b2[64], W3[16][64], b3[16].  Plain numpy, written out by the chain rule.
"""
import numpy as np

SHAPES = [("W1", (64, 8)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (16, 64)), ("b3", (16,))]
COUNT = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(p):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(p[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([d[name].ravel() for name, _ in SHAPES])


def forward(p, X):
    w = unpack(p)
    a1 = X @ w["W1"].T + w["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ w["W3"].T + w["b3"]
    return z, (h1, h2)


def loss_and_grad(p, X, y):
    """(mean loss, per-sample losses, packed gradient of the mean loss)."""
    X = np.asarray(X, dtype=np.float64)
    B = X.shape[0]
    w = unpack(p)
    z, (h1, h2) = forward(p, X)
    zmax = z.max(axis=1, keepdims=True)
    ez = np.exp(z - zmax)
    prob = ez / ez.sum(axis=1, keepdims=True)
    losses = -np.log(prob[np.arange(B), y])
    dz = prob.copy()
    dz[np.arange(B), y] -= 1.0
    dz /= B
    g = {"W3": dz.T @ h2, "b3": dz.sum(axis=0)}
    dh2 = (dz @ w["W3"]) * (h2 > 0)
    g["W2"] = dh2.T @ h1
    g["b2"] = dh2.sum(axis=0)
    dh1 = (dh2 @ w["W2"]) * (h1 > 0)
    g["W1"] = dh1.T @ X
    g["b1"] = dh1.sum(axis=0)
    return losses.mean(), losses, pack(g)
