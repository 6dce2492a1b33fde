"""Oracle for the cost-model MLP: plain fp64 numpy forward, backward and Adam.

TEST INFRASTRUCTURE ONLY (see the package docstring). The network is the
8 -> 64 -> 64 -> 1 ReLU perceptron trained on measured layer times; parameters
are packed as W1[64][8], b1[64], W2[64][64], b2[64], W3[64], b3 (4801 values).
The loss is the mean squared error over the batch.

Backpropagation is written from its definition (chain rule through each
affine map and ReLU) and pinned by central finite differences in the tests;
Adam follows Kingma & Ba (ICLR 2015, Algorithm 1).
"""
import numpy as np

IN, H = 8, 64
SIZES = [("W1", (H, IN)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H,)), ("b3", (1,))]
NPARAM = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(p):
    return np.concatenate([np.asarray(p[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def forward(theta, X):
    """y = W3 . relu(W2 relu(W1 x + b1) + b2) + b3, for every row x of X."""
    p = unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    a1 = X @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    y = h2 @ p["W3"] + p["b3"][0]
    return y, (X, a1, h1, a2, h2)


def loss(theta, X, T):
    y, _ = forward(theta, X)
    return float(np.mean((y - np.asarray(T, dtype=np.float64)) ** 2))


def loss_grad(theta, X, T):
    """(loss, dloss/dtheta) of the mean squared error."""
    p = unpack(theta)
    y, (X, a1, h1, a2, h2) = forward(theta, X)
    B = X.shape[0]
    dy = 2.0 * (y - np.asarray(T, dtype=np.float64)) / B
    g = {"W3": dy @ h2, "b3": np.array([dy.sum()])}
    da2 = np.outer(dy, p["W3"]) * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (a1 > 0)
    g["W1"] = da1.T @ X
    g["b1"] = da1.sum(axis=0)
    return float(np.mean((y - T) ** 2)), pack(g)


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step; returns (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mhat = m / (1 - b1 ** step)
    vhat = v / (1 - b2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
