"""Oracle (test infrastructure only): FP64 point-MLP of the learned GMRES warm start.

Architecture (the warm-start network; the paper motivates reusing the previous iteration's
solution, Sec. 5 "fast update", and leaves the method open):
    h1 = silu(X W1 + b1),  h2 = silu(h1 W2 + b2),  y = h2 W3 + b3
with silu(z) = z * sigmoid(z).  Loss L = mean over all outputs of (y - Y)^2.
Backward pass by the chain rule; Adam (Kingma & Ba 2015) with bias correction.
Parity pinned by tests/test_oracle_mlp_td.py (a closed-form forward pass, central finite differences,
Adam closed forms).
"""
import numpy as np


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def silu_grad(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init_params(d_in, width, d_out=3, seed=0):
    """Deterministic init from an explicit seed (scaled normal, zero biases)."""
    rng = np.random.default_rng(seed)
    return dict(W1=rng.normal(size=(d_in, width)) / np.sqrt(d_in), b1=np.zeros(width),
                W2=rng.normal(size=(width, width)) / np.sqrt(width), b2=np.zeros(width),
                W3=rng.normal(size=(width, d_out)) / np.sqrt(width), b3=np.zeros(d_out))


def forward(p, X):
    z1 = X @ p["W1"] + p["b1"]
    h1 = silu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = silu(z2)
    y = h2 @ p["W3"] + p["b3"]
    return y, (X, z1, h1, z2, h2)


def loss_and_grad(p, X, Y):
    y, (X, z1, h1, z2, h2) = forward(p, X)
    n = y.size
    L = np.sum((y - Y) ** 2) / n
    dy = 2.0 * (y - Y) / n
    g = {}
    g["W3"] = h2.T @ dy
    g["b3"] = dy.sum(0)
    dz2 = (dy @ p["W3"].T) * silu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(0)
    dz1 = (dz2 @ p["W2"].T) * silu_grad(z1)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(0)
    return L, g


class Adam:
    def __init__(self, params, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = {k: np.zeros_like(v) for k, v in params.items()}
        self.v = {k: np.zeros_like(v) for k, v in params.items()}
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        for k in params:
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * grads[k]
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * grads[k] ** 2
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            params[k] = params[k] - self.lr * mh / (np.sqrt(vh) + self.eps)
        return params
