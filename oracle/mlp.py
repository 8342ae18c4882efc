"""Surrogate network for a learned initial guess (not part of the paper).

The network maps normalised parameters (mu_s, lambda_s) in [-1, 1]^2 to the
standardised coefficients of a snapshot (POD) basis U_0:

    h1 = gelu(W1 x + b1)   (64)
    h2 = gelu(W2 h1 + b2)  (64)
    y  = W3 h2 + b3        (r = 30)

gelu(z) = z * Phi(z) with the exact normal CDF Phi (erf form).  Loss: mean
squared error over the batch and the r outputs.  Optimiser: Adam with bias
correction.  Weights W are stored (out x in).  Everything is float64.

Parity unpinned against the paper (the paper has no network); the pins are
finite-difference gradients, the GELU identities and the first Adam step.
"""
from __future__ import annotations

import math

import numpy as np

_SQRT1_2 = 1.0 / math.sqrt(2.0)
_INV_SQRT_2PI = 1.0 / math.sqrt(2.0 * math.pi)


def _erf(z):
    return np.vectorize(math.erf, otypes=[np.float64])(z)


def gelu(z):
    return 0.5 * z * (1.0 + _erf(z * _SQRT1_2))


def gelu_grad(z):
    """d/dz [z Phi(z)] = Phi(z) + z phi(z)."""
    return 0.5 * (1.0 + _erf(z * _SQRT1_2)) + z * _INV_SQRT_2PI * np.exp(-0.5 * z * z)


def normalise_inputs(mu, lam, mu_range, lam_range):
    """Affine map of each parameter range onto [-1, 1]."""
    x0 = 2.0 * (np.asarray(mu) - mu_range[0]) / (mu_range[1] - mu_range[0]) - 1.0
    x1 = 2.0 * (np.asarray(lam) - lam_range[0]) / (lam_range[1] - lam_range[0]) - 1.0
    return np.column_stack([x0, x1])


def forward(params, X):
    """params = [W1, b1, W2, b2, W3, b3]; X: (B, 2).  Returns (Y, cache)."""
    W1, b1, W2, b2, W3, b3 = params
    Z1 = X @ W1.T + b1
    H1 = gelu(Z1)
    Z2 = H1 @ W2.T + b2
    H2 = gelu(Z2)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(Y, T):
    return float(np.mean((Y - T) ** 2))


def backward(params, cache, Y, T):
    """Gradients of the mean squared error, same order as params."""
    W1, b1, W2, b2, W3, b3 = params
    X, Z1, H1, Z2, H2 = cache
    dY = 2.0 * (Y - T) / Y.size
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dZ2 = (dY @ W3) * gelu_grad(Z2)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dZ1 = (dZ2 @ W2) * gelu_grad(Z1)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return [dW1, db1, dW2, db2, dW3, db3]


class Adam:
    def __init__(self, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps
        self.m = [np.zeros_like(p) for p in params]
        self.v = [np.zeros_like(p) for p in params]
        self.t = 0

    def step(self, params, grads):
        self.t += 1
        out = []
        for k, (p, g) in enumerate(zip(params, grads)):
            self.m[k] = self.b1 * self.m[k] + (1.0 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1.0 - self.b2) * g * g
            mh = self.m[k] / (1.0 - self.b1 ** self.t)
            vh = self.v[k] / (1.0 - self.b2 ** self.t)
            out.append(p - self.lr * mh / (np.sqrt(vh) + self.eps))
        return out


def train(params, X, T, epochs, lr=1e-3):
    """Full-batch Adam; returns (params, loss history)."""
    opt = Adam(params, lr=lr)
    hist = []
    for _ in range(epochs):
        Y, cache = forward(params, X)
        hist.append(loss(Y, T))
        params = opt.step(params, backward(params, cache, Y, T))
    return params, hist


def pod_basis(snapshots, r):
    """Leading r left singular vectors of the snapshot matrix (n x s)."""
    U, s, _ = np.linalg.svd(snapshots, full_matrices=False)
    return U[:, :r], s


def standardise(C):
    mu = C.mean(axis=0)
    sd = C.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return (C - mu) / sd, mu, sd
