"""FP64 oracle of the warm-start network (test infrastructure; never on the product path).

The network maps 32 summary statistics of a dataset to the 3 initial
log-hyperparameters: three linear layers 32 -> 128 -> 128 -> 3 with the exact
(erf) GELU after the first two, trained with a mean-squared-error loss and
Adam.  Parameters live in one flat vector in the order
W1 (128x32, row-major [out][in]), b1 (128), W2 (128x128), b2 (128), W3 (3x128), b3 (3),
21,123 numbers in all.

Loss: mean over the batch and the three outputs of (pred - label)^2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

MLP_SIZES = (32, 128, 128, 3)
_SHAPES = [(128, 32), (128,), (128, 128), (128,), (3, 128), (3,)]
N_PARAMS = sum(int(np.prod(s)) for s in _SHAPES)


def mlp_unpack(p: np.ndarray):
    """Views (W1, b1, W2, b2, W3, b3) into the flat parameter vector."""
    out = []
    off = 0
    for s in _SHAPES:
        sz = int(np.prod(s))
        out.append(p[off:off + sz].reshape(s))
        off += sz
    return out


def mlp_init(seed: int) -> np.ndarray:
    """He-normal weights (std sqrt(2/fan_in)), zero biases, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    parts = []
    for s in _SHAPES:
        if len(s) == 2:
            parts.append(rng.normal(0.0, math.sqrt(2.0 / s[1]), size=s).ravel())
        else:
            parts.append(np.zeros(s))
    return np.concatenate(parts)


def gelu(x):
    """Exact GELU: x * Phi(x) = x/2 (1 + erf(x / sqrt 2))."""
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def _gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def mlp_forward(p, X):
    """Network output for a batch X (B x 32)."""
    W1, b1, W2, b2, W3, b3 = mlp_unpack(np.asarray(p, dtype=np.float64))
    h1 = gelu(X @ W1.T + b1)
    h2 = gelu(h1 @ W2.T + b2)
    return h2 @ W3.T + b3


def mlp_loss_and_grad(p, X, Y):
    """MSE loss (mean over B x 3 entries) and its gradient w.r.t. the flat parameters."""
    p = np.asarray(p, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    W1, b1, W2, b2, W3, b3 = mlp_unpack(p)
    a1 = X @ W1.T + b1
    h1 = gelu(a1)
    a2 = h1 @ W2.T + b2
    h2 = gelu(a2)
    out = h2 @ W3.T + b3
    diff = out - Y
    nB = X.shape[0]
    loss = float(np.mean(diff * diff))
    d_out = 2.0 * diff / (nB * Y.shape[1])
    gW3 = d_out.T @ h2
    gb3 = d_out.sum(axis=0)
    d_h2 = d_out @ W3
    d_a2 = d_h2 * _gelu_grad(a2)
    gW2 = d_a2.T @ h1
    gb2 = d_a2.sum(axis=0)
    d_h1 = d_a2 @ W2
    d_a1 = d_h1 * _gelu_grad(a1)
    gW1 = d_a1.T @ X
    gb1 = d_a1.sum(axis=0)
    grad = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3.ravel(), gb3])
    return loss, grad


def mlp_adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """Elementwise Adam (Kingma and Ba, 2015) with bias correction; t is 1-based."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
