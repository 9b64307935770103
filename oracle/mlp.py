"""Oracle: a plain FP64 multilayer perceptron, forward, backward and Adam.
Test infrastructure.  (The network is not in the paper; it is the learned
warm start layered on the per-frequency solve.)

Network: Y = W3^T s(W2^T s(W1^T X^T + b1) + b2) + b3 written row-wise as
    Z1 = X W1 + b1,  H1 = silu(Z1),  Z2 = H1 W2 + b2,  H2 = silu(Z2),  Y = H2 W3 + b3,
silu(z) = z / (1 + e^{-z}).  Loss: mean over samples and outputs of (Y - T)^2.
Adam: m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
p -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).

Flat parameter layout (shared by any implementation that takes a flat
vector): W1 [d_in, H] row-major, b1 [H], W2 [H, H], b2 [H], W3 [H, d_out], b3 [d_out].
"""
from __future__ import annotations

import numpy as np


def sizes(d_in, hidden, d_out):
    return [(d_in, hidden), (hidden,), (hidden, hidden), (hidden,), (hidden, d_out), (d_out,)]


def n_params(d_in, hidden, d_out):
    return sum(int(np.prod(s)) for s in sizes(d_in, hidden, d_out))


def unpack(p, d_in, hidden, d_out):
    out, o = [], 0
    for shp in sizes(d_in, hidden, d_out):
        n = int(np.prod(shp))
        out.append(p[o:o + n].reshape(shp))
        o += n
    return out


def init(d_in, hidden, d_out, seed):
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights and biases."""
    rng = np.random.default_rng(seed)
    parts = []
    for shp, fan in zip(sizes(d_in, hidden, d_out), [d_in, d_in, hidden, hidden, hidden, hidden]):
        b = 1.0 / np.sqrt(fan)
        parts.append(rng.uniform(-b, b, size=shp).reshape(-1))
    return np.concatenate(parts)


def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


def forward(p, X, d_in, hidden, d_out):
    W1, b1, W2, b2, W3, b3 = unpack(p, d_in, hidden, d_out)
    Z1 = X @ W1 + b1
    H1 = silu(Z1)
    Z2 = H1 @ W2 + b2
    H2 = silu(Z2)
    Y = H2 @ W3 + b3
    return Y, (Z1, H1, Z2, H2)


def loss_and_grad(p, X, T, d_in, hidden, d_out):
    W1, b1, W2, b2, W3, b3 = unpack(p, d_in, hidden, d_out)
    Y, (Z1, H1, Z2, H2) = forward(p, X, d_in, hidden, d_out)
    n = X.shape[0]
    R = Y - T
    loss = np.mean(R ** 2)
    dY = 2.0 * R / R.size
    gW3 = H2.T @ dY
    gb3 = dY.sum(0)
    dZ2 = (dY @ W3.T) * dsilu(Z2)
    gW2 = H1.T @ dZ2
    gb2 = dZ2.sum(0)
    dZ1 = (dZ2 @ W2.T) * dsilu(Z1)
    gW1 = X.T @ dZ1
    gb1 = dZ1.sum(0)
    del n
    return loss, np.concatenate([g.reshape(-1) for g in (gW1, gb1, gW2, gb2, gW3, gb3)])


def adam_step(p, g, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    m = beta1 * m + (1 - beta1) * g
    v = beta2 * v + (1 - beta2) * g * g
    mh = m / (1 - beta1 ** t)
    vh = v / (1 - beta2 ** t)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v
