"""FP64 reference of the element-block cost model -- TEST ONLY.

A multilayer perceptron 12 -> 64 -> 64 -> 1 with ReLU hidden layers predicts
the log of a work item's measured assembly cycles from its features. The
paper observes that an element's cost cannot be estimated a priori and that
the number of Gauss points is a poor weight (abstract; Section 4.1); this
model learns the weight from cycle counts the assembly records.

Parameters are one flat vector, in this order: W1[64,12] (row-major), b1[64],
W2[64,64], b2[64], W3[64], b3[1] (5,057 values). Inputs are standardised
with a fixed per-feature mean and scale before the first layer. Training
minimises the mean squared error with Adam (beta1 0.9, beta2 0.999,
eps 1e-8, bias-corrected).
"""
from __future__ import annotations

import numpy as np

N_IN, N_H = 12, 64
SIZES = [(N_H, N_IN), (N_H,), (N_H, N_H), (N_H,), (N_H,), (1,)]
N_PARAMS = sum(int(np.prod(s)) for s in SIZES)


def unpack(theta):
    out, o = [], 0
    for s in SIZES:
        n = int(np.prod(s))
        out.append(theta[o:o + n].reshape(s))
        o += n
    return out


def init(seed):
    """He-normal weights, zero biases (seeded)."""
    rng = np.random.default_rng(seed)
    W1 = rng.standard_normal((N_H, N_IN)) * np.sqrt(2.0 / N_IN)
    W2 = rng.standard_normal((N_H, N_H)) * np.sqrt(2.0 / N_H)
    W3 = rng.standard_normal(N_H) * np.sqrt(2.0 / N_H)
    return np.concatenate([W1.ravel(), np.zeros(N_H), W2.ravel(), np.zeros(N_H), W3, [0.0]])


def forward(theta, X, mean, scale):
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    Z = (X - mean) / scale
    a1 = Z @ W1.T + b1
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ W2.T + b2
    h2 = np.maximum(a2, 0.0)
    y = h2 @ W3 + b3[0]
    return y, (Z, a1, h1, a2, h2)


def loss_grad(theta, X, t, mean, scale):
    """Mean squared error and its gradient (flat, same layout as theta)."""
    W1, b1, W2, b2, W3, b3 = unpack(theta)
    y, (Z, a1, h1, a2, h2) = forward(theta, X, mean, scale)
    n = X.shape[0]
    r = y - t
    loss = float(np.mean(r * r))
    dy = 2.0 * r / n
    gW3 = h2.T @ dy
    gb3 = np.array([dy.sum()])
    dh2 = np.outer(dy, W3)
    da2 = dh2 * (a2 > 0)
    gW2 = da2.T @ h1
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ W2
    da1 = dh1 * (a1 > 0)
    gW1 = da1.T @ Z
    gb1 = da1.sum(axis=0)
    g = np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2, gW3, gb3])
    return loss, g


def adam_step(theta, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step counts from 1). Returns new (theta, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
