"""FP64 reference of the learned placement network -- TEST INFRASTRUCTURE ONLY.

A small MLP x -> (z1/r, z2/r) maps a point to its position on the screen of a
converged PixelSNE embedding: Linear - GELU - Linear - GELU - Linear, trained
with the mean squared error
    loss = (1/B) sum_b sum_d (out_bd - y_bd)^2.
GELU is the exact form x * Phi(x).  The GPU kernels feed every matrix product
with bfloat16 operands and accumulate in FP32; ``forward``/``grads`` with
``bf16=True`` round the same operands to bfloat16 (round to nearest even) at
the same points so that the two can be compared:
  forward:  X, W1 | H1, W2 | H2, W3 rounded before each product
  backward: dA2, H1, W2 and dA1, X rounded before the products that use them;
            the 2-wide head (dW3, dH2) uses the rounded H2 and W3.
Without ``bf16`` everything is FP64 (pinned by finite differences).

Parameters are a flat vector: W1 [d,h1], b1 [h1], W2 [h1,h2], b2 [h2],
W3 [h2,2], b3 [2] (row-major).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def shapes(d, h1, h2):
    return [(d, h1), (h1,), (h1, h2), (h2,), (h2, 2), (2,)]


def unflatten(theta, d, h1, h2):
    out, o = [], 0
    for s in shapes(d, h1, h2):
        m = int(np.prod(s))
        out.append(np.asarray(theta[o:o + m], dtype=np.float64).reshape(s))
        o += m
    return out


def flatten(parts):
    return np.concatenate([np.asarray(p, dtype=np.float64).ravel() for p in parts])


def bf16(x):
    """Round to bfloat16 (via float32, both round-to-nearest-even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2 * math.pi)


def forward(theta, X, d, h1, h2, bf=False):
    W1, b1, W2, b2, W3, b3 = unflatten(theta, d, h1, h2)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    A1 = r(X) @ r(W1) + b1
    H1 = gelu(A1)
    A2 = r(H1) @ r(W2) + b2
    H2 = gelu(A2)
    out = r(H2) @ r(W3) + b3
    return out, (A1, H1, A2, H2)


def loss(theta, X, Y, d, h1, h2, bf=False):
    out, _ = forward(theta, X, d, h1, h2, bf)
    return float(np.sum((out - Y) ** 2) / X.shape[0])


def grads(theta, X, Y, d, h1, h2, bf=False):
    """(loss, flat gradient) of the mean squared error."""
    W1, b1, W2, b2, W3, b3 = unflatten(theta, d, h1, h2)
    r = bf16 if bf else (lambda a: np.asarray(a, dtype=np.float64))
    out, (A1, H1, A2, H2) = forward(theta, X, d, h1, h2, bf)
    B = X.shape[0]
    L = float(np.sum((out - Y) ** 2) / B)
    dout = 2.0 * (out - Y) / B
    dW3 = r(H2).T @ dout
    db3 = dout.sum(0)
    dA2 = (dout @ r(W3).T) * gelu_grad(A2)
    dW2 = r(H1).T @ r(dA2)
    db2 = dA2.sum(0)
    dA1 = (r(dA2) @ r(W2).T) * gelu_grad(A1)
    dW1 = r(X).T @ r(dA1)
    db1 = dA1.sum(0)
    return L, flatten([dW1, db1, dW2, db2, dW3, db3])


def standardize_stats(X):
    """Per-feature mean and standard deviation (population), FP64."""
    X = np.asarray(X, dtype=np.float64)
    mu = X.mean(0)
    sd = X.std(0)
    sd[sd == 0] = 1.0
    return mu, sd


def adam_step(theta, m1, m2, grad, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba, 2015, Algorithm 1), step number t >= 1:
    biased first and second moment estimates, their bias corrections by
    1 - b^t, and theta - lr * m_hat / (sqrt(v_hat) + eps).  FP64.
    Returns (theta, m1, m2)."""
    g = np.asarray(grad, dtype=np.float64)
    m1 = b1 * np.asarray(m1, dtype=np.float64) + (1.0 - b1) * g
    m2 = b2 * np.asarray(m2, dtype=np.float64) + (1.0 - b2) * g * g
    m_hat = m1 / (1.0 - b1 ** t)
    v_hat = m2 / (1.0 - b2 ** t)
    return np.asarray(theta, dtype=np.float64) - lr * m_hat / (np.sqrt(v_hat) + eps), m1, m2


def place(theta, X, d, h1, h2, mean, inv_std, screen, s, bf=False):
    """Initial embedding of new points from the network: the standardised
    input (x - mean) * inv_std through the MLP, each output clamped to
    [0, 1 - 2^-24] (the screen's half-open range), then scaled to the pixel
    frame (times screen) and to y units (times s per axis).  FP64 [n, 2]."""
    Xs = (np.asarray(X, dtype=np.float64) - np.asarray(mean, dtype=np.float64)) * \
        np.asarray(inv_std, dtype=np.float64)
    out, _ = forward(theta, Xs, d, h1, h2, bf)
    top = 1.0 - 2.0 ** -24
    return np.clip(out, 0.0, top) * float(screen) * np.asarray(s, dtype=np.float64)[None, :]
