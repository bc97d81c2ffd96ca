"""Textbook exact t-SNE in NumPy (FP64, O(n^2)) -- TEST INFRASTRUCTURE ONLY.

An independent second reference used to pin the C oracle: it works directly
in the embedding frame y with dense matrices, in the textbook form of the
objective and gradient (paper Eq. 3-5), with no tree, no pixel frame and no
code shared with the C oracle.

  w_ij = 1 / (1 + |y_i - y_j|^2),  Z = sum_{k != l} w_kl,  q_ij = w_ij / Z  (Eq. 3)
  C    = sum_{i != j} p_ij log(p_ij / q_ij)                                  (Eq. 4)
  dC/dy_i = 4 sum_j (p_ij - q_ij) w_ij (y_i - y_j)                          (Eq. 5)
"""
from __future__ import annotations

import numpy as np


def kernel(Y):
    Y = np.asarray(Y, dtype=np.float64)
    diff = Y[:, None, :] - Y[None, :, :]
    W = 1.0 / (1.0 + np.sum(diff * diff, axis=-1))
    np.fill_diagonal(W, 0.0)
    return W, diff


def kl(Y, P) -> float:
    """Eq. 4 over all i != j with dense P (zero entries contribute 0)."""
    W, _ = kernel(Y)
    Q = W / W.sum()
    P = np.asarray(P, dtype=np.float64)
    mask = P > 0
    return float(np.sum(P[mask] * np.log(P[mask] / Q[mask])))


def gradient(Y, P, alpha: float = 1.0):
    """Eq. 5 with P multiplied by alpha (early exaggeration)."""
    W, diff = kernel(Y)
    Q = W / W.sum()
    M = (alpha * np.asarray(P, dtype=np.float64) - Q) * W
    return 4.0 * np.einsum("ij,ijd->id", M, diff)


def repulsion(Y):
    """(sum_j w_ij^2 (y_i - y_j), Z) -- the un-normalised repulsive term."""
    W, diff = kernel(Y)
    return np.einsum("ij,ijd->id", W * W, diff), float(W.sum())


def attraction(Y, P):
    """sum_j p_ij w_ij (y_i - y_j)."""
    W, diff = kernel(Y)
    return np.einsum("ij,ijd->id", np.asarray(P, dtype=np.float64) * W, diff)


def dense_from_csr(P, n: int):
    rp, col, val = P
    D = np.zeros((n, n))
    for i in range(n):
        D[i, col[rp[i]:rp[i + 1]]] = val[rp[i]:rp[i + 1]]
    return D


def run(Y0, P, n_iter: int, eta: float = 200.0, mom0: float = 0.5, mom1: float = 0.8,
        mom_switch: int = 250, exaggeration: float = 12.0, exag_iters: int = 250,
        min_gain: float = 0.01, t0: int = 0):
    """Plain exact t-SNE in the y frame with the Barnes-Hut-SNE optimiser
    (gains, momentum, early exaggeration), stepping on dC/dy / 4."""
    Y = np.array(Y0, dtype=np.float64)
    U = np.zeros_like(Y)
    G = np.ones_like(Y)
    for it in range(n_iter):
        t = t0 + it
        alpha = exaggeration if t < exag_iters else 1.0
        mu = mom0 if t < mom_switch else mom1
        dY = gradient(Y, P, alpha) / 4.0
        flip = np.sign(dY) != np.sign(U)
        G = np.where(flip, G + 0.2, G * 0.8)
        G = np.maximum(G, min_gain)
        U = mu * U - eta * G * dY
        Y = Y + U
    return Y
