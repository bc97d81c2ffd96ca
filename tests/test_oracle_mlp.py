"""Pins of the FP64 MLP reference: finite differences, GELU against the normal
CDF, bfloat16 rounding against torch's conversion."""
import math

import numpy as np
import torch
from scipy.stats import norm

from oracle import mlp


def _small(seed=0, d=5, h1=7, h2=6, B=9):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(sum(int(np.prod(s)) for s in mlp.shapes(d, h1, h2))) * 0.5
    X = rng.standard_normal((B, d))
    Y = rng.random((B, 2))
    return theta, X, Y, d, h1, h2


def test_gradient_matches_finite_differences():
    theta, X, Y, d, h1, h2 = _small()
    L, g = mlp.grads(theta, X, Y, d, h1, h2)
    assert abs(L - mlp.loss(theta, X, Y, d, h1, h2)) < 1e-15 * max(1.0, L)
    h = 1e-6
    fd = np.empty_like(theta)
    for i in range(theta.size):
        tp = theta.copy(); tp[i] += h
        tm = theta.copy(); tm[i] -= h
        fd[i] = (mlp.loss(tp, X, Y, d, h1, h2) - mlp.loss(tm, X, Y, d, h1, h2)) / (2 * h)
    assert np.max(np.abs(fd - g)) <= 1e-6 * np.max(np.abs(g))


def test_gelu_is_x_times_normal_cdf():
    x = np.linspace(-8, 8, 2001)
    np.testing.assert_allclose(mlp.gelu(x), x * norm.cdf(x), rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(mlp.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.standard_normal(10000) * 10 ** rng.uniform(-5, 5, 10000),
                        [1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, -1 - 2 ** -8, 0.0, -0.0]])
    ref = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(mlp.bf16(x), ref)
    assert mlp.bf16(1 + 2 ** -8) == 1.0 and mlp.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


def test_bf16_emulation_is_close_to_fp64():
    theta, X, Y, d, h1, h2 = _small(seed=3, d=16, h1=32, h2=24, B=64)
    _, g = mlp.grads(theta, X, Y, d, h1, h2)
    _, gb = mlp.grads(theta, X, Y, d, h1, h2, bf=True)
    assert np.linalg.norm(gb - g) <= 3e-2 * np.linalg.norm(g)
