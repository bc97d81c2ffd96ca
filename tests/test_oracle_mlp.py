"""Pins of the FP64 MLP reference: finite differences, GELU against the normal
CDF, bfloat16 rounding against torch's conversion."""

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


def test_adam_matches_torch_optimizer():
    """Five steps of the reference Adam against torch.optim.Adam (an independent
    implementation) on the same gradient sequence, FP64."""
    rng = np.random.default_rng(4)
    theta = rng.standard_normal(50)
    p = torch.nn.Parameter(torch.tensor(theta.copy()))
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m1 = np.zeros_like(theta)
    m2 = np.zeros_like(theta)
    for t in range(1, 6):
        g = rng.standard_normal(50) * 10.0 ** rng.uniform(-6, 2, 50)
        theta, m1, m2 = mlp.adam_step(theta, m1, m2, g, t, 3e-3)
        p.grad = torch.tensor(g)
        opt.step()
        np.testing.assert_allclose(theta, p.detach().numpy(), rtol=1e-14, atol=1e-16)


def test_adam_first_step_is_sign_descent():
    """From zero moments, step 1 has m_hat = g and v_hat = g^2, so each
    parameter moves by lr * g / (|g| + eps): lr * sign(g) up to eps/|g|."""
    g = np.array([3.0, -2e-3, 1e-5, -7.0, 0.0])
    th, _, _ = mlp.adam_step(np.zeros(5), np.zeros(5), np.zeros(5), g, 1, 0.01)
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-12, atol=0)
    assert th[4] == 0.0 and th[0] < 0 < th[1]


def test_place_clamps_and_scales():
    """With a zero output layer the network outputs its bias b3 for every row:
    the placement is clamp(b3, 0, 1 - 2^-24) * screen * s exactly."""
    d, h1, h2 = 3, 4, 5
    rng = np.random.default_rng(6)
    parts = [rng.standard_normal((d, h1)), np.zeros(h1), rng.standard_normal((h1, h2)),
             np.zeros(h2), np.zeros((h2, 2)), np.array([0.25, 1.5])]
    theta = mlp.flatten(parts)
    X = rng.standard_normal((7, d))
    Y = mlp.place(theta, X, d, h1, h2, np.zeros(d), np.ones(d), 2048, np.array([0.01, 0.003]))
    assert np.all(Y[:, 0] == 0.25 * 2048 * 0.01)
    assert np.all(Y[:, 1] == (1.0 - 2.0 ** -24) * 2048 * 0.003)
    parts[5] = np.array([-0.5, 0.0])
    Y = mlp.place(mlp.flatten(parts), X, d, h1, h2, np.zeros(d), np.ones(d), 512, np.ones(2))
    assert np.all(Y == 0.0)


def test_place_standardises_inputs():
    """Placement of x with (mean, inv_std) equals placement of the
    standardised rows with the identity standardisation."""
    theta, X, _, d, h1, h2 = _small(seed=8)
    mu = np.linspace(-1, 1, d)
    isd = np.linspace(0.5, 2, d)
    a = mlp.place(theta, X, d, h1, h2, mu, isd, 1024, np.array([0.1, 0.2]))
    b = mlp.place(theta, (X - mu) * isd, d, h1, h2, np.zeros(d), np.ones(d), 1024,
                  np.array([0.1, 0.2]))
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-300)
    out, _ = mlp.forward(theta, (X - mu) * isd, d, h1, h2)
    inside = (out > 0) & (out < 1 - 2.0 ** -24)
    np.testing.assert_allclose(a[inside], (out * 1024 * np.array([0.1, 0.2]))[inside], rtol=1e-13)
