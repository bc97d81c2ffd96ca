"""GPU placement network against the FP64 reference with bfloat16 emulation.

Bars: gradient norm-wise rel <= 1e-3 per parameter block and loss rel <= 1e-4
(FP32 accumulation order and FP32 vs FP64 GELU are the only differences from
the emulated reference); forward rel <= 1e-3.  Adam: the FP32 update against
the FP64 one to FP32 rounding.  Placement: the clamped outputs bit-exact where
the network's output is clearly outside [0, 1), otherwise within the forward
bar.
"""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def psne():
    from paper_1611_02568_amd import pixelsne
    pixelsne.load()
    return pixelsne


def _setup(psne, d, h1, h2, n, seed):
    rng = np.random.default_rng(seed)
    net = psne.MLP(d, h1, h2, seed=seed)
    theta = (rng.standard_normal(net.n_params) * 0.2).astype(np.float32)
    net.set_params(torch.as_tensor(theta))
    net.set_norm(np.zeros(d, np.float32), np.ones(d, np.float32))
    X = rng.standard_normal((n, d)).astype(np.float32)
    Y = rng.random((n, 2)).astype(np.float32)
    return net, theta.astype(np.float64), X, Y


@pytest.mark.parametrize("d,h1,h2,n", [(100, 130, 70, 333), (128, 512, 512, 512),
                                       (100, 1024, 1024, 300), (16, 64, 64, 2048), (1, 3, 5, 7)])
def test_grad_parity(psne, d, h1, h2, n):
    net, theta, X, Y = _setup(psne, d, h1, h2, n, seed=d + n)
    loss, g = net.grad(torch.as_tensor(X).cuda(), torch.as_tensor(Y).cuda())
    L, gr = omlp.grads(theta, X.astype(np.float64), Y.astype(np.float64), d, h1, h2, bf=True)
    assert abs(loss - L) <= 1e-4 * L
    g = g.double().cpu().numpy()
    off = 0
    for s in omlp.shapes(d, h1, h2):
        m = int(np.prod(s))
        a, b = g[off:off + m], gr[off:off + m]
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-12, (s, np.linalg.norm(a - b) / np.linalg.norm(b))
        off += m


def test_forward_parity(psne):
    d, h1, h2, n = 128, 512, 512, 3000
    net, theta, X, Y = _setup(psne, d, h1, h2, n, seed=5)
    out = net.forward(torch.as_tensor(X).cuda()).double().cpu().numpy()
    ref, _ = omlp.forward(theta, X.astype(np.float64), d, h1, h2, bf=True)
    assert np.linalg.norm(out - ref) <= 1e-3 * np.linalg.norm(ref)


def test_fit_norm_matches_numpy(psne):
    """Standardisation fitted on the GPU gives the same outputs as NumPy's."""
    rng = np.random.default_rng(8)
    X = (rng.standard_normal((5000, 37)) * rng.uniform(0.5, 9, 37)
         + rng.uniform(-3, 3, 37)).astype(np.float32)
    mu, sd = omlp.standardize_stats(X)
    a_net, b_net = psne.MLP(37, 8, 8, seed=1), psne.MLP(37, 8, 8, seed=1)
    a_net.fit_norm(torch.as_tensor(X).cuda())
    b_net.set_norm(mu.astype(np.float32), (1.0 / sd).astype(np.float32))
    theta = (rng.standard_normal(a_net.n_params) * 0.3).astype(np.float32)
    a_net.set_params(torch.as_tensor(theta))
    b_net.set_params(torch.as_tensor(theta))
    a = a_net.forward(torch.as_tensor(X).cuda()).cpu().numpy()
    b = b_net.forward(torch.as_tensor(X).cuda()).cpu().numpy()
    assert np.max(np.abs(a - b)) <= 2e-2 * np.max(np.abs(b))


def test_training_fits_a_smooth_map(psne):
    """Training with the GPU kernels drives the loss down on a learnable target."""
    rng = np.random.default_rng(11)
    n, d = 20000, 32
    X = rng.standard_normal((n, d)).astype(np.float32)
    W = rng.standard_normal((d, 2)) / np.sqrt(d)
    Y = (1.0 / (1.0 + np.exp(-(X @ W)))).astype(np.float32)          # in (0, 1)
    net = psne.MLP(d, 128, 128, seed=3)
    Xd, Yd = torch.as_tensor(X).cuda(), torch.as_tensor(Y).cuda()
    net.fit_norm(Xd)
    l0, _ = net.grad(Xd[:4096], Yd[:4096])
    lt = net.train(Xd, Yd, epochs=20, batch=1024, lr=1e-3)
    l1, _ = net.grad(Xd[:4096], Yd[:4096])
    assert lt < 0.05 * l0 and l1 < 0.05 * l0, (l0, lt, l1)


def test_adam_step_parity(psne):
    """Four Adam steps with caller gradients of widely spread magnitudes
    against the FP64 reference started from the same FP32 parameters: each
    FP32 update carries a few roundings (relative 1e-6) and the parameters
    are rounded to FP32 after each step."""
    d, h1, h2 = 24, 40, 32
    rng = np.random.default_rng(21)
    net = psne.MLP(d, h1, h2, seed=2)
    theta = (rng.standard_normal(net.n_params) * 0.2).astype(np.float32)
    net.set_params(torch.as_tensor(theta))
    th = theta.astype(np.float64)
    m1 = np.zeros_like(th)
    m2 = np.zeros_like(th)
    lr = 2e-3
    for t in range(1, 5):
        g = (rng.standard_normal(net.n_params) * 10.0 ** rng.uniform(-7, 1, net.n_params))
        g = g.astype(np.float32)
        net.adam_step(torch.as_tensor(g), lr)
        th, m1, m2 = omlp.adam_step(th, m1, m2, g.astype(np.float64), t, lr)
        got = net.params().double().cpu().numpy()
        tol = t * (2.0 ** -23 * np.abs(th) + 1e-5 * lr)
        assert np.all(np.abs(got - th) <= tol), (t, np.max(np.abs(got - th) / tol))
    moved = np.abs(net.params().double().cpu().numpy() - theta.astype(np.float64))
    assert np.median(moved) > lr                       # the steps did move the parameters


def test_place_parity(psne):
    """Placement (standardise, forward, clamp to [0, 1 - 2^-24], times screen
    and s) against the FP64 reference with bfloat16 emulation."""
    d, h1, h2, n, screen = 128, 512, 512, 4000, 2048
    net, theta, X, _ = _setup(psne, d, h1, h2, n, seed=12)
    # outputs spread around the screen's middle, partly beyond either edge
    parts = omlp.unflatten(theta, d, h1, h2)
    parts[4] *= 0.03
    parts[5][:] = 0.5
    theta = omlp.flatten(parts).astype(np.float32).astype(np.float64)
    net.set_params(torch.as_tensor(theta.astype(np.float32)))
    rng = np.random.default_rng(13)
    mu = rng.uniform(-0.5, 0.5, d).astype(np.float32)
    isd = rng.uniform(0.5, 2.0, d).astype(np.float32)
    net.set_norm(mu, isd)
    s = np.array([0.0123, 0.0071])
    Y = net.place(torch.as_tensor(X).cuda(), screen, s).cpu().numpy()
    Xs = ((X - mu) * isd).astype(np.float32).astype(np.float64)   # standardised in FP32
    ref = omlp.place(theta, Xs, d, h1, h2, np.zeros(d), np.ones(d), screen, s, bf=True)
    out, _ = omlp.forward(theta, Xs, d, h1, h2, bf=True)
    scale = screen * s[None, :]
    top = 1.0 - 2.0 ** -24
    lo, hi = out < -1e-2, out > 1.0 + 1e-2
    assert lo.sum() > 100 and hi.sum() > 100 and (~lo & ~hi).sum() > 100
    assert np.all(Y[lo] == 0.0)
    assert np.all(Y[hi] == (top * screen * np.broadcast_to(s, Y.shape))[hi])
    mid = ~lo & ~hi
    err = np.abs(Y - ref) / scale
    assert np.linalg.norm(err[mid]) <= 1e-3 * np.linalg.norm(np.abs(out[mid]))


def test_place_with_zero_output_layer(psne):
    """A zero output layer places every point at its bias b3, clamped."""
    d, h1, h2 = 20, 64, 64
    net = psne.MLP(d, h1, h2, seed=4)
    th = net.params().cpu().numpy()
    parts = omlp.unflatten(th, d, h1, h2)
    parts[4][:] = 0.0
    parts[5][:] = (0.375, 7.0)
    net.set_params(torch.as_tensor(omlp.flatten(parts).astype(np.float32)))
    X = torch.randn(999, d, device="cuda")
    Y = net.place(X, 1024, (0.5, 0.25)).cpu().numpy()
    assert np.all(Y[:, 0] == 0.375 * 1024 * 0.5)
    assert np.all(Y[:, 1] == (1.0 - 2.0 ** -24) * 1024 * 0.25)
