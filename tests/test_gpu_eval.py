"""Embedding neighbours and neighbourhood precision (Eq. 14) on the GPU against
the oracle's FP64 brute-force kNN of y = s * z.

Bars: neighbour lists identical except where two candidates' FP64 distances
agree to 1e-12 relative (the two sides round the metric differently), sorted
distance sequences within 1e-12 relative everywhere, and precision equal to
the oracle's exactly when no list holds such a near tie.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1611_02568_amd import datagen

pytestmark = pytest.mark.gpu

KS = [1, 3, 5, 10, 20, 30]


@pytest.fixture(scope="module")
def psne():
    from paper_1611_02568_amd import pixelsne
    pixelsne.load()
    assert torch.cuda.is_available()
    return pixelsne


def _knn_check(y, lo, rows=None):
    """lo: GPU lists (caller order) for `rows`; returns rows holding near ties."""
    rows = np.arange(y.shape[0]) if rows is None else rows
    ref, d2 = oracle.knn(y, lo.shape[1], rows=rows)
    tied = []
    for a, i in enumerate(rows):
        if np.array_equal(lo[a], ref[a]):
            continue
        dg = np.sum((y[lo[a]] - y[i]) ** 2, axis=1)
        assert len(set(lo[a].tolist())) == lo.shape[1] and i not in lo[a]
        np.testing.assert_allclose(dg, d2[a], rtol=1e-12, atol=0)
        tied.append(a)
    return ref, tied


def _y(ctx):
    st = ctx.get_state()
    return st["z"].double().cpu().numpy() * np.array(st["s"])


@pytest.mark.parametrize("prec", [0, 1])
def test_knn2d_and_precision_after_steps(psne, prec):
    """2000 points (a ragged last tile of 208), 200 iterations from the standard start."""
    X, _ = datagen.small_mixture(n=2000)
    P = oracle.build_P(X, 30.0)
    hi, _ = oracle.knn(X, 30)
    ctx = psne.Context.from_P(*P, screen=512,
                              Y_init=torch.as_tensor(datagen.initial_embedding(2000, seed=1)),
                              precision=prec)
    ctx.step(200)
    lo = ctx.knn2d().cpu().numpy()
    y = _y(ctx)
    ref, tied = _knn_check(y, lo)
    assert len(tied) <= 2, tied
    got = ctx.neighborhood_precision(torch.as_tensor(hi).cuda(), KS)
    want = oracle.neighborhood_precision(hi, ref, KS)
    for k, g, w in zip(KS, got, want):
        assert abs(g - w) <= len(tied) / (k * 2000), (k, g, w)
    assert want[3] > 4 * 10 / 1999                 # well above chance: neighbourhoods kept


def test_knn2d_sampled_rows_large(psne):
    """20 000 points in several tiles, 400 rows checked one by one."""
    n = 20000
    z = datagen.clustered_pixels(n, 1024, seed=7)
    z = np.minimum(z, np.nextafter(1024.0, 0.0))
    P = _ring_P(n)
    ctx = psne.Context.from_P(*P, screen=1024,
                              Y_init=torch.as_tensor(datagen.initial_embedding(n, seed=2)),
                              precision=1)
    s = (0.013, 0.021)
    ctx.set_state(z, s)
    lo = ctx.knn2d().cpu().numpy()
    rows = np.random.default_rng(3).choice(n, 400, replace=False)
    _, tied = _knn_check(z * np.array(s), lo[rows], rows)
    assert len(tied) <= 4, tied


def test_precision_identity_and_minimum_size(psne):
    """n = 33 (the smallest allowed): every list holds all 32 other points, so
    precision at k = 32 is 1 whatever the high-dimensional order; n = 32 is
    rejected."""
    n = 33
    P = _ring_P(n)
    y0 = datagen.initial_embedding(n, seed=4)
    ctx = psne.Context.from_P(*P, screen=64, Y_init=torch.as_tensor(y0), precision=1)
    ctx.set_state(datagen.uniform_pixels(n, 64, seed=5), (0.1, 0.1))
    rng = np.random.default_rng(6)
    hi = np.stack([rng.permutation(np.delete(np.arange(n), i)) for i in range(n)]).astype(np.int32)
    assert ctx.neighborhood_precision(torch.as_tensor(hi).cuda(), [32]) == [1.0]
    lo = ctx.knn2d().cpu().numpy()
    _knn_check(_y(ctx), lo)
    ctx32 = psne.Context.from_P(*_ring_P(32), screen=64,
                                Y_init=torch.as_tensor(datagen.initial_embedding(32, seed=4)),
                                precision=1)
    with pytest.raises(RuntimeError):
        ctx32.knn2d()
    with pytest.raises(RuntimeError):
        ctx.neighborhood_precision(torch.as_tensor(hi).cuda(), [33])


def _ring_P(n):
    """Each point's two ring neighbours, p = 1/(2n) each (one neighbour for n = 2)."""
    if n == 2:
        return np.array([0, 1, 2], np.int64), np.array([1, 0], np.int32), np.array([0.5, 0.5])
    rp = np.arange(0, 2 * n + 1, 2, dtype=np.int64)
    col = np.stack([(np.arange(n) - 1) % n, (np.arange(n) + 1) % n], 1)
    col = np.sort(col, 1).ravel().astype(np.int32)
    val = np.full(2 * n, 1.0 / (2 * n))
    return rp, col, val
