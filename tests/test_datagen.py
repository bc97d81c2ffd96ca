"""The seeded input generators against the recipes they state: shapes, value
types, component sizes, seeds and reproducibility (CPU only, reduced sizes
where the recipe does not depend on n)."""
import numpy as np

from paper_1611_02568_amd import datagen


def test_seeds():
    assert datagen.seed_for(0) == 161102568
    assert datagen.seed_for(2, 1) == 161102568 + 21


def test_largest_remainder_sizes():
    w = np.arange(1, 101, dtype=np.float64) ** -1.1
    for n in (1, 999, 1_000_000):
        s = datagen._largest_remainder(n, w)
        assert s.sum() == n and (s >= 0).all()
        q = n * w / w.sum()
        assert np.all(np.abs(s - q) < 1.0)


def test_small_mixture():
    X, lab = datagen.small_mixture()
    assert X.shape == (2000, 50) and X.dtype == np.float64
    assert np.array_equal(np.bincount(lab), np.full(10, 200))
    X2, lab2 = datagen.small_mixture()
    assert np.array_equal(X, X2) and np.array_equal(lab, lab2)
    X3, _ = datagen.small_mixture(seed=1)
    assert not np.array_equal(X, X3)
    # unit variance around each component's mean
    for k in range(10):
        rows = X[lab == k]
        assert abs(rows.var(axis=0, ddof=1).mean() - 1.0) < 0.1


def test_uint8_mixture():
    X, lab = datagen.uint8_mixture(n=2000)
    assert X.shape == (2000, 784) and X.dtype == np.uint8
    assert np.array_equal(np.bincount(lab), np.full(10, 200))
    # support 0.2, 10% of it dropped: about 82% zeros or more (clipping adds some)
    zeros = (X == 0).mean()
    assert 0.80 <= zeros <= 0.86
    X2, _ = datagen.uint8_mixture(n=2000)
    assert np.array_equal(X, X2)


def test_zipf_mixture_sizes_and_spread():
    n = 20_000
    X, lab, mix = datagen.zipf_mixture_1m(n=n)
    assert X.shape == (n, 128) and X.dtype == np.float32
    assert mix.K == 100 and mix.a == 1.1
    assert np.array_equal(np.bincount(lab, minlength=100),
                          datagen._largest_remainder(n, np.arange(1, 101) ** -1.1))
    assert ((mix.sigmas ** 2 >= 0.5) & (mix.sigmas ** 2 <= 2.0)).all()
    for k in range(3):
        rows = X[lab == k].astype(np.float64)
        assert np.abs(rows.mean(axis=0) - mix.means[k]).max() < 6 * mix.sigmas[k] / np.sqrt(len(rows)) + 1e-3
        assert abs(rows.var(axis=0, ddof=1).mean() / mix.sigmas[k] ** 2 - 1.0) < 0.05
    # the held-out draws come from the same components, with other numbers
    H, hl = datagen.heldout(mix, n=5000)
    assert H.shape == (5000, 128)
    assert np.array_equal(np.bincount(hl, minlength=100),
                          datagen._largest_remainder(5000, mix.weights))
    rows = H[hl == 0].astype(np.float64)
    assert np.abs(rows.mean(axis=0) - mix.means[0]).max() < 6 * mix.sigmas[0] / np.sqrt(len(rows)) + 1e-3


def test_outlier_mixture():
    n = 20_000
    X, lab, mix = datagen.zipf_mixture_outliers(n=n, K=50)
    assert X.shape == (n, 100) and X.dtype == np.float32
    out = lab == -1
    assert out.sum() == 200
    lo = mix.means.min(0) - 3 * mix.sigmas.max()
    hi = mix.means.max(0) + 3 * mix.sigmas.max()
    assert (X[out] >= lo.astype(np.float32) - 1e-4).all() and (X[out] <= hi.astype(np.float32) + 1e-4).all()
    assert np.array_equal(np.bincount(lab[~out], minlength=50),
                          datagen._largest_remainder(n - 200, mix.weights))


def test_initial_embedding_and_screens():
    y = datagen.initial_embedding(100_000, seed=7)
    assert y.shape == (100_000, 2) and y.dtype == np.float64
    assert abs(y.std() / 1e-4 - 1.0) < 0.01
    assert np.array_equal(y, datagen.initial_embedding(100_000, seed=7))
    y3 = datagen.initial_embedding(10, seed=7, dim=3)
    assert y3.shape == (10, 3)
    for dim in (2, 3):
        u = datagen.uniform_pixels(5000, 64, seed=1, dim=dim)
        assert u.shape == (5000, dim) and (u >= 0).all() and (u < 64).all()
        c = datagen.clustered_pixels(5000, 64, seed=1, dim=dim)
        assert (c >= 0).all() and (c < 64).all()
        assert (c.min(0) == 0).all() and (np.floor(c.max(0)) == 63).all()


def test_circulant_affinities():
    n, h = 1000, 7
    rp, col, val = datagen.circulant_affinities(n, h, seed=3)
    assert rp.dtype == np.int64 and col.dtype == np.int32 and val.dtype == np.float64
    assert np.array_equal(rp, np.arange(0, n * 2 * h + 1, 2 * h))
    assert abs(val.sum() - 1.0) < 1e-12 and (val > 0).all()
    rows = np.repeat(np.arange(n), 2 * h)
    assert (col != rows).all()
    assert all((np.diff(col[rp[i]:rp[i + 1]]) > 0).all() for i in range(n))
    dense = np.zeros((n, n))
    dense[rows, col] = val
    assert np.array_equal(dense, dense.T)
