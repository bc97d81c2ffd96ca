"""Seeded synthetic inputs shared by the GPU path, the oracle and the benchmark.

This module only draws random inputs.  It holds none of the method's
arithmetic (no distances, affinities, trees or gradients), so that the GPU
path and the CPU oracle can both consume identical arrays while sharing no
code that computes anything PixelSNE defines.

The paper evaluates on MNIST, a facial-expression CNN feature set, two
word2vec-averaged news corpora and Yelp (Section 5.1.1).  None of those are
available here, so each workload below is a Gaussian-mixture stand-in with
the shape (n, D), value type and cluster structure of the workload it
replaces.  Random numbers the method itself draws (the initial embedding) are
produced here as well and passed in as inputs.

Seeds: data = 161102568 + 10 * cfg, initial embedding = data + 1,
held-out draws = data + 2.
"""
from __future__ import annotations

import numpy as np

BASE_SEED = 161102568


def seed_for(cfg: int, offset: int = 0) -> int:
    return BASE_SEED + 10 * cfg + offset


def _largest_remainder(n: int, w: np.ndarray) -> np.ndarray:
    """Integer sizes summing to n, proportional to weights w."""
    w = np.asarray(w, dtype=np.float64)
    q = n * w / w.sum()
    sizes = np.floor(q).astype(np.int64)
    rem = n - int(sizes.sum())
    if rem > 0:
        order = np.argsort(-(q - sizes), kind="stable")
        sizes[order[:rem]] += 1
    return sizes


def _mixture(rng, n, D, means, sigmas, sizes, dtype):
    X = np.empty((n, D), dtype=dtype)
    labels = np.empty(n, dtype=np.int32)
    off = 0
    for k, m in enumerate(sizes):
        m = int(m)
        if m == 0:
            continue
        blk = rng.standard_normal((m, D)).astype(np.float64)
        blk *= sigmas[k]
        blk += means[k]
        X[off:off + m] = blk.astype(dtype)
        labels[off:off + m] = k
        off += m
    perm = rng.permutation(n)
    return X[perm], labels[perm]


def small_mixture(n: int = 2000, D: int = 50, K: int = 10, seed: int | None = None,
                  dtype=np.float64):
    """10-component isotropic mixture: means ~ N(0, 25 I), unit variance,
    equal weights, rows shuffled.  Default shape is the 2,000 x 50 float64
    parity workload (screen 512, perplexity 30)."""
    rng = np.random.default_rng(seed_for(0) if seed is None else seed)
    means = rng.standard_normal((K, D)) * 5.0
    sizes = _largest_remainder(n, np.ones(K))
    return _mixture(rng, n, D, means, np.ones(K), sizes, dtype)


def uint8_mixture(n: int = 70000, D: int = 784, K: int = 10, seed: int | None = None):
    """MNIST-shaped stand-in: per-cluster Bernoulli(0.2) support masks (about
    80% zeros), prototypes ~ N(128, 48^2) on the mask, samples = prototype +
    N(0, 32^2), each on-mask entry dropped with probability 0.1, rounded and
    clipped to 0..255, stored as uint8."""
    rng = np.random.default_rng(seed_for(1) if seed is None else seed)
    masks = rng.random((K, D)) < 0.2
    protos = np.clip(rng.normal(128.0, 48.0, (K, D)), 0, 255) * masks
    sizes = _largest_remainder(n, np.ones(K))
    X = np.zeros((n, D), dtype=np.uint8)
    labels = np.empty(n, dtype=np.int32)
    off = 0
    for k, m in enumerate(sizes):
        m = int(m)
        v = protos[k][None, :] + rng.normal(0.0, 32.0, (m, D))
        keep = masks[k][None, :] & (rng.random((m, D)) >= 0.1)
        v = np.clip(np.rint(v), 0, 255) * keep
        X[off:off + m] = v.astype(np.uint8)
        labels[off:off + m] = k
        off += m
    perm = rng.permutation(n)
    return X[perm], labels[perm]


class ZipfMixture:
    """Gaussian mixture with Zipf(a) component weights, means ~ N(0, 25 I)
    and per-component isotropic variance ~ U(0.5, 2).  Draws are reproducible
    from the mixture seed; held-out draws use a separate seed but the same
    components."""

    def __init__(self, K: int, D: int, a: float, seed: int):
        rng = np.random.default_rng(seed)
        self.K, self.D, self.a = K, D, a
        self.weights = np.arange(1, K + 1, dtype=np.float64) ** (-a)
        self.means = rng.standard_normal((K, D)) * 5.0
        self.sigmas = np.sqrt(rng.uniform(0.5, 2.0, K))
        self._rng = rng

    def sample(self, n: int, rng=None, dtype=np.float32):
        rng = self._rng if rng is None else rng
        sizes = _largest_remainder(n, self.weights)
        return _mixture(rng, n, self.D, self.means, self.sigmas, sizes, dtype)


def zipf_mixture_1m(n: int = 1_000_000, D: int = 128, K: int = 100, a: float = 1.1,
                    seed: int | None = None):
    """Yelp-sized stand-in: 1,000,000 x 128 float32, 100 components with
    Zipf(1.1) sizes (largest-remainder rounding), variance ~ U(0.5, 2)."""
    mix = ZipfMixture(K, D, a, seed_for(2) if seed is None else seed)
    X, lab = mix.sample(n)
    return X, lab, mix


def heldout(mix: ZipfMixture, n: int = 200_000, seed: int | None = None):
    """Fresh draws from an existing mixture (held-out placement workload)."""
    rng = np.random.default_rng(seed_for(3, 2) if seed is None else seed)
    return mix.sample(n, rng=rng)


def zipf_mixture_outliers(n: int = 5_000_000, D: int = 100, K: int = 1000, a: float = 1.3,
                          outlier_frac: float = 0.01, seed: int | None = None):
    """5,000,000 x 100 float32: Zipf(1.3) mixture of 1,000 components plus 1%
    outliers drawn uniformly in the bounding box of the means expanded by
    three times the largest component standard deviation."""
    s = seed_for(4) if seed is None else seed
    mix = ZipfMixture(K, D, a, s)
    n_out = int(round(n * outlier_frac))
    X, lab = mix.sample(n - n_out)
    lo = mix.means.min(0) - 3 * mix.sigmas.max()
    hi = mix.means.max(0) + 3 * mix.sigmas.max()
    rng = np.random.default_rng(s + 5)
    O = rng.uniform(lo, hi, (n_out, D)).astype(np.float32)
    X = np.concatenate([X, O])
    lab = np.concatenate([lab, np.full(n_out, -1, np.int32)])
    perm = rng.permutation(n)
    return X[perm], lab[perm], mix


def initial_embedding(n: int, seed: int, sigma: float = 1e-4, dim: int = 2) -> np.ndarray:
    """y(0) ~ N(0, sigma^2 I) in dim dimensions, float64, shape (n, dim)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal((n, dim)) * sigma


def uniform_pixels(n: int, r: int, seed: int, dtype=np.float64, dim: int = 2) -> np.ndarray:
    """n positions uniform over the screen [0, r)^dim (tree and traversal tests)."""
    rng = np.random.default_rng(seed)
    top = np.nextafter(np.asarray(r, dtype), np.asarray(0, dtype))
    return np.minimum((rng.random((n, dim)) * r).astype(dtype), top)


def clustered_pixels(n: int, r: int, seed: int, n_clusters: int = 8, spread: float = 0.02,
                     dtype=np.float64, dim: int = 2) -> np.ndarray:
    """n positions in [0, r)^dim concentrated in a few tight blobs (many points
    share a pixel), with min 0 and the max pixel r - 1 on each axis so the
    whole screen is spanned as after normalisation."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_clusters, dim)) * r
    lab = rng.integers(0, n_clusters, n)
    z = centres[lab] + rng.standard_normal((n, dim)) * (spread * r)
    top = np.nextafter(np.asarray(r, dtype), np.asarray(0, dtype))
    z = np.clip(z.astype(dtype), np.asarray(0, dtype), top)
    z[0] = 0
    z[1] = top
    return z


def circulant_affinities(n: int, half_degree: int, seed: int):
    """A symmetric sparse matrix of n rows with 2 * half_degree nonzeros per row,
    standing in for P at a given size and row length where building P from
    data would take too long on the CPU: row i holds the columns i +- d mod n
    for half_degree distinct random offsets d in [1, n / 2), with a positive
    random weight per unordered pair (the same for (i, j) and (j, i)), all
    weights scaled to sum to 1.  Returns (row_ptr int64 [n+1], col int32 [nnz]
    ascending per row, val float64 [nnz])."""
    rng = np.random.default_rng(seed)
    offs = rng.choice(np.arange(1, (n - 1) // 2), size=half_degree, replace=False)
    offs = np.concatenate([offs, -offs]).astype(np.int64)
    rows = np.arange(n, dtype=np.int64)[:, None]
    col = np.sort((rows + offs[None, :]) % n, axis=1)
    lo = np.minimum(rows, col)
    hi = np.maximum(rows, col)
    h = (lo * 0x9E3779B1 + hi * 0x85EBCA77 + seed) & 0xFFFFFFFF
    h = (h ^ (h >> 15)) * 0x2C1B3C6D & 0xFFFFFFFF
    h = h ^ (h >> 12)
    val = 0.5 + (h & 0xFFFF).astype(np.float64) / 65536.0
    val /= val.sum()
    deg = 2 * half_degree
    rp = np.arange(0, n * deg + 1, deg, dtype=np.int64)
    return rp, col.astype(np.int32).ravel(), val.ravel()
