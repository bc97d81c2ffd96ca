"""Pins of the oracle's 3-D embedding (voxel octree, three-axis scaling).

Section 1 notes that the method carries over to 3-D embeddings; the oracle's
3-D functions run the 2-D steps over three axes.  They are checked here
against the textbook exact t-SNE (dimension-generic NumPy), finite
differences of the objective, and pure-Python brute force on tiny inputs.
"""
import math

import numpy as np
import pytest

from oracle import exact_tsne as ex
from paper_1611_02568_amd import datagen


def _distinct_voxels(n, r, seed, centre=False):
    rng = np.random.default_rng(seed)
    flat = rng.choice(r ** 3, size=n, replace=False)
    v = np.stack([flat % r, (flat // r) % r, flat // (r * r)], 1).astype(np.float64)
    if centre:
        return v + 0.5
    return v + rng.uniform(0.0, 1.0, (n, 3)) * (1 - 1e-9)


def _dense_P(orc, n, D, u, seed):
    X, _ = datagen.small_mixture(n=n, D=D, K=3, seed=seed)
    idx, d2 = orc.knn(X, n - 1)
    Pc, _, _ = orc.perplexity(d2, u)
    return orc.symmetrize(idx, Pc, n)


def test_two_points_closed_form(orc):
    X = np.array([[0.0, 0.0], [3.0, 4.0]])
    idx, d2 = orc.knn(X, 1)
    Pc, _, _ = orc.perplexity(d2, 1.0)
    P = orc.symmetrize(idx, Pc, 2)
    z = np.array([[10.3, 200.7, 5.5], [400.2, 31.9, 250.25]])
    s = np.array([0.01, 0.02, 0.015])
    g = orc.gradient3(z, 512, s, P, theta=0.5)
    w = 1.0 / (1.0 + np.sum(((z[0] - z[1]) * s) ** 2))
    assert abs(g["Z"] - 2 * w) <= 1e-15 * 2 * w
    assert np.max(np.abs(g["B"])) <= 1e-15 * np.max(np.abs(g["A"]))
    assert abs(orc.kl3(z, s, P)) <= 1e-15


@pytest.mark.parametrize("n", [3, 10, 50, 200])
def test_theta0_equals_exact_repulsion(orc, n):
    r = 64
    z = _distinct_voxels(n, r, seed=300 + n)
    s = np.array([0.013, 0.021, 0.017])
    R, Zi, vis = orc.Tree3(z, r).repulsion(s * s, 0.0)
    Ry, Z = ex.repulsion(z * s)
    np.testing.assert_allclose(R * s, Ry, rtol=1e-12, atol=1e-14 * np.abs(Ry).max())
    assert abs(Zi.sum() - Z) <= 1e-12 * Z
    assert np.all(np.abs(R.sum(0)) <= 1e-10 * np.abs(R).sum(0))


def test_gradient_matches_kl_finite_differences(orc):
    n, r = 10, 1024
    P = _dense_P(orc, n, 5, 4.0, seed=37)
    z = _distinct_voxels(n, r, seed=38)
    s = np.array([5.0 / r, 3.0 / r, 4.0 / r])
    g = orc.gradient3(z, r, s, P, theta=0.0)
    grad_y = 4.0 * g["B"] * s
    Pd = ex.dense_from_csr(P, n)
    h = 1e-6
    fd = np.zeros_like(z)
    fd_np = np.zeros_like(z)
    for i in range(n):
        for d in range(3):
            zp = z.copy(); zp[i, d] += h / s[d]
            zm = z.copy(); zm[i, d] -= h / s[d]
            fd[i, d] = (orc.kl3(zp, s, P) - orc.kl3(zm, s, P)) / (2 * h)
            fd_np[i, d] = (ex.kl(zp * s, Pd) - ex.kl(zm * s, Pd)) / (2 * h)
    scale = np.abs(grad_y).max()
    assert np.max(np.abs(fd - grad_y)) <= 1e-6 * scale
    assert np.max(np.abs(fd_np - grad_y)) <= 1e-6 * scale
    np.testing.assert_allclose(grad_y, ex.gradient(z * s, Pd), rtol=1e-10, atol=1e-13 * scale)


def _interleave3(v, L):
    key = np.zeros(v.shape[0], np.uint64)
    for b in range(L):
        for d in range(3):
            key |= ((v[:, d].astype(np.uint64) >> np.uint64(b)) & np.uint64(1)) \
                << np.uint64(3 * b + d)
    return key


@pytest.mark.parametrize("gen", ["uniform", "clustered"])
def test_octree_against_bruteforce(orc, gen):
    r, n, L = 32, 3000, 5
    z = (datagen.uniform_pixels(n, r, seed=41, dim=3) if gen == "uniform"
         else datagen.clustered_pixels(n, r, seed=42, spread=0.02, dim=3))
    v = np.clip(np.floor(z), 0, r - 1).astype(np.int64)
    key = _interleave3(v, L)
    tree = orc.Tree3(z, r)
    assert tree.L == L
    prev = None
    for l in range(L + 1):
        pre, cnt, sm = tree.level(l)
        w = 2 ** (L - l)
        cell = key >> np.uint64(3 * (L - l))
        upre, inv = np.unique(cell, return_inverse=True)
        assert np.array_equal(pre.astype(np.uint64), upre)
        assert np.array_equal(cnt, np.bincount(inv))
        ref = np.array([[math.fsum(z[inv == c, d]) for d in range(3)] for c in range(upre.size)])
        np.testing.assert_allclose(sm, ref, rtol=8e-16, atol=0)
        # each point lies in its cell [c w, (c + 1) w) on every axis
        for d in range(3):
            cd = np.zeros(n, np.int64)
            for b in range(l):
                cd |= ((cell.astype(np.int64) >> (3 * b + d)) & 1) << b
            assert np.all((cd * w <= z[:, d]) & (z[:, d] < (cd + 1) * w))
        if prev is not None:
            ppre, pcnt = prev
            par = np.searchsorted(ppre, pre >> 3)
            assert np.array_equal(np.bincount(par, weights=cnt, minlength=ppre.size), pcnt)
        prev = (pre, cnt)


def _bh3_python(z, r, beta, theta):
    L = int(round(math.log2(r)))
    n = len(z)
    v = np.clip(np.floor(z), 0, r - 1).astype(int)
    R = np.zeros((n, 3)); Zi = np.zeros(n); vis = np.zeros(n, int)

    def visit(i, level, o):
        w = 2 ** (L - level)
        mem = [j for j in range(n) if all(o[d] <= v[j, d] < o[d] + w for d in range(3))]
        if not mem:
            return
        vis[i] += 1
        if level == L:
            use = [j for j in mem if j != i]
            if not use:
                return
        else:
            use = mem
        m = len(use)
        c = np.array([math.fsum(z[use, d]) for d in range(3)]) / m
        dz = z[i] - c
        d2 = float(np.sum(beta * dz * dz))
        if level < L and not (w * w * beta.sum() < theta * theta * d2):
            h = w // 2
            for q in range(8):                   # child 4 zbit + 2 ybit + xbit
                visit(i, level + 1, (o[0] + (q & 1) * h, o[1] + ((q >> 1) & 1) * h,
                                     o[2] + (q >> 2) * h))
            return
        q = 1.0 / (1.0 + d2)
        Zi[i] += m * q
        R[i] += m * q * q * dz

    for i in range(n):
        visit(i, 0, (0, 0, 0))
    return R, Zi, vis


@pytest.mark.parametrize("theta", [0.0, 0.3, 0.5, 0.9])
def test_bh_traversal_bruteforce(orc, theta):
    r, n = 16, 80
    z = datagen.clustered_pixels(n, r, seed=51, n_clusters=3, spread=0.08, dim=3)
    beta = np.array([0.37, 0.22, 0.29])
    R, Zi, vis = orc.Tree3(z, r).repulsion(beta, theta)
    Rp, Zp, vp = _bh3_python(z, r, beta, theta)
    assert np.array_equal(vis, vp)
    np.testing.assert_allclose(Zi, Zp, rtol=1e-13)
    np.testing.assert_allclose(R, Rp, rtol=1e-11, atol=1e-13 * np.abs(Rp).max())


def test_bh_error_small_and_monotone(orc):
    """theta > 0 approximates theta = 0 (sanity only: the error level is not
    fixed by the paper -- parity unpinned)."""
    r, n = 256, 2000
    z = datagen.clustered_pixels(n, r, seed=61, n_clusters=6, spread=0.05, dim=3)
    beta = np.array([0.02, 0.02, 0.02]) ** 2
    tree = orc.Tree3(z, r)
    R0, _, v0 = tree.repulsion(beta, 0.0)
    errs = []
    for th in (0.2, 0.5, 0.8):
        R, _, v = tree.repulsion(beta, th)
        errs.append(np.linalg.norm(R - R0) / np.linalg.norm(R0))
        assert v.mean() < v0.mean()
    assert errs[0] < errs[1] < errs[2] < 0.05


def test_scale_compensation(orc):
    n, r = 40, 512
    P = _dense_P(orc, n, 6, 8.0, seed=39)
    z = _distinct_voxels(n, r, seed=40)
    s = np.array([0.0071, 0.0123, 0.0097])
    g = orc.gradient3(z, r, s, P, theta=0.0, alpha=3.0)
    ref = ex.gradient(z * s, ex.dense_from_csr(P, n), alpha=3.0) / 4.0
    np.testing.assert_allclose(g["B"] * s, ref, rtol=1e-10, atol=1e-12 * np.abs(ref).max())


def test_voxel_frame_optimiser_tracks_exact_tsne(orc):
    n, r, T = 30, 1024, 60
    X, _ = datagen.small_mixture(n=n, D=8, K=3, seed=43)
    P = orc.build_P(X, 5.0, k=15)
    Pd = ex.dense_from_csr(P, n)
    y0 = datagen.initial_embedding(n, seed=44, dim=3)
    st = orc.State3(y0, r)
    p = orc.params(r, theta=0.0, exag_iters=8, mom_switch=8)
    orc.iterate3(st, p, P, T)
    z0, g0, _ = orc.normalize3(y0, r)
    Ye = ex.run(z0 * (g0 / r), Pd, T, exag_iters=8, mom_switch=8)
    Yo = st.y() - st.y().mean(0)
    Ye = Ye - Ye.mean(0)
    assert len({tuple(p) for p in np.floor(st.z).astype(int)}) == n
    assert np.max(np.abs(Yo - Ye)) <= 1e-9 * np.abs(Ye).max()


def test_normalisation_range(orc):
    X, _ = datagen.small_mixture(n=500, D=10, seed=45)
    P = orc.build_P(X, 10.0)
    st = orc.State3(datagen.initial_embedding(500, seed=46, dim=3), 256)
    p = orc.params(256)
    for _ in range(4):
        orc.iterate3(st, p, P, 3)
        assert np.all(st.z.min(0) == 0.0)
        assert np.all(st.z < 256)
        assert np.all(np.floor(st.z.max(0)) == 255)


def test_kl_against_numpy(orc):
    X, _ = datagen.small_mixture(n=120, D=8, seed=47)
    P = orc.build_P(X, 6.0)
    z = datagen.uniform_pixels(120, 128, seed=48, dim=3)
    s = np.array([0.03, 0.05, 0.04])
    ref = ex.kl(z * s, ex.dense_from_csr(P, 120))
    assert abs(orc.kl3(z, s, P) - ref) <= 1e-12 * abs(ref)
