"""PixelSNE CPU oracle -- TEST INFRASTRUCTURE ONLY.

Plain, slow FP64 reference of what PixelSNE (arXiv:1611.02568) computes,
used by the tests, the smoke check and the benchmark's CPU baseline to check
the GPU library.  The product path never imports this package.  The
arithmetic lives in ``pixelsne_oracle.c`` (C99 + OpenMP, built into
``liboracle.so`` by ``oracle/build.py``); ``exact_tsne.py`` is an
independent NumPy O(n^2) t-SNE used to pin it, and ``mlp.py`` is the FP64
reference of the learned placement network.

Functions follow the paper's sections:
  knn / perplexity / symmetrize ......... Section 3.2-3.3 (sparse P)
  morton / sorted_order / Tree .......... Eq. 1-2, Section 4.1 (P-Quadtree)
  repulsion ............................. Eq. 5, 11, 12; Section 4.1 leaf stop
  attraction ............................ Eq. 5, 12
  normalize ............................. Section 4.2 (screen-driven scaling)
  gradient / iterate .................... Eq. 5 in the pixel frame, Eq. 13
  kl .................................... Eq. 4 with exact Z
  neighborhood_precision ................ Eq. 14
  Tree3 / gradient3 / iterate3 / kl3 .... the 3-D embedding (Section 1): voxel
                                          octree, three-axis scaling
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u64p = np.ctypeslib.ndpointer(dtype=np.uint64, flags="C_CONTIGUOUS")


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    vp = C.c_void_p
    lib.orc_version.restype = C.c_int
    lib.orc_num_threads.restype = C.c_int
    lib.orc_set_num_threads.argtypes = [C.c_int]
    lib.orc_knn.argtypes = [_dp, C.c_int64, C.c_int32, C.c_int32, vp, C.c_int64, _i32p, _dp]
    lib.orc_knn_approx.argtypes = [_dp, C.c_int64, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                   C.c_int32, C.c_uint64, _i32p, _dp]
    lib.orc_perplexity.argtypes = [_dp, C.c_int64, C.c_int32, C.c_double, C.c_double, C.c_int32,
                                   _dp, _dp, _i32p]
    lib.orc_symmetrize.restype = C.c_int64
    lib.orc_symmetrize.argtypes = [_i32p, _dp, C.c_int64, C.c_int32, vp, vp, vp, C.c_int64]
    lib.orc_morton.argtypes = [_dp, C.c_int64, C.c_int32, _u32p]
    lib.orc_tree_build.restype = vp
    lib.orc_tree_build.argtypes = [_dp, C.c_int64, C.c_int32]
    lib.orc_dtree_build.restype = vp
    lib.orc_dtree_build.argtypes = [_dp, C.c_int64, C.c_int32]
    lib.orc_tree_level64.argtypes = [vp, C.c_int32, _u64p, _i64p, _dp]
    lib.orc_tree_free.argtypes = [vp]
    lib.orc_tree_depth.restype = C.c_int32
    lib.orc_tree_depth.argtypes = [vp]
    lib.orc_tree_num_nodes.restype = C.c_int64
    lib.orc_tree_num_nodes.argtypes = [vp]
    lib.orc_tree_level_sizes.argtypes = [vp, _i64p]
    lib.orc_tree_level.argtypes = [vp, C.c_int32, _u32p, _i64p, _dp]
    lib.orc_sorted_order.argtypes = [_dp, C.c_int64, C.c_int32, _u32p, _i64p]
    lib.orc_repulsion.argtypes = [vp, _dp, _dp, C.c_double, C.c_int32, _dp, _dp, _i64p]
    lib.orc_repulsion_rows.argtypes = [vp, _dp, _dp, C.c_double, C.c_int32, C.c_int32, vp,
                                       C.c_int64, _dp, _dp, _i64p]
    lib.orc_attraction_rows.argtypes = [_dp, C.c_int64, _dp, _i64p, _i32p, _dp, vp, C.c_int64,
                                        _dp]
    lib.orc_sum.restype = C.c_double
    lib.orc_sum.argtypes = [_dp, C.c_int64]
    lib.orc_attraction.argtypes = [_dp, C.c_int64, _dp, _i64p, _i32p, _dp, _dp]
    lib.orc_normalize.argtypes = [_dp, C.c_int64, C.c_int32, C.c_double, _dp, _dp, _dp]
    lib.orc_gradient.argtypes = [_dp, C.c_int64, C.c_int32, _dp, C.c_double, C.c_int32,
                                 C.c_int32, C.c_int32, C.c_double, _i64p, _i32p, _dp, _dp, _dp,
                                 _dp, _dp, _i64p, _dp]
    lib.orc_iterate.argtypes = [C.c_void_p, C.c_int64, _i64p, _i32p, _dp, _dp, _dp, _dp, _dp,
                                C.c_int32, C.c_int32, vp]
    lib.orc_kl.restype = C.c_double
    lib.orc_kl.argtypes = [_dp, C.c_int64, _dp, _i64p, _i32p, _dp]
    lib.orc_tree3_build.restype = vp
    lib.orc_tree3_build.argtypes = [_dp, C.c_int64, C.c_int32]
    lib.orc_tree3_free.argtypes = [vp]
    lib.orc_tree3_level_sizes.argtypes = [vp, _i64p]
    lib.orc_tree3_level.argtypes = [vp, C.c_int32, _u32p, _i64p, _dp]
    lib.orc_repulsion3.argtypes = [vp, _dp, _dp, C.c_double, _dp, _dp, _i64p]
    lib.orc_gradient3.argtypes = [_dp, C.c_int64, C.c_int32, _dp, C.c_double, C.c_double, _i64p,
                                  _i32p, _dp, _dp, _dp, _dp, _dp, _i64p, _dp]
    lib.orc_iterate3.argtypes = [C.c_void_p, C.c_int64, _i64p, _i32p, _dp, _dp, _dp, _dp, _dp,
                                 C.c_int32, C.c_int32]
    lib.orc_normalize3.argtypes = [_dp, C.c_int64, C.c_int32, C.c_double, _dp, _dp, _dp]
    lib.orc_kl3.restype = C.c_double
    lib.orc_kl3.argtypes = [_dp, C.c_int64, _dp, _i64p, _i32p, _dp]
    _lib = lib
    return lib


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def num_threads() -> int:
    return _load().orc_num_threads()


def set_num_threads(t: int) -> None:
    _load().orc_set_num_threads(int(t))


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


# --------------------------------------------------------------------------
# Section 3.2-3.3: sparse P
# --------------------------------------------------------------------------
def knn(X, k: int, rows=None):
    """k nearest neighbours (squared Euclidean, FP64, self excluded, ties to
    the smaller index).  Returns (idx int32 [m,k], d2 float64 [m,k])."""
    X = _f64(X)
    n, D = X.shape
    if rows is None:
        m, rp = n, None
        rows_arr = None
    else:
        rows_arr = np.ascontiguousarray(rows, dtype=np.int64)
        m = rows_arr.size
        rp = rows_arr.ctypes.data
    idx = np.empty((m, k), np.int32)
    d2 = np.empty((m, k), np.float64)
    _check(_load().orc_knn(X, n, D, k, rp, m, idx, d2), "knn")
    return idx, d2


def knn_approx(X, k: int, n_trees: int = 4, leaf_size: int | None = None, explore: int = 1,
               seed: int = 0):
    """Approximate kNN of Section 4.3 (random-projection trees, then rounds of
    neighbours of neighbours); leaf_size (>= 2k + 2) defaults to 2k + 2.
    Returns (idx int32 [n,k], d2 float64 [n,k]) ascending by (d2, index)."""
    X = _f64(X)
    n, D = X.shape
    leaf = 2 * k + 2 if leaf_size is None else int(leaf_size)
    idx = np.empty((n, k), np.int32)
    d2 = np.empty((n, k), np.float64)
    _check(_load().orc_knn_approx(X, n, D, k, int(n_trees), leaf, int(explore),
                                  int(seed) & (2 ** 64 - 1), idx, d2), "knn_approx")
    return idx, d2


def perplexity(d2, u: float, tol: float = 1e-5, max_iter: int = 200):
    """Row-wise Gaussian calibration to perplexity u.  Returns
    (P_cond [m,k], beta [m], evaluations [m])."""
    d2 = _f64(d2)
    m, k = d2.shape
    P = np.empty_like(d2)
    beta = np.empty(m, np.float64)
    it = np.empty(m, np.int32)
    _check(_load().orc_perplexity(d2, m, k, float(u), float(tol), int(max_iter), P, beta, it),
           "perplexity")
    return P, beta, it


def symmetrize(idx, Pc, n: int):
    """p_ij = (p_{j|i} + p_{i|j}) / 2n on the union pattern -> CSR
    (row_ptr int64 [n+1], col int32 [nnz], val float64 [nnz])."""
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    Pc = _f64(Pc)
    k = idx.shape[1]
    lib = _load()
    nnz = lib.orc_symmetrize(idx, Pc, n, k, None, None, None, 0)
    if nnz < 0:
        raise RuntimeError(f"oracle symmetrize failed ({nnz})")
    rp = np.empty(n + 1, np.int64)
    col = np.empty(nnz, np.int32)
    val = np.empty(nnz, np.float64)
    got = lib.orc_symmetrize(idx, Pc, n, k, rp.ctypes.data, col.ctypes.data, val.ctypes.data, nnz)
    if got != nnz:
        raise RuntimeError("oracle symmetrize size mismatch")
    return rp, col, val


def build_P(X, u: float, k: int | None = None):
    """kNN -> perplexity -> symmetric CSR P (sums to 1)."""
    n = X.shape[0]
    if k is None:
        k = int(3 * u)
    idx, d2 = knn(X, k)
    Pc, _, _ = perplexity(d2, u)
    return symmetrize(idx, Pc, n)


# --------------------------------------------------------------------------
# Eq. 1-2 and Section 4.1: pixels, Morton order, P-Quadtree
# --------------------------------------------------------------------------
def morton(z, r: int):
    z = _f64(z)
    key = np.empty(z.shape[0], np.uint32)
    _check(_load().orc_morton(z, z.shape[0], r, key), "morton")
    return key


def sorted_order(z, r: int):
    """(keys ascending, permutation) of the stable sort by Morton key."""
    z = _f64(z)
    n = z.shape[0]
    key = np.empty(n, np.uint32)
    perm = np.empty(n, np.int64)
    _check(_load().orc_sorted_order(z, n, r, key, perm), "sorted_order")
    return key, perm


class Tree:
    """P-Quadtree (kind 0) of pixel positions z (n x 2) on an r x r screen, or
    the D-Quadtree of Barnes-Hut-SNE (kind 1) over the same frame: split until
    each leaf holds one point (or one cell of the 2^32 grid), levels 0..32."""

    def __init__(self, z, r: int, kind: int = 0):
        self._lib = _load()
        self.z = _f64(z)
        self.r = r
        self.kind = kind
        build = self._lib.orc_dtree_build if kind == 1 else self._lib.orc_tree_build
        self.h = build(self.z, self.z.shape[0], r)
        if not self.h:
            raise RuntimeError("oracle tree build failed")
        self.L = self._lib.orc_tree_depth(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._lib.orc_tree_free(h)
            self.h = None

    def level_sizes(self):
        s = np.empty(self.L + 1, np.int64)
        self._lib.orc_tree_level_sizes(self.h, s)
        return s

    def level(self, l: int):
        """(prefix, count int64, sums float64 [m,2]) ascending by prefix; the
        prefix is uint32 (P-Quadtree) or uint64 on the 2^32 grid (D-Quadtree)."""
        m = int(self.level_sizes()[l])
        cnt = np.empty(m, np.int64)
        sm = np.empty((m, 2), np.float64)
        if self.kind == 1:
            pre = np.empty(m, np.uint64)
            _check(self._lib.orc_tree_level64(self.h, l, pre, cnt, sm), "tree level")
        else:
            pre = np.empty(m, np.uint32)
            _check(self._lib.orc_tree_level(self.h, l, pre, cnt, sm), "tree level")
        return pre, cnt, sm

    def repulsion(self, beta, theta: float, com_mode: int = 0, rows=None, predicate: int = 0):
        """(R, Z_i, visits) for every point, or for the points in rows.
        predicate 0: the opening test in FP64; 1: in FP32 (operands rounded to
        FP32, each operation rounded in the written order)."""
        if rows is None:
            m, rp = self.z.shape[0], None
        else:
            rows = np.ascontiguousarray(rows, dtype=np.int64)
            m, rp = rows.size, rows.ctypes.data
        R = np.empty((m, 2), np.float64)
        Zi = np.empty(m, np.float64)
        vis = np.empty(m, np.int64)
        _check(self._lib.orc_repulsion_rows(self.h, self.z, _f64(beta), float(theta),
                                            int(com_mode), int(predicate), rp, m, R, Zi, vis),
               "repulsion")
        return R, Zi, vis


def csum(v) -> float:
    v = _f64(v).ravel()
    return _load().orc_sum(v, v.size)


# --------------------------------------------------------------------------
# Eq. 5 / 12: attraction, gradient; Section 4.2: scaling; Eq. 4: KL
# --------------------------------------------------------------------------
def _csr(P):
    rp, col, val = P
    return (np.ascontiguousarray(rp, np.int64), np.ascontiguousarray(col, np.int32), _f64(val))


def attraction(z, beta, P, rows=None):
    """A_i for every point, or for the points in rows."""
    z = _f64(z)
    rp, col, val = _csr(P)
    if rows is None:
        m, rptr = z.shape[0], None
    else:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        m, rptr = rows.size, rows.ctypes.data
    A = np.empty((m, 2), np.float64)
    _check(_load().orc_attraction_rows(z, z.shape[0], _f64(beta), rp, col, val, rptr, m, A),
           "attraction")
    return A


def normalize(zh, r: int, eps: float = 1e-6):
    """Screen-driven scaling: returns (z, gamma[2], zmin[2])."""
    zh = _f64(zh)
    z = np.empty_like(zh)
    g = np.empty(2)
    m = np.empty(2)
    _check(_load().orc_normalize(zh, zh.shape[0], r, float(eps), z, g, m), "normalize")
    return z, g, m


def gradient(z, r: int, s, P, theta: float = 0.5, com_mode: int = 0, alpha: float = 1.0,
             predicate: int = 0, tree: int = 0):
    """Pixel-frame bracket B = alpha*A - R/Z and its parts (dict); predicate
    selects the FP64 (0) or FP32 (1) opening test, forces FP64 either way;
    tree selects the P-Quadtree (0) or the D-Quadtree (1)."""
    z = _f64(z)
    n = z.shape[0]
    rp, col, val = _csr(P)
    B = np.empty_like(z)
    A = np.empty_like(z)
    R = np.empty_like(z)
    Zi = np.empty(n)
    vis = np.empty(n, np.int64)
    Z = np.empty(1)
    _check(_load().orc_gradient(z, n, r, _f64(s), float(theta), int(com_mode), int(predicate),
                                int(tree), float(alpha), rp, col, val, B, A, R, Zi, vis, Z),
           "gradient")
    return {"B": B, "A": A, "R": R, "Zi": Zi, "visits": vis, "Z": float(Z[0])}


class Params(C.Structure):
    _fields_ = [("r", C.c_int32), ("theta", C.c_double), ("com_mode", C.c_int32),
                ("eta", C.c_double), ("mom0", C.c_double), ("mom1", C.c_double),
                ("mom_switch", C.c_int32), ("exaggeration", C.c_double),
                ("exag_iters", C.c_int32), ("min_gain", C.c_double), ("eps", C.c_double),
                ("predicate", C.c_int32), ("tree", C.c_int32)]


def params(r: int, theta: float = 0.5, com_mode: int = 0, eta: float = 200.0, mom0: float = 0.5,
           mom1: float = 0.8, mom_switch: int = 250, exaggeration: float = 12.0,
           exag_iters: int = 250, min_gain: float = 0.01, eps: float = 1e-6,
           predicate: int = 0, tree: int = 0) -> Params:
    return Params(r, theta, com_mode, eta, mom0, mom1, mom_switch, exaggeration, exag_iters,
                  min_gain, eps, predicate, tree)


class State:
    """Optimiser state in the pixel frame: z, velocity u, gains g, scale s, t."""

    def __init__(self, y0, r: int, eps: float = 1e-6):
        y0 = _f64(y0)
        self.z, gamma, _ = normalize(y0, r, eps)
        self.s = gamma / float(r)              # y units per pixel (initial frame: y itself)
        self.u = np.zeros_like(self.z)
        self.g = np.ones_like(self.z)
        self.t = 0

    def y(self):
        return self.z * self.s[None, :]


def iterate(state: State, p: Params, P, n_iter: int, Z_hist: bool = False):
    rp, col, val = _csr(P)
    n = state.z.shape[0]
    zh = np.empty(n_iter) if Z_hist else None
    _check(_load().orc_iterate(C.byref(p), n, rp, col, val, state.z, state.u, state.g, state.s,
                               state.t, n_iter, zh.ctypes.data if Z_hist else None), "iterate")
    state.t += n_iter
    return zh


def kl(z, s, P) -> float:
    """KL(P || Q) with exact Z over all pairs (O(n^2))."""
    z = _f64(z)
    rp, col, val = _csr(P)
    return float(_load().orc_kl(z, z.shape[0], _f64(s), rp, col, val))


# --------------------------------------------------------------------------
# Eq. 14: neighbourhood precision
# --------------------------------------------------------------------------
def neighborhood_precision(hi, lo, ks):
    """(1 / kN) sum_i |N_D^(k)(i) intersect N_d^(k)(i)| for each k in ks, where
    N_D^(k)(i) = first k entries of hi[i] (high-dimensional neighbours, nearest
    first) and N_d^(k)(i) = first k of lo[i] (embedding neighbours)."""
    hi = np.asarray(hi)
    lo = np.asarray(lo)
    n = hi.shape[0]
    out = []
    for k in ks:
        common = 0
        for i in range(n):
            common += len(set(hi[i, :k].tolist()) & set(lo[i, :k].tolist()))
        out.append(common / (k * n))
    return out


# --------------------------------------------------------------------------
# The 3-D embedding (Section 1): voxel octree of fixed depth log2 r, the
# steps of the 2-D functions above run over three axes.
# --------------------------------------------------------------------------
class Tree3:
    """Voxel octree of z (n x 3) in an r x r x r cube (r a power of two, at
    most 1024): levels 0..log2 r, unit-voxel leaves, octant prefix = Morton
    key with x, y, z in bits 3b, 3b+1, 3b+2."""

    def __init__(self, z, r: int):
        self._lib = _load()
        self.z = _f64(z)
        self.r = r
        self.L = int(r).bit_length() - 1
        self.h = self._lib.orc_tree3_build(self.z, self.z.shape[0], r)
        if not self.h:
            raise RuntimeError("oracle octree build failed")

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self._lib.orc_tree3_free(h)
            self.h = None

    def level_sizes(self):
        s = np.empty(self.L + 1, np.int64)
        self._lib.orc_tree3_level_sizes(self.h, s)
        return s

    def level(self, l: int):
        """(prefix uint32, count int64, sums float64 [m,3]) ascending by prefix."""
        m = int(self.level_sizes()[l])
        pre = np.empty(m, np.uint32)
        cnt = np.empty(m, np.int64)
        sm = np.empty((m, 3), np.float64)
        _check(self._lib.orc_tree3_level(self.h, l, pre, cnt, sm), "octree level")
        return pre, cnt, sm

    def repulsion(self, beta, theta: float):
        """(R [n,3], Z_i, visits) with the FP64 opening test and centres of mass."""
        n = self.z.shape[0]
        R = np.empty((n, 3), np.float64)
        Zi = np.empty(n, np.float64)
        vis = np.empty(n, np.int64)
        _check(self._lib.orc_repulsion3(self.h, self.z, _f64(beta), float(theta), R, Zi, vis),
               "repulsion3")
        return R, Zi, vis


def gradient3(z, r: int, s, P, theta: float = 0.5, alpha: float = 1.0):
    """Voxel-frame bracket B = alpha*A - R/Z of a 3-D embedding and its parts."""
    z = _f64(z)
    n = z.shape[0]
    rp, col, val = _csr(P)
    B = np.empty_like(z)
    A = np.empty_like(z)
    R = np.empty_like(z)
    Zi = np.empty(n)
    vis = np.empty(n, np.int64)
    Z = np.empty(1)
    _check(_load().orc_gradient3(z, n, r, _f64(s), float(theta), float(alpha), rp, col, val, B, A,
                                 R, Zi, vis, Z), "gradient3")
    return {"B": B, "A": A, "R": R, "Zi": Zi, "visits": vis, "Z": float(Z[0])}


def normalize3(zh, r: int, eps: float = 1e-6):
    """Three-axis screen-driven scaling: (z, gamma[3], zmin[3])."""
    zh = _f64(zh)
    z = np.empty_like(zh)
    g = np.empty(3)
    m = np.empty(3)
    _check(_load().orc_normalize3(zh, zh.shape[0], r, float(eps), z, g, m), "normalize3")
    return z, g, m


class State3(State):
    """Optimiser state of a 3-D embedding in the voxel frame."""

    def __init__(self, y0, r: int, eps: float = 1e-6):
        y0 = _f64(y0)
        self.z, gamma, _ = normalize3(y0, r, eps)
        self.s = gamma / float(r)
        self.u = np.zeros_like(self.z)
        self.g = np.ones_like(self.z)
        self.t = 0


def iterate3(state: State3, p: Params, P, n_iter: int):
    """n_iter iterations of the 3-D loop (centres of mass, FP64 opening test;
    p.com_mode, p.predicate and p.tree are not read)."""
    rp, col, val = _csr(P)
    _check(_load().orc_iterate3(C.byref(p), state.z.shape[0], rp, col, val, state.z, state.u,
                                state.g, state.s, state.t, n_iter), "iterate3")
    state.t += n_iter


def kl3(z, s, P) -> float:
    """KL(P || Q) of a 3-D embedding with exact Z over all pairs (O(n^2))."""
    z = _f64(z)
    rp, col, val = _csr(P)
    return float(_load().orc_kl3(z, z.shape[0], _f64(s), rp, col, val))
