"""ctypes binding of libpixelsne.so (the gfx950 PixelSNE library).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory (tensors) and the stream.  Loading
fails loudly when the library has not been built; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpixelsne.so")

PSNE_OK, PSNE_E_INVAL, PSNE_E_NOMEM, PSNE_E_DEVICE = 0, -1, -2, -3
PSNE_E_NUMERIC, PSNE_E_STATE, PSNE_E_UNSUPPORTED = -4, -5, -6
FP32, FP64 = 0, 1
FORK_SNAP, FORK_CELLS, FORK_AUTO = 0, 1, 2
COM_MASS, COM_CELL_CENTER = 0, 1
X_F32, X_F64, X_U8 = 0, 1, 2
TREE_PIXEL, TREE_DATA = 0, 1
FRAME_PIXEL, FRAME_SCREEN, FRAME_Y = 0, 1, 2

_STATUS = {PSNE_E_INVAL: "invalid argument", PSNE_E_NOMEM: "out of device memory",
           PSNE_E_DEVICE: "device error", PSNE_E_NUMERIC: "non-finite values",
           PSNE_E_STATE: "context unusable", PSNE_E_UNSUPPORTED: "unsupported"}


class PixelSNEError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_STATUS.get(code, code)}: {msg}")
        self.code = code


class Params(C.Structure):
    _fields_ = [
        ("struct_size", C.c_uint32), ("k", C.c_int32), ("theta", C.c_double),
        ("exag_iters", C.c_int32), ("exaggeration", C.c_double), ("eta", C.c_double),
        ("mom0", C.c_double), ("mom1", C.c_double), ("mom_switch", C.c_int32),
        ("min_gain", C.c_double), ("eps", C.c_double), ("init_sigma", C.c_double),
        ("seed", C.c_uint64), ("precision", C.c_int32), ("com_mode", C.c_int32),
        ("x_dtype", C.c_int32), ("Y_init", C.c_void_p), ("stream", C.c_void_p),
        ("reorder_every", C.c_int32),
        ("data_order", C.c_int32),
        ("graphs", C.c_int32),
        ("reorder_growth", C.c_double),
        ("opening_fp64", C.c_int32),
        ("tree", C.c_int32),
        ("knn_trees", C.c_int32),
        ("knn_leaf", C.c_int32),
        ("knn_explore", C.c_int32),
        ("attract_blocks_per_cu", C.c_int32),
        ("attract_help_blocks_per_cu", C.c_int32),
        ("attract_fork", C.c_int32),
    ]


class Stats(C.Structure):
    _fields_ = [
        ("n", C.c_int64), ("nnz", C.c_int64), ("n_nodes", C.c_int64),
        ("r", C.c_int32), ("L", C.c_int32), ("k", C.c_int32),
        ("precision", C.c_int32), ("com_mode", C.c_int32), ("iteration", C.c_int32),
        ("s", C.c_double * 2), ("Z", C.c_double), ("level_size", C.c_int64 * 17),
        ("renumberings", C.c_int32), ("fork_cells", C.c_int32),
        ("fork_ms", C.c_double * 2),
    ]


class PassTimes(C.Structure):
    _fields_ = [("snap_ms", C.c_double), ("sort_ms", C.c_double), ("tree_ms", C.c_double),
                ("traverse_ms", C.c_double), ("zsum_ms", C.c_double),
                ("attract_ms", C.c_double), ("finalize_ms", C.c_double),
                ("reorder_ms", C.c_double), ("iterations", C.c_int32)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class RefineResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("reached", C.c_int32), ("fallback", C.c_int32),
                ("kl_start", C.c_double), ("kl", C.c_double), ("iter_ms", C.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# exported symbol -> (restype, argtypes)
_vp, _i64, _i32, _d, _u64 = C.c_void_p, C.c_int64, C.c_int32, C.c_double, C.c_uint64
SIGNATURES = {
    "pixelsne_default_params": (None, [C.POINTER(Params)]),
    "pixelsne_init": (_vp, [_vp, _i64, _i32, _d, _i32, _i32]),
    "pixelsne_init_ex": (_vp, [_vp, _i64, _i32, _d, _i32, _i32, C.POINTER(Params)]),
    "pixelsne_init_with_P": (_vp, [_i64, _i64, _vp, _vp, _vp, _i32, _i32, C.POINTER(Params)]),
    "pixelsne_step": (C.c_int, [_vp, _i32]),
    "pixelsne_step_async": (C.c_int, [_vp, _i32]),
    "pixelsne_step_profiled": (C.c_int, [_vp, _i32, C.POINTER(PassTimes)]),
    "pixelsne_get_Y": (C.c_int, [_vp, _vp, _i32]),
    "pixelsne_destroy": (None, [_vp]),
    "pixelsne_last_error": (C.c_char_p, []),
    "pixelsne_get_stats": (C.c_int, [_vp, C.POINTER(Stats)]),
    "pixelsne_set_state": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _i32]),
    "pixelsne_get_state": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double),
                                     C.POINTER(C.c_int32)]),
    "pixelsne_gradient": (C.c_int, [_vp, _d, _vp, _vp, _vp, _vp, _vp, _vp,
                                    C.POINTER(C.c_double)]),
    "pixelsne_export_tree": (C.c_int, [_vp, C.POINTER(C.c_int64), _vp, _vp, _vp, _vp, _vp]),
    "pixelsne_export_P": (C.c_int, [_vp, C.POINTER(C.c_int64), _vp, _vp, _vp]),
    "pixelsne_export_tree64": (C.c_int, [_vp, C.POINTER(C.c_int64), _vp, _vp, _vp, _vp, _vp]),
    "pixelsne_knn": (C.c_int, [_vp, _i64, _i32, _i32, _i32, _vp, _vp, _vp]),
    "pixelsne_perplexity": (C.c_int, [_vp, _i64, _i32, _d, _vp, _vp, _vp]),
    "pixelsne_knn_approx": (C.c_int, [_vp, _i64, _i32, _i32, _i32, _i32, _i32, _i32, _u64, _vp,
                                      _vp, _vp]),
    "pixelsne_mlp_create": (_vp, [_i32, _i32, _i32, _u64, _vp]),
    "pixelsne_mlp_destroy": (None, [_vp]),
    "pixelsne_mlp_num_params": (_i64, [_vp]),
    "pixelsne_mlp_set_params": (C.c_int, [_vp, _vp]),
    "pixelsne_mlp_get_params": (C.c_int, [_vp, _vp]),
    "pixelsne_mlp_set_norm": (C.c_int, [_vp, _vp, _vp]),
    "pixelsne_mlp_fit_norm": (C.c_int, [_vp, _vp, _i64]),
    "pixelsne_mlp_grad": (C.c_int, [_vp, _vp, _vp, _i64, _vp, C.POINTER(C.c_double)]),
    "pixelsne_mlp_train": (C.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, C.c_float,
                                     C.POINTER(C.c_double)]),
    "pixelsne_mlp_forward": (C.c_int, [_vp, _vp, _i64, _vp]),
    "pixelsne_mlp_place": (C.c_int, [_vp, _vp, _i64, _i32, C.POINTER(C.c_double), _vp]),
    "pixelsne_kl": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "pixelsne_refine": (C.c_int, [_vp, _d, _i32, _i32, _i32, C.POINTER(RefineResult)]),
    "pixelsne_kl_noalloc": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "pixelsne_mlp_adam_step": (C.c_int, [_vp, _vp, C.c_float]),
    "pixelsne_knn2d": (C.c_int, [_vp, _vp]),
    "pixelsne3_init_ex": (_vp, [_vp, _i64, _i32, _d, _i32, C.POINTER(Params)]),
    "pixelsne3_init_with_P": (_vp, [_i64, _i64, _vp, _vp, _vp, _i32, C.POINTER(Params)]),
    "pixelsne3_destroy": (None, [_vp]),
    "pixelsne3_step": (C.c_int, [_vp, _i32]),
    "pixelsne3_get_Y": (C.c_int, [_vp, _vp, _i32]),
    "pixelsne3_set_state": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double), _i32]),
    "pixelsne3_get_state": (C.c_int, [_vp, _vp, _vp, _vp, C.POINTER(C.c_double),
                                      C.POINTER(C.c_int32)]),
    "pixelsne3_gradient": (C.c_int, [_vp, _d, _vp, _vp, _vp, _vp, _vp, C.POINTER(C.c_double)]),
    "pixelsne3_export_tree": (C.c_int, [_vp, C.POINTER(C.c_int64), _vp, _vp, _vp, _vp, _vp]),
    "pixelsne3_kl": (C.c_int, [_vp, C.POINTER(C.c_double)]),
    "pixelsne_neighborhood_precision": (C.c_int, [_vp, _vp, _i32, C.POINTER(_i32), _i32,
                                                  C.POINTER(C.c_double)]),
}

_lib = None


def load():
    """Load libpixelsne.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_1611_02568_amd.build` (no CPU fallback exists)")
    lib = C.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _err():
    return load().pixelsne_last_error().decode(errors="replace")


def _check(rc):
    if rc != PSNE_OK:
        raise PixelSNEError(rc, _err())


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous CUDA tensor")
    return C.c_void_p(t.data_ptr())


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def default_params(**kw) -> Params:
    p = Params()
    load().pixelsne_default_params(C.byref(p))
    for k, v in kw.items():
        if not hasattr(p, k):
            raise AttributeError(k)
        setattr(p, k, v)
    return p


_X_TYPES = {torch.float32: X_F32, torch.float64: X_F64, torch.uint8: X_U8}


class Context:
    """A PixelSNE embedding on the current GPU (wraps pixelsne_ctx*)."""

    def __init__(self, handle, n, params: Params, keep=()):
        if not handle:
            raise PixelSNEError(PSNE_E_INVAL, _err())
        self._h = C.c_void_p(handle)
        self.n = n
        self.params = params
        self._keep = keep
        self.state_dtype = torch.float64 if params.precision == FP64 else torch.float32

    # --- construction -----------------------------------------------------
    @classmethod
    def from_data(cls, X: torch.Tensor, perplexity: float, screen: int, Y_init=None, **kw):
        """pixelsne_init_ex on a device matrix X [n, D] (float32/float64/uint8).
        Keyword arguments set fields of pixelsne_params (include/pixelsne.h),
        e.g. precision, theta, reorder_every, reorder_growth, graphs."""
        n, D = X.shape
        p = default_params(**kw)
        p.x_dtype = _X_TYPES[X.dtype]
        if Y_init is not None:
            Y_init = Y_init.to(device=X.device, dtype=torch.float64).contiguous()
            p.Y_init = Y_init.data_ptr()
        p.stream = _stream().value
        h = load().pixelsne_init_ex(_ptr(X.contiguous()), n, D, float(perplexity), screen, screen,
                                    C.byref(p))
        return cls(h, n, p, (Y_init,))

    @classmethod
    def from_P(cls, row_ptr, col, val, screen: int, Y_init=None, **kw):
        """pixelsne_init_with_P on a device CSR P (int64 / int32 / float64).
        Keyword arguments set fields of pixelsne_params as for from_data."""
        dev = torch.device("cuda")
        row_ptr = torch.as_tensor(row_ptr, dtype=torch.int64).to(dev).contiguous()
        col = torch.as_tensor(col, dtype=torch.int32).to(dev).contiguous()
        val = torch.as_tensor(val, dtype=torch.float64).to(dev).contiguous()
        n = row_ptr.numel() - 1
        p = default_params(**kw)
        if Y_init is not None:
            Y_init = torch.as_tensor(Y_init, dtype=torch.float64).to(dev).contiguous()
            p.Y_init = Y_init.data_ptr()
        p.stream = _stream().value
        h = load().pixelsne_init_with_P(n, val.numel(), _ptr(row_ptr), _ptr(col), _ptr(val),
                                        screen, screen, C.byref(p))
        return cls(h, n, p, (Y_init,))

    @classmethod
    def from_data_plain(cls, X: torch.Tensor, perplexity: float, screen: int):
        """pixelsne_init with its default parameters (float32 X)."""
        n, D = X.shape
        h = load().pixelsne_init(_ptr(X.contiguous()), n, D, float(perplexity), screen, screen)
        return cls(h, n, default_params())

    # --- iteration ---------------------------------------------------------
    def step(self, n_iter: int = 1):
        _check(load().pixelsne_step(self._h, int(n_iter)))

    def step_async(self, n_iter: int = 1):
        _check(load().pixelsne_step_async(self._h, int(n_iter)))

    def step_profiled(self, n_iter: int = 1) -> PassTimes:
        t = PassTimes()
        _check(load().pixelsne_step_profiled(self._h, int(n_iter), C.byref(t)))
        return t

    def get_Y(self, frame: int = FRAME_Y) -> torch.Tensor:
        dt = torch.int32 if frame == FRAME_SCREEN else torch.float64
        out = torch.empty((self.n, 2), dtype=dt, device="cuda")
        _check(load().pixelsne_get_Y(self._h, _ptr(out), int(frame)))
        return out

    def stats(self) -> Stats:
        s = Stats()
        _check(load().pixelsne_get_stats(self._h, C.byref(s)))
        return s

    def set_state(self, z, s, u=None, g=None, iteration: int = 0):
        z = torch.as_tensor(z, dtype=self.state_dtype).cuda().contiguous()
        u = None if u is None else torch.as_tensor(u, dtype=self.state_dtype).cuda().contiguous()
        g = None if g is None else torch.as_tensor(g, dtype=self.state_dtype).cuda().contiguous()
        sv = (C.c_double * 2)(float(s[0]), float(s[1]))
        _check(load().pixelsne_set_state(self._h, _ptr(z), _ptr(u), _ptr(g), sv, int(iteration)))

    def get_state(self):
        z = torch.empty((self.n, 2), dtype=self.state_dtype, device="cuda")
        u = torch.empty_like(z)
        g = torch.empty_like(z)
        sv = (C.c_double * 2)()
        it = C.c_int32()
        _check(load().pixelsne_get_state(self._h, _ptr(z), _ptr(u), _ptr(g), sv, C.byref(it)))
        return {"z": z, "u": u, "g": g, "s": (sv[0], sv[1]), "iteration": it.value}

    def gradient(self, alpha: float = 1.0):
        """Pixel-frame bracket B = alpha*A - R/Z and its parts at the current state."""
        B = torch.empty((self.n, 2), dtype=self.state_dtype, device="cuda")
        A = torch.empty_like(B)
        R = torch.empty_like(B)
        Zi = torch.empty(self.n, dtype=torch.float64, device="cuda")
        vis = torch.empty(self.n, dtype=torch.int32, device="cuda")
        used = torch.empty(self.n, dtype=torch.int32, device="cuda")
        Z = C.c_double()
        _check(load().pixelsne_gradient(self._h, float(alpha), _ptr(B), _ptr(A), _ptr(R),
                                        _ptr(Zi), _ptr(vis), _ptr(used), C.byref(Z)))
        return {"B": B, "A": A, "R": R, "Zi": Zi, "visits": vis, "used": used, "Z": Z.value}

    def export_tree(self):
        st = self.stats()
        L = st.L
        sizes = (C.c_int64 * (L + 1))()
        _check(load().pixelsne_export_tree(self._h, sizes, None, None, None, None, None))
        sizes = [sizes[i] for i in range(L + 1)]
        m = sum(sizes)
        keys = torch.empty(self.n, dtype=torch.int32, device="cuda")
        perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        pre = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        cnt = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        sm = torch.empty((max(m, 1), 2), dtype=torch.float64, device="cuda")
        s2 = (C.c_int64 * (L + 1))()
        _check(load().pixelsne_export_tree(self._h, s2, _ptr(keys), _ptr(perm), _ptr(pre),
                                           _ptr(cnt), _ptr(sm)))
        return {"level_size": sizes, "keys": keys, "perm": perm, "prefix": pre[:m],
                "count": cnt[:m], "sum": sm[:m]}

    def export_tree64(self):
        """The data-driven tree (TREE_DATA): level sizes 0..32, 64-bit keys,
        permutation, prefixes, counts and sums, as export_tree."""
        sizes = (C.c_int64 * 33)()
        _check(load().pixelsne_export_tree64(self._h, sizes, None, None, None, None, None))
        sizes = [sizes[i] for i in range(33)]
        m = sum(sizes)
        keys = torch.empty(self.n, dtype=torch.int64, device="cuda")
        perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        pre = torch.empty(max(m, 1), dtype=torch.int64, device="cuda")
        cnt = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        sm = torch.empty((max(m, 1), 2), dtype=torch.float64, device="cuda")
        s2 = (C.c_int64 * 33)()
        _check(load().pixelsne_export_tree64(self._h, s2, _ptr(keys), _ptr(perm), _ptr(pre),
                                             _ptr(cnt), _ptr(sm)))
        return {"level_size": sizes, "keys": keys, "perm": perm, "prefix": pre[:m],
                "count": cnt[:m], "sum": sm[:m]}

    def kl(self) -> float:
        """KL(P || Q) with the exact normaliser (O(n^2) on the GPU)."""
        v = C.c_double()
        _check(load().pixelsne_kl(self._h, C.byref(v)))
        return v.value

    def kl_noalloc(self) -> float:
        """pixelsne_kl_noalloc: the same KL with no device allocation."""
        v = C.c_double()
        _check(load().pixelsne_kl_noalloc(self._h, C.byref(v)))
        return v.value

    def refine(self, kl_target: float, check_every: int = 10, refine_iters: int = 100,
               max_iters: int = 1000) -> dict:
        """pixelsne_refine: iterate until the exact KL <= kl_target; the plain
        method continues past refine_iters (fallback)."""
        res = RefineResult()
        _check(load().pixelsne_refine(self._h, float(kl_target), int(check_every),
                                      int(refine_iters), int(max_iters), C.byref(res)))
        return res.as_dict()

    def knn2d(self) -> torch.Tensor:
        """The 32 nearest neighbours of each point in the embedding, int32 [n, 32]."""
        idx = torch.empty((self.n, 32), dtype=torch.int32, device="cuda")
        _check(load().pixelsne_knn2d(self._h, _ptr(idx)))
        return idx

    def neighborhood_precision(self, hi_knn: torch.Tensor, ks) -> list:
        """Eq. (14) precision of the embedding against high-dimensional neighbours
        hi_knn (device int32 [n, k_hi], nearest first) for each k in ks."""
        hi = hi_knn.to(torch.int32).contiguous()
        if hi.dim() != 2 or hi.shape[0] != self.n or not hi.is_cuda:
            raise ValueError("hi_knn must be a device tensor of shape [n, k_hi]")
        ks = [int(k) for k in ks]
        karr = (_i32 * len(ks))(*ks)
        out = (C.c_double * len(ks))()
        _check(load().pixelsne_neighborhood_precision(self._h, _ptr(hi), hi.shape[1], karr,
                                                      len(ks), out))
        return list(out)

    def export_P(self):
        nnz = C.c_int64()
        _check(load().pixelsne_export_P(self._h, C.byref(nnz), None, None, None))
        rp = torch.empty(self.n + 1, dtype=torch.int64, device="cuda")
        col = torch.empty(max(nnz.value, 1), dtype=torch.int32, device="cuda")
        val = torch.empty(max(nnz.value, 1), dtype=torch.float64, device="cuda")
        _check(load().pixelsne_export_P(self._h, C.byref(nnz), _ptr(rp), _ptr(col), _ptr(val)))
        return rp, col[:nnz.value], val[:nnz.value]

    def close(self):
        if getattr(self, "_h", None):
            load().pixelsne_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Context3:
    """A 3-D PixelSNE embedding on the current GPU (wraps pixelsne3_ctx*):
    voxel octree, three-axis scaling, FP64 throughout."""

    def __init__(self, handle, n, r, params: Params, keep=()):
        if not handle:
            raise PixelSNEError(PSNE_E_INVAL, _err())
        self._h = C.c_void_p(handle)
        self.n = n
        self.r = r
        self.L = int(r).bit_length() - 1
        self.params = params
        self._keep = keep

    @staticmethod
    def _params(Y_init, dev, kw):
        kw.setdefault("precision", FP64)
        p = default_params(**kw)
        if Y_init is not None:
            Y_init = torch.as_tensor(Y_init, dtype=torch.float64).to(dev).contiguous()
            p.Y_init = Y_init.data_ptr()
        p.stream = _stream().value
        return p, Y_init

    @classmethod
    def from_data(cls, X: torch.Tensor, perplexity: float, screen: int, Y_init=None, **kw):
        """pixelsne3_init_ex on a device matrix X [n, D]; Y_init [n, 3] (y frame)."""
        n, D = X.shape
        p, Y_init = cls._params(Y_init, X.device, kw)
        p.x_dtype = _X_TYPES[X.dtype]
        h = load().pixelsne3_init_ex(_ptr(X.contiguous()), n, D, float(perplexity), screen,
                                     C.byref(p))
        return cls(h, n, screen, p, (Y_init,))

    @classmethod
    def from_P(cls, row_ptr, col, val, screen: int, Y_init=None, **kw):
        """pixelsne3_init_with_P on a CSR P (int64 / int32 / float64)."""
        dev = torch.device("cuda")
        row_ptr = torch.as_tensor(row_ptr, dtype=torch.int64).to(dev).contiguous()
        col = torch.as_tensor(col, dtype=torch.int32).to(dev).contiguous()
        val = torch.as_tensor(val, dtype=torch.float64).to(dev).contiguous()
        n = row_ptr.numel() - 1
        p, Y_init = cls._params(Y_init, dev, kw)
        h = load().pixelsne3_init_with_P(n, val.numel(), _ptr(row_ptr), _ptr(col), _ptr(val),
                                         screen, C.byref(p))
        return cls(h, n, screen, p, (Y_init,))

    def step(self, n_iter: int = 1):
        _check(load().pixelsne3_step(self._h, int(n_iter)))

    def get_Y(self, frame: int = FRAME_Y) -> torch.Tensor:
        dt = torch.int32 if frame == FRAME_SCREEN else torch.float64
        out = torch.empty((self.n, 3), dtype=dt, device="cuda")
        _check(load().pixelsne3_get_Y(self._h, _ptr(out), int(frame)))
        return out

    def set_state(self, z, s, u=None, g=None, iteration: int = 0):
        f = lambda a: None if a is None else torch.as_tensor(a, dtype=torch.float64).cuda().contiguous()
        z, u, g = f(z), f(u), f(g)
        sv = (C.c_double * 3)(*[float(x) for x in s])
        _check(load().pixelsne3_set_state(self._h, _ptr(z), _ptr(u), _ptr(g), sv, int(iteration)))

    def get_state(self):
        z = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        u = torch.empty_like(z)
        g = torch.empty_like(z)
        sv = (C.c_double * 3)()
        it = C.c_int32()
        _check(load().pixelsne3_get_state(self._h, _ptr(z), _ptr(u), _ptr(g), sv, C.byref(it)))
        return {"z": z, "u": u, "g": g, "s": (sv[0], sv[1], sv[2]), "iteration": it.value}

    def gradient(self, alpha: float = 1.0):
        """Voxel-frame bracket B = alpha*A - R/Z and its parts at the current state."""
        B = torch.empty((self.n, 3), dtype=torch.float64, device="cuda")
        A = torch.empty_like(B)
        R = torch.empty_like(B)
        Zi = torch.empty(self.n, dtype=torch.float64, device="cuda")
        vis = torch.empty(self.n, dtype=torch.int32, device="cuda")
        Z = C.c_double()
        _check(load().pixelsne3_gradient(self._h, float(alpha), _ptr(B), _ptr(A), _ptr(R),
                                         _ptr(Zi), _ptr(vis), C.byref(Z)))
        return {"B": B, "A": A, "R": R, "Zi": Zi, "visits": vis, "Z": Z.value}

    def export_tree(self):
        L = self.L
        sizes = (C.c_int64 * (L + 1))()
        _check(load().pixelsne3_export_tree(self._h, sizes, None, None, None, None, None))
        sizes = [sizes[i] for i in range(L + 1)]
        m = sum(sizes)
        keys = torch.empty(self.n, dtype=torch.int32, device="cuda")
        perm = torch.empty(self.n, dtype=torch.int32, device="cuda")
        pre = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        cnt = torch.empty(max(m, 1), dtype=torch.int32, device="cuda")
        sm = torch.empty((max(m, 1), 3), dtype=torch.float64, device="cuda")
        s2 = (C.c_int64 * (L + 1))()
        _check(load().pixelsne3_export_tree(self._h, s2, _ptr(keys), _ptr(perm), _ptr(pre),
                                            _ptr(cnt), _ptr(sm)))
        return {"level_size": sizes, "keys": keys, "perm": perm, "prefix": pre[:m],
                "count": cnt[:m], "sum": sm[:m]}

    def kl(self) -> float:
        """KL(P || Q) of the 3-D embedding with the exact normaliser."""
        v = C.c_double()
        _check(load().pixelsne3_kl(self._h, C.byref(v)))
        return v.value

    def close(self):
        if getattr(self, "_h", None):
            load().pixelsne3_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def knn(X: torch.Tensor, k: int):
    """Device kNN of the rows of X: (idx int32 [n,k], d2 float64 [n,k])."""
    n, D = X.shape
    X = X.contiguous()
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, k), dtype=torch.float64, device=X.device)
    _check(load().pixelsne_knn(_ptr(X), n, D, _X_TYPES[X.dtype], int(k), _ptr(idx), _ptr(d2),
                               _stream()))
    return idx, d2


def knn_approx(X: torch.Tensor, k: int, trees: int = 4, leaf_size: int = 0, explore: int = 1,
               seed: int = 0):
    """Approximate kNN (random-projection trees + neighbour exploring):
    (idx int32 [n,k], d2 float64 [n,k])."""
    n, D = X.shape
    X = X.contiguous()
    idx = torch.empty((n, k), dtype=torch.int32, device=X.device)
    d2 = torch.empty((n, k), dtype=torch.float64, device=X.device)
    _check(load().pixelsne_knn_approx(_ptr(X), n, D, _X_TYPES[X.dtype], int(k), int(trees),
                                      int(leaf_size), int(explore), int(seed) & (2 ** 64 - 1),
                                      _ptr(idx), _ptr(d2), _stream()))
    return idx, d2


def perplexity(d2: torch.Tensor, u: float):
    """Device perplexity calibration: (P_cond float64 [n,k], beta float64 [n])."""
    n, k = d2.shape
    d2 = d2.to(torch.float64).contiguous()
    P = torch.empty_like(d2)
    beta = torch.empty(n, dtype=torch.float64, device=d2.device)
    _check(load().pixelsne_perplexity(_ptr(d2), n, k, float(u), _ptr(P), _ptr(beta), _stream()))
    return P, beta


class MLP:
    """Learned placement network on the GPU (wraps pixelsne_mlp*)."""

    def __init__(self, d_in: int, h1: int, h2: int, seed: int = 0):
        h = load().pixelsne_mlp_create(int(d_in), int(h1), int(h2), int(seed), _stream())
        if not h:
            raise PixelSNEError(PSNE_E_INVAL, _err())
        self._h = C.c_void_p(h)
        self.d, self.h1, self.h2 = d_in, h1, h2
        self.n_params = load().pixelsne_mlp_num_params(self._h)

    def params(self) -> torch.Tensor:
        t = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        _check(load().pixelsne_mlp_get_params(self._h, _ptr(t)))
        return t

    def set_params(self, theta):
        t = torch.as_tensor(theta, dtype=torch.float32).cuda().contiguous()
        _check(load().pixelsne_mlp_set_params(self._h, _ptr(t)))

    def set_norm(self, mean, inv_std):
        mu = torch.as_tensor(mean, dtype=torch.float32).cuda().contiguous()
        isd = torch.as_tensor(inv_std, dtype=torch.float32).cuda().contiguous()
        _check(load().pixelsne_mlp_set_norm(self._h, _ptr(mu), _ptr(isd)))

    def fit_norm(self, X: torch.Tensor):
        X = X.contiguous()
        _check(load().pixelsne_mlp_fit_norm(self._h, _ptr(X), X.shape[0]))

    def grad(self, X: torch.Tensor, Y01: torch.Tensor):
        X, Y01 = X.contiguous(), Y01.contiguous()
        g = torch.empty(self.n_params, dtype=torch.float32, device="cuda")
        loss = C.c_double()
        _check(load().pixelsne_mlp_grad(self._h, _ptr(X), _ptr(Y01), X.shape[0], _ptr(g),
                                        C.byref(loss)))
        return loss.value, g

    def train(self, X: torch.Tensor, Y01: torch.Tensor, epochs: int, batch: int = 4096,
              lr: float = 1e-3) -> float:
        X, Y01 = X.contiguous(), Y01.contiguous()
        loss = C.c_double()
        _check(load().pixelsne_mlp_train(self._h, _ptr(X), _ptr(Y01), X.shape[0], int(epochs),
                                         int(batch), float(lr), C.byref(loss)))
        return loss.value

    def adam_step(self, grad, lr: float = 1e-3):
        """One Adam step with a caller-supplied flat FP32 gradient."""
        g = torch.as_tensor(grad, dtype=torch.float32).cuda().contiguous()
        _check(load().pixelsne_mlp_adam_step(self._h, _ptr(g), float(lr)))

    def forward(self, X: torch.Tensor) -> torch.Tensor:
        X = X.contiguous()
        out = torch.empty((X.shape[0], 2), dtype=torch.float32, device="cuda")
        _check(load().pixelsne_mlp_forward(self._h, _ptr(X), X.shape[0], _ptr(out)))
        return out

    def place(self, X: torch.Tensor, screen: int, s) -> torch.Tensor:
        """Initial embedding (float64 [n, 2], y frame) for Context.from_data(Y_init=...)."""
        X = X.contiguous()
        Y = torch.empty((X.shape[0], 2), dtype=torch.float64, device="cuda")
        sv = (C.c_double * 2)(float(s[0]), float(s[1]))
        _check(load().pixelsne_mlp_place(self._h, _ptr(X), X.shape[0], int(screen), sv, _ptr(Y)))
        return Y

    def close(self):
        if getattr(self, "_h", None):
            load().pixelsne_mlp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
