"""PixelSNE (Kim et al., arXiv:1611.02568) on AMD Instinct MI355X (gfx950).

The method runs in hand-written HIP kernels behind the C ABI of
``include/pixelsne.h`` (``libpixelsne.so``); ``pixelsne`` is its ctypes
binding and ``datagen`` draws the seeded synthetic workloads.  The binding is
imported lazily so that ``datagen`` can be used without loading the GPU
library.
"""
from . import datagen  # noqa: F401

_BINDING = ("Context", "knn", "perplexity", "default_params", "load", "PixelSNEError")


def __getattr__(name):
    if name in _BINDING or name == "pixelsne":
        import importlib
        mod = importlib.import_module(__name__ + ".pixelsne")
        return mod if name == "pixelsne" else getattr(mod, name)
    raise AttributeError(name)
