"""m2s -- MI355X-native matrix-free stencil sweeps (Mat2Stencil hot path).

The compute path is the C-ABI library libm2s.so (hand-written HIP kernels for
gfx950, declared in include/m2s.h); this package only marshals torch tensors
into it.  Importing the package is cheap: the library is loaded on first use,
and every entry point raises if it cannot be loaded.
"""
import importlib

from . import inputs  # noqa: F401

__all__ = ["inputs"]


def __getattr__(name):
    if name.startswith("_") or name in ("api", "build"):
        return importlib.import_module(f"{__name__}.{name}")
    api = importlib.import_module(f"{__name__}.api")
    try:
        return getattr(api, name)
    except AttributeError:
        raise AttributeError(name) from None
