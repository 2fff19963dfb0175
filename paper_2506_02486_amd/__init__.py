"""MI355X-native acoustic isotropic finite-difference hot path (HIP for gfx950).

The C ABI lives in ``include/fd.h`` / ``libfd.so``; this package is its thin Python
binding (``_lib``), torch-facing wrappers (``api``), the checkpointed FWI gradient
(``fwi``) and the shot server (``serving``).  Importing the package does not load
the library; the first call into it does, and raises if it was not built.
"""
from importlib import import_module

__all__ = ["api", "fwi", "serving", "build"]


def __getattr__(name):
    if name in __all__:
        return import_module(f".{name}", __name__)
    raise AttributeError(name)
