"""SIBFA many-body polarization on MI355X (gfx950).

The computation lives in libsibfa_pol.so (HIP kernels behind the C-ABI of
include/sibfa_pol.h); this package is its Python binding.  Importing the
package does not load the library; creating an Engine does, and fails if
it has not been built.
"""
from ._lib import LIB_PATH, exported_names, FP64, MIXED  # noqa: F401


def __getattr__(name):
    if name in ("Engine", "SibfaError", "default_params", "footprint_bytes"):
        from . import engine
        return getattr(engine, name)
    raise AttributeError(name)
