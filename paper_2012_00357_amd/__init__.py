"""MI355X (gfx950) projection library for model-free data-driven solid mechanics.

The computation lives in libdd.so (HIP kernels behind a C ABI, include/dd.h);
this package is its Python binding (`_lib`) and build script (`build`).
Importing the package does not load the library; `paper_2012_00357_amd.lib()`
or any binding function does, and raises if libdd.so has not been built.
"""

__all__ = ["lib"]


def lib():
    """The ctypes binding module (loads libdd.so; raises ImportError if it is not built)."""
    from . import _lib
    return _lib
