"""Differentiable implicit soft-body step and adjoint for AMD MI355X (gfx950).

The compute path is the HIP library libisb.so (C ABI in include/isb.h); this package is its
thin Python binding. Importing it does not load the library; `isb.load_library()` (called
by `Context`) does, and raises ImportError if it has not been built.
"""
from . import isb  # noqa: F401
from .isb import Context, IsbError, load_library  # noqa: F401

__all__ = ["Context", "IsbError", "load_library", "isb"]
