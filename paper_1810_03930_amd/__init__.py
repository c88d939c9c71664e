"""MI355X (gfx950) PLAM / PCAL solver for min f(X) s.t. X^T X = I.

The compute path is the HIP library ``libstiefel.so`` (C ABI in
``include/stiefel.h``); ``stiefel`` is its Python binding.
"""
from . import _lib  # noqa: F401

__all__ = ["stiefel", "_lib"]
