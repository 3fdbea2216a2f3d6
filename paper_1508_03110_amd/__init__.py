"""MI355X-native ALS / ALS-NCG hot path (arXiv:1508.03110).

``_lib``   -- ctypes binding of libalsncg.so (the C ABI in include/alsncg.h);
``solver`` -- device buffers (PyTorch) and the ALS / ALS-NCG loops calling it.

Importing the package does not touch the GPU; the library is loaded on first
use and its absence is an error (there is no CPU fallback).
"""
from . import _lib  # noqa: F401

__all__ = ["_lib"]
