"""Ratio-filter dechirping (arXiv:2601.18835) on AMD MI355X.

The compute path is librfd.so (hand-written HIP for gfx950, C ABI in
include/rfd.h); `rfd` is its ctypes binding and `pipeline` a small driver
that moves synthetic inputs into device tensors and calls the library.
Importing the package loads librfd.so and fails if it has not been built.
"""
from . import rfd  # noqa: F401  (loads librfd.so or raises)
from .rfd import *  # noqa: F401,F403
