"""hmps: multi-level power-series H-matrix solver (arXiv 2307.03968) for one
AMD Instinct MI355X.

The compute path is libhmps.so (HIP kernels for gfx950 behind the C-ABI of
include/hmps.h); ``hmps`` is its ctypes binding.  Importing the package does
not load the library; the first call does, and fails loudly if it is not
built.
"""
from . import hmps  # noqa: F401
from .hmps import HMatrix, read_export, header_functions  # noqa: F401
