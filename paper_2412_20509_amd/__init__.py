"""MI355X-native block-wise adaptive SGD for generalized matrix factorization.

The compute lives in ``libgmf.so`` (hand-written HIP for gfx950, C ABI in
``include/gmf.h``); :mod:`paper_2412_20509_amd.gmf` is its ctypes binding.
"""
from . import gmf  # noqa: F401  (raises ImportError when libgmf.so is missing)

__all__ = ["gmf"]
