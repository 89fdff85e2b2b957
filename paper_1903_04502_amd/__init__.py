"""MI355X (gfx950) library for the Dual Forward-Backward ADMM imaging path.

The compute runs in ``libpurimi.so`` (HIP kernels behind the C ABI of
``include/purimi.h``); ``purimi`` is its thin ctypes binding.
"""
from . import purimi  # noqa: F401
