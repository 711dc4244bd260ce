"""MI355X (gfx950) implementation of the LCS flow-map / FTLE hot path.

The compute lives in a C-ABI HIP library (``liblcs_hip.so``, declared in
``include/lcs.h``); ``lcs`` is its thin ctypes binding.  ``inputs`` produces
seeded synthetic velocity frames and seed grids.
"""
from . import inputs  # noqa: F401

__all__ = ["inputs"]
