"""MI355X term-network contractor for the SVD-based approximate simulation of
noisy quantum circuits (arXiv 2211.17028).

The compute path is the HIP library libtn_gfx950.so (C ABI in include/tn.h);
``tn`` is its ctypes binding.  Build with ``python -m paper_2211_17028_amd.build``.
"""
from . import tn  # noqa: F401
