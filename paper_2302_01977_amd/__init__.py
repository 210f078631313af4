"""MI355X-native sketching for adaptive HSS construction (arXiv 2302.01977).

The compute path is the C-ABI library ``libhsketch.so`` (include/sketch.h) with
hand-written HIP kernels for gfx950; ``api`` is a thin binding over it.
"""
from . import _abi  # noqa: F401

__all__ = ["api", "_abi"]
