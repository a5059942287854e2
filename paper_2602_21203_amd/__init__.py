"""MI355X (gfx950) implementation of the Squint visual SAC update (arXiv 2602.21203).

The compute lives in libsquint.so (HIP kernels behind the C ABI of
include/squint.h); this package is the Python binding.  Importing `api`
loads the library and raises if it was not built.
"""
from .configs import CONFIGS  # noqa: F401
