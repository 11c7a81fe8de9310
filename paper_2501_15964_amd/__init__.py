"""MI355X (gfx950) convex clustering path library.

The compute lives in libccm.so (hand-written HIP kernels behind a C ABI, see
include/ccm.h); this package is a thin ctypes binding that passes device
pointers and sizes.  PyTorch is used only to own device memory and streams.
"""
from .ccm import *  # noqa: F401,F403
from .ccm import __all__  # noqa: F401
