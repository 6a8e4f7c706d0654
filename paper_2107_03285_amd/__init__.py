"""MI355X (gfx950) hot path of Sparse Gauss-Newton sensitivity analysis.

The compute lives in libsgn.so (HIP kernels behind the C ABI of
include/sgn.h); ``paper_2107_03285_amd.sgn`` is its ctypes binding.
"""
from .sgn import Context, default_options, load_library  # noqa: F401
