"""MI355X (gfx950) motif-based community detection (arXiv 2412.12382).

The compute path is libmcd.so (hand-written HIP kernels behind the C ABI in
include/mcd.h); ``paper_2412_12382_amd.mcd`` is its ctypes binding.
"""
from . import mcd  # noqa: F401
