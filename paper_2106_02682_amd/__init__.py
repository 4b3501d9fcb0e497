"""MI355X-native hot path of the translation-invariant two-marginal SDP solver
(Khoo & Lindsey, arXiv 2106.02682, Algorithm 6).

The compute path is libvemb.so (HIP kernels for gfx950 behind the C ABI of
include/vemb.h); ``vemb`` is its ctypes binding.
"""
from . import vemb  # noqa: F401
