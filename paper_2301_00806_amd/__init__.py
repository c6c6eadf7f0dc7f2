"""MI355X engine for the weak-pseudo-manifold sweep of arXiv 2301.00806.

The compute path lives in libwpm.so (C++ host preparation and HIP kernels for
gfx950) behind the C ABI of include/wpm.h; this package binds it with ctypes.
Importing the package loads nothing: the library is loaded on first use and
raises ImportError if it has not been built.
"""
__all__ = ["engine"]
