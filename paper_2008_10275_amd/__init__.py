"""MI355X-native low-rank ChebyshevT solver for parameter-dependent matrix
equations (Benner, Richter, Weinhandl, arXiv 2008.10275).

The product is liblrcheb.so (HIP kernels for gfx950 + host factorisation)
behind the C ABI of include/lrcheb.h; ``lrcheb`` is its ctypes binding.
"""
from . import lrcheb  # noqa: F401
