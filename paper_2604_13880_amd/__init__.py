"""MI355X-native integral-image cartograms.

The compute path is libcg.so (HIP kernels for gfx950 behind the C ABI in
include/cg.h); `binding` is its ctypes binding.  Import the binding
explicitly: importing the package does not load the library.
"""
__all__ = ["binding", "build"]
