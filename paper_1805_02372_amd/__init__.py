"""MI355X-native Toeplitz-hash privacy amplification (arXiv 1805.02372).

The compute path is libpa.so (HIP kernels for gfx950 behind the C ABI in
include/pa.h); ``pa`` is its ctypes binding.
"""
