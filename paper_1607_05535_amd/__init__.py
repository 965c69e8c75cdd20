"""MI355X-native HEVI dynamical-core step of THOR (arXiv:1607.05535).

The computation lives in libthor.so (HIP kernels for gfx950 behind the C ABI
of include/thor.h); ``thor`` is its ctypes binding.
"""
