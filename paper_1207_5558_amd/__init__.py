"""MI355X-native directional SLSHT (Khalid et al., IEEE TSP 2013).

The transform runs in the gfx950 kernels of libslsht.so (C ABI in
include/slsht.h); ``api`` wraps it for PyTorch device tensors and streams, and
``inputs`` draws the seeded synthetic workloads.  Nothing is loaded at import
time: the library is opened on first use and a missing build is an error.
"""
__all__ = ["api", "inputs", "serving"]
