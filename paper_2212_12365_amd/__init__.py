"""MI355X-native LES residual and Runge-Kutta stepping (arXiv 2212.12365 hot path).

The compute path is the HIP library liblesmi.so (C ABI in include/lesmi.h); the Python
module :mod:`paper_2212_12365_amd.lesmi` is its thin ctypes binding.
"""
__all__ = ["lesmi"]
