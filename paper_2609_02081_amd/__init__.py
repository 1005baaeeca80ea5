"""Bilinear biquaternion GEMM for AMD MI355X (gfx950).

The compute path is the HIP library libbq.so behind the C-ABI declared in
include/bq.h; this package is a thin ctypes binding over it.  The binding is
loaded on first use and raises if the library is missing: there is no CPU
fallback.
"""
__all__ = ["inputs"]
