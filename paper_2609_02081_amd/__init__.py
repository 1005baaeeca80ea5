"""Bilinear biquaternion GEMM for AMD MI355X (gfx950).

The compute path is the HIP library libbq.so behind the C-ABI declared in
include/bq.h; this package is a thin ctypes binding over it.  The library is
loaded on first use and a missing library raises: there is no CPU fallback.
"""
from ._binding import (BqError, FULL, REAL_QUAT, COMPLEX, REAL, bq_gemm, bq_gemm_noalloc, re_gemm, cx_gemm,
                       rq_gemm, workspace_size, plan_real_gemms, lib, handle, matrix, last_error,
                       trace_enable, trace_read, GroupedPlan, heev, heev_workspace_size)

__all__ = ["BqError", "FULL", "REAL_QUAT", "COMPLEX", "REAL", "bq_gemm", "bq_gemm_noalloc", "re_gemm", "cx_gemm",
           "rq_gemm", "workspace_size", "plan_real_gemms", "lib", "handle", "matrix", "last_error",
           "trace_enable", "trace_read", "GroupedPlan", "heev", "heev_workspace_size"]
