"""MI355X (gfx950) row-wise sparse Tucker ALS (P-Tucker, arXiv 1710.02261).

The work runs in the HIP library ``libptucker.so`` built from ``csrc/``; its C
ABI is ``include/ptucker.h``. This package is a thin ctypes binding with the
same call names: it checks and marshals arguments (torch tensors are used only
as device memory and for the current stream) and raises ``PtkError`` on a
failing status. There is no CPU fallback: importing the binding fails when the
library has not been built.
"""
from ._native import (  # noqa: F401
    Context, PtkError, Server, PREC_FP64_ACC, PREC_FP32, PREC_BF16, PREC_BF16X3, library_path,
    load_library, coo_scan, coo_read, fp64_rates,
)

__all__ = ["Context", "PtkError", "Server", "PREC_FP64_ACC", "PREC_FP32", "PREC_BF16", "PREC_BF16X3",
           "library_path", "load_library", "coo_scan", "coo_read",
           "fp64_rates"]
