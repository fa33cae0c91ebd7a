"""MI355X (gfx950) implementation of Unified Spectral Bundling with Sketching (USBS,
Angell & McCallum, arXiv 2312.11801): the per-iteration block-Lanczos eigen step of
C - A^* y over CSR, the Nystrom sketch update and A(.) on low-rank factors, with the
rest of Alg. 1 (master QP interior point method, candidate, descent test, model update)
also in HIP kernels, behind the C ABI of include/usbs.h.

Importing the package loads nothing; `native.load_library()` loads libusbs.so.
"""
from .native import (Params, Solver, Server, UsbsError, footprint_bytes, load_library, solve_packed,  # noqa: F401
                     EXPORTS, LIB_PATH)

__all__ = ["Params", "Solver", "Server", "UsbsError", "footprint_bytes", "load_library", "solve_packed", "EXPORTS",
           "LIB_PATH"]
