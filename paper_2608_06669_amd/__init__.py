"""pnkcc: preconditioned Newton-Krylov CCSD on AMD MI355X (gfx950).

The solver runs in libpnkcc.so (hand-written HIP kernels behind the C
boundary of include/pnkcc.h); this package only marshals arguments.
"""

from ._lib import LIB_PATH, load  # noqa: F401
from .api import (CCError, DeviceGauge, DeviceProblem, Handle, Server, diag_gemm, diag_gemm_batched,  # noqa: F401
                  fp_opts, gemm_noalloc, hessenberg_eigenvalues, occ_sets, pnk_opts, workspace_bytes)

__all__ = ["CCError", "DeviceGauge", "DeviceProblem", "Handle", "Server", "diag_gemm", "diag_gemm_batched", "fp_opts", "gemm_noalloc",
           "hessenberg_eigenvalues", "occ_sets", "pnk_opts",
           "workspace_bytes", "load", "LIB_PATH"]
