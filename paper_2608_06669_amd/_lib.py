"""ctypes binding of libpnkcc.so (include/pnkcc.h).

Argument marshalling only: every step of the solver runs in the library's
HIP kernels. Tensors are torch tensors on the GPU (float64, contiguous);
the binding passes their data pointers and the current HIP stream.
"""

from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpnkcc.so")

CC_OK = 0
CC_NOT_CONVERGED = 1
CC_ERR_ARG = -1
CC_ERR_OOM = -2
CC_ERR_HIP = -3
CC_ERR_NAN = -4
CC_ERR_REJECTED = -5
CC_ERR_INTERNAL = -6
STATUS_NAMES = {0: "CC_OK", 1: "CC_NOT_CONVERGED", -1: "CC_ERR_ARG", -2: "CC_ERR_OOM", -3: "CC_ERR_HIP",
                -4: "CC_ERR_NAN", -5: "CC_ERR_REJECTED", -6: "CC_ERR_INTERNAL"}

CC_FP64, CC_FP32, CC_BF16 = 0, 1, 2
PRECISIONS = {"fp64": CC_FP64, "fp32": CC_FP32, "bf16": CC_BF16}
CC_PNK, CC_NK, CC_INK = 0, 1, 2
PROTOCOLS = {"pnk": CC_PNK, "nk": CC_NK, "ink": CC_INK}


class cc_problem(ctypes.Structure):
    _fields_ = [("nocc", ctypes.c_int32), ("nvir", ctypes.c_int32), ("naux", ctypes.c_int32),
                ("f_oo", ctypes.c_void_p), ("f_ov", ctypes.c_void_p), ("f_vv", ctypes.c_void_p),
                ("L", ctypes.c_void_p)]


class cc_pnk_opts(ctypes.Structure):
    _fields_ = [("tol_inf", ctypes.c_double), ("max_newton", ctypes.c_int), ("m_max", ctypes.c_int),
                ("gamma", ctypes.c_double), ("alpha", ctypes.c_double), ("eta0", ctypes.c_double),
                ("eta_max", ctypes.c_double), ("inner_rtol", ctypes.c_double), ("inner_maxit", ctypes.c_int),
                ("inner_restart", ctypes.c_int), ("jvp_prec", ctypes.c_int), ("use_fd_jvp", ctypes.c_int),
                ("init_mp2", ctypes.c_int), ("protocol", ctypes.c_int), ("ccd", ctypes.c_int),
                ("stall_window", ctypes.c_int), ("stall_factor", ctypes.c_double),
                ("inner_rtol_jv", ctypes.c_double)]


class cc_fp_opts(ctypes.Structure):
    _fields_ = [("tol_inf", ctypes.c_double), ("max_iter", ctypes.c_int), ("diis_size", ctypes.c_int),
                ("diis_start", ctypes.c_int), ("level_shift", ctypes.c_double), ("init_mp2", ctypes.c_int),
                ("ccd", ctypes.c_int)]


class cc_gauge(ctypes.Structure):
    _fields_ = [("w_oo", ctypes.c_void_p), ("w_vv", ctypes.c_void_p), ("m_occ", ctypes.c_int),
                ("m_vir", ctypes.c_int)]


class cc_info(ctypes.Structure):
    _fields_ = [("e_corr", ctypes.c_double), ("res_inf", ctypes.c_double), ("res_2", ctypes.c_double),
                ("converged", ctypes.c_int), ("newton_iters", ctypes.c_int), ("n_residual", ctypes.c_int),
                ("n_jvp", ctypes.c_int), ("n_afmv", ctypes.c_int), ("n_inner_iters", ctypes.c_int),
                ("seconds", ctypes.c_double), ("stalled", ctypes.c_int)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class cc_server_stats(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint64), ("running", ctypes.c_uint64), ("finished", ctypes.c_uint64),
                ("rejected", ctypes.c_uint64), ("bytes_in_use", ctypes.c_size_t), ("peak_bytes", ctypes.c_size_t),
                ("budget", ctypes.c_size_t), ("max_slots", ctypes.c_int), ("peak_running", ctypes.c_int),
                ("host_bytes_held", ctypes.c_size_t), ("requests_held", ctypes.c_uint64),
                ("cached_bytes", ctypes.c_size_t), ("cached_handles", ctypes.c_uint64),
                ("handle_reuses", ctypes.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


P = ctypes.c_void_p
D = ctypes.c_double
I = ctypes.c_int
PP = ctypes.POINTER(ctypes.c_void_p)

# name -> (restype, argtypes)
SIGNATURES = {
    "cc_create": (I, [PP, I, ctypes.c_size_t]),
    "cc_destroy": (None, [P]),
    "cc_last_error": (ctypes.c_char_p, [P]),
    "cc_workspace_bytes": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, I, I, I, I]),
    "cc_residual": (I, [P, ctypes.POINTER(cc_problem), P, P, P, P, ctypes.POINTER(D), P]),
    "cc_energy": (I, [P, ctypes.POINTER(cc_problem), P, P, ctypes.POINTER(D), P]),
    "cc_jvp": (I, [P, ctypes.POINTER(cc_problem), P, P, P, P, P, P, I, P]),
    "cc_fock_apply": (I, [P, ctypes.POINTER(cc_problem), P, P, P, P, P]),
    "cc_precond_solve": (I, [P, ctypes.POINTER(cc_problem), P, P, P, P, D, I, ctypes.POINTER(I), P]),
    "cc_precond_solve_pairsym": (I, [P, ctypes.POINTER(cc_problem), P, P, P, P, D, I, ctypes.POINTER(I), P]),
    "cc_fp_spectral_radius": (I, [P, ctypes.POINTER(cc_problem), P, P, P, P, D, I, ctypes.POINTER(D), P, P,
                                  ctypes.POINTER(I), P]),
    "cc_diag_hessenberg_eigenvalues": (I, [I, P, P, P]),
    "cc_diag_occ_sets": (I, [I, P, P, P, ctypes.c_int64, ctypes.POINTER(I)]),
    "cc_pnk_opts_default": (None, [ctypes.POINTER(cc_pnk_opts)]),
    "cc_fp_opts_default": (None, [ctypes.POINTER(cc_fp_opts)]),
    "cc_solve_pnk": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_pnk_opts), P, P,
                         ctypes.POINTER(cc_info), P]),
    "cc_solve_fp_diis": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_fp_opts), P, P,
                             ctypes.POINTER(cc_info), P]),
    "cc_gauge_transform": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_gauge), I, P, P, P, P, P]),
    "cc_residual_gauge": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_gauge), P, P, P, P,
                              ctypes.POINTER(D), P]),
    "cc_jvp_gauge": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_gauge), P, P, P, P, P, P, I, P]),
    "cc_solve_pnk_gauge": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_gauge), ctypes.POINTER(cc_pnk_opts),
                               P, P, ctypes.POINTER(cc_info), P]),
    "cc_solve_fp_diis_gauge": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_gauge),
                                   ctypes.POINTER(cc_fp_opts), P, P, ctypes.POINTER(cc_info), P]),
    "cc_last_history": (I, [P, ctypes.POINTER(D), I]),
    "cc_server_create": (I, [PP, I, ctypes.c_size_t, I]),
    "cc_server_submit": (I, [P, ctypes.POINTER(cc_problem), ctypes.POINTER(cc_pnk_opts),
                             ctypes.POINTER(ctypes.c_uint64)]),
    "cc_server_poll": (I, [P, ctypes.c_uint64, ctypes.POINTER(I), ctypes.POINTER(cc_info), P, P]),
    "cc_server_drain": (I, [P]),
    "cc_server_get_stats": (I, [P, ctypes.POINTER(cc_server_stats)]),
    "cc_server_request_times": (I, [P, ctypes.c_uint64, ctypes.POINTER(D), ctypes.POINTER(D),
                                    ctypes.POINTER(D)]),
    "cc_server_destroy": (None, [P]),
    "cc_diag_timing": (I, [P, I]),
    "cc_diag_timing_read": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(D)]),
    "cc_diag_contraction_flops": (I, [P, ctypes.POINTER(cc_problem), I, ctypes.POINTER(D), ctypes.POINTER(D), P]),
    "cc_diag_gemm": (I, [I, I, I, P, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64, P,
                         ctypes.c_int64, ctypes.c_int64, D, D, I, P]),
    "cc_diag_gemm_batched": (I, [I, I, I, I, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int64,
                                 ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                 D, D, I, I, P]),
    "cc_gemm_noalloc": (I, [I, I, I, I, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int64,
                            ctypes.c_int64, ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                            D, D, I, I, P]),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2608_06669_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
