"""Python face of the C boundary: same names as include/pnkcc.h, torch
tensors in place of raw device pointers. Marshalling only."""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L
from ._lib import cc_fp_opts, cc_gauge, cc_info, cc_pnk_opts, cc_problem, cc_server_stats


class CCError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _lib():
    return L.load()


def _ptr(t: torch.Tensor) -> int:
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if t.dtype != torch.float64 or not t.is_contiguous() or t.device.type != "cuda":
        raise ValueError("tensors must be contiguous float64 on a GPU")
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, torch.cuda.Stream):
        return stream.cuda_stream
    return int(stream)


class DeviceProblem:
    """f_oo, f_ov, f_vv, L as device tensors plus the cc_problem struct."""

    def __init__(self, f_oo, f_ov, f_vv, Lfac, device="cuda"):
        conv = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device).contiguous()  # noqa: E731
        self.f_oo, self.f_ov, self.f_vv, self.L = conv(f_oo), conv(f_ov), conv(f_vv), conv(Lfac)
        self.nocc = self.f_oo.shape[0]
        self.nvir = self.f_vv.shape[0]
        self.naux = self.L.shape[0]
        self.struct = cc_problem(self.nocc, self.nvir, self.naux, _ptr(self.f_oo), _ptr(self.f_ov),
                                 _ptr(self.f_vv), _ptr(self.L))

    @classmethod
    def from_problem(cls, p, device="cuda"):
        return cls(p.f_oo, p.f_ov, p.f_vv, p.L, device=device)

    def zeros_t(self):
        o, v = self.nocc, self.nvir
        dev = self.f_oo.device
        return (torch.zeros(o, v, dtype=torch.float64, device=dev),
                torch.zeros(o, o, v, v, dtype=torch.float64, device=dev))


class DeviceGauge:
    """W_o [o][m_o] and W_v [v][m_v] of a non-orthogonal (m = o, v) or
    redundant (m above) gauge as device tensors plus the cc_gauge struct
    (column mu: gauge function mu in the orbitals)."""

    def __init__(self, w_oo, w_vv, device="cuda"):
        conv = lambda a: torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device=device).contiguous()  # noqa: E731
        self.w_oo, self.w_vv = conv(w_oo), conv(w_vv)
        self.m_occ, self.m_vir = int(self.w_oo.shape[1]), int(self.w_vv.shape[1])
        self.struct = cc_gauge(_ptr(self.w_oo), _ptr(self.w_vv), self.m_occ, self.m_vir)

    def zeros_theta(self):
        dev = self.w_oo.device
        mo, mv = self.m_occ, self.m_vir
        return (torch.zeros(mo, mv, dtype=torch.float64, device=dev),
                torch.zeros(mo, mo, mv, mv, dtype=torch.float64, device=dev))

    def theta_shapes(self):
        return (self.m_occ, self.m_vir), (self.m_occ, self.m_occ, self.m_vir, self.m_vir)

    def orbital_shapes(self):
        o, v = int(self.w_oo.shape[0]), int(self.w_vv.shape[0])
        return (o, v), (o, o, v, v)


def pnk_opts(**kw) -> cc_pnk_opts:
    o = cc_pnk_opts()
    _lib().cc_pnk_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if k == "jvp_prec" and isinstance(v, str):
            v = L.PRECISIONS[v]
        if k == "protocol" and isinstance(v, str):
            v = L.PROTOCOLS[v]
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def fp_opts(**kw) -> cc_fp_opts:
    o = cc_fp_opts()
    _lib().cc_fp_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


class Handle:
    def __init__(self, device: int = 0, workspace_limit: int = 0):
        h = ctypes.c_void_p()
        st = _lib().cc_create(ctypes.byref(h), device, workspace_limit)
        if st != L.CC_OK:
            raise CCError(st, "cc_create failed")
        self._h = h

    def close(self):
        if self._h:
            _lib().cc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, st, ok=(L.CC_OK,)):
        if st not in ok:
            raise CCError(st, _lib().cc_last_error(self._h).decode())
        return st

    # ---- the C calls ----
    def residual(self, p: DeviceProblem, t1, t2, r1=None, r2=None, energy=False, stream=None):
        r1 = torch.empty_like(t1) if r1 is None else r1
        r2 = torch.empty_like(t2) if r2 is None else r2
        e = ctypes.c_double(0.0)
        self._check(_lib().cc_residual(self._h, ctypes.byref(p.struct), _ptr(t1), _ptr(t2), _ptr(r1), _ptr(r2),
                                       ctypes.byref(e) if energy else None, _stream(stream)))
        return (r1, r2, e.value) if energy else (r1, r2)

    def energy(self, p: DeviceProblem, t1, t2, stream=None):
        e = ctypes.c_double(0.0)
        self._check(_lib().cc_energy(self._h, ctypes.byref(p.struct), _ptr(t1), _ptr(t2), ctypes.byref(e),
                                     _stream(stream)))
        return e.value

    def jvp(self, p: DeviceProblem, t1, t2, v1, v2, prec="fp64", out=None, stream=None):
        y1, y2 = (torch.empty_like(v1), torch.empty_like(v2)) if out is None else out
        pr = L.PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self._check(_lib().cc_jvp(self._h, ctypes.byref(p.struct), _ptr(t1), _ptr(t2), _ptr(v1), _ptr(v2),
                                  _ptr(y1), _ptr(y2), pr, _stream(stream)))
        return y1, y2

    def fock_apply(self, p: DeviceProblem, x1, x2, stream=None):
        y1, y2 = torch.empty_like(x1), torch.empty_like(x2)
        self._check(_lib().cc_fock_apply(self._h, ctypes.byref(p.struct), _ptr(x1), _ptr(x2), _ptr(y1), _ptr(y2),
                                         _stream(stream)))
        return y1, y2

    def precond_solve(self, p: DeviceProblem, b1, b2, rtol=1e-12, maxit=200, stream=None, pair_symmetric=False):
        """A_F x = b; pair_symmetric=True calls cc_precond_solve_pairsym (b2
        must satisfy b2[j, i] = b2[i, j].T)."""
        x1, x2 = torch.empty_like(b1), torch.empty_like(b2)
        it = ctypes.c_int(0)
        fn = _lib().cc_precond_solve_pairsym if pair_symmetric else _lib().cc_precond_solve
        st = self._check(fn(self._h, ctypes.byref(p.struct), _ptr(b1), _ptr(b2), _ptr(x1), _ptr(x2), rtol, maxit,
                            ctypes.byref(it), _stream(stream)),
                         ok=(L.CC_OK, L.CC_NOT_CONVERGED))
        return x1, x2, it.value, st == L.CC_OK

    def solve_pnk(self, p: DeviceProblem, t1=None, t2=None, stream=None, **opts):
        o = pnk_opts(**opts)
        if t1 is None:
            t1, t2 = p.zeros_t()
            o.init_mp2 = 1 if "init_mp2" not in opts else o.init_mp2
        info = cc_info()
        st = self._check(_lib().cc_solve_pnk(self._h, ctypes.byref(p.struct), ctypes.byref(o), _ptr(t1), _ptr(t2),
                                             ctypes.byref(info), _stream(stream)),
                         ok=(L.CC_OK, L.CC_NOT_CONVERGED, L.CC_ERR_NAN))
        return t1, t2, dict(info.as_dict(), status=L.STATUS_NAMES[st])

    def solve_fp_diis(self, p: DeviceProblem, t1=None, t2=None, stream=None, **opts):
        o = fp_opts(**opts)
        if t1 is None:
            t1, t2 = p.zeros_t()
        info = cc_info()
        st = self._check(_lib().cc_solve_fp_diis(self._h, ctypes.byref(p.struct), ctypes.byref(o), _ptr(t1),
                                                 _ptr(t2), ctypes.byref(info), _stream(stream)),
                         ok=(L.CC_OK, L.CC_NOT_CONVERGED, L.CC_ERR_NAN))
        return t1, t2, dict(info.as_dict(), status=L.STATUS_NAMES[st])

    def fp_spectral_radius(self, p: DeviceProblem, t1, t2, q1, q2, shift=0.0, m=30, stream=None):
        """Spectral radius of the (S)FP map's Jacobian at (t1, t2) by m Arnoldi
        steps from (q1, q2); returns (rho, Ritz values as a complex array)."""
        rho = ctypes.c_double(0.0)
        nr = ctypes.c_int(0)
        re = np.zeros(m)
        im = np.zeros(m)
        self._check(_lib().cc_fp_spectral_radius(self._h, ctypes.byref(p.struct), _ptr(t1), _ptr(t2), _ptr(q1),
                                                 _ptr(q2), float(shift), int(m), ctypes.byref(rho),
                                                 re.ctypes.data, im.ctypes.data, ctypes.byref(nr), _stream(stream)))
        return rho.value, (re + 1j * im)[: nr.value]

    # ---- non-orthogonal gauges ----
    def gauge_transform(self, p: DeviceProblem, g: DeviceGauge, x1, x2, to_gauge=True, stream=None):
        s1, s2 = g.theta_shapes() if to_gauge else g.orbital_shapes()
        y1 = torch.empty(s1, dtype=torch.float64, device=x1.device)
        y2 = torch.empty(s2, dtype=torch.float64, device=x1.device)
        self._check(_lib().cc_gauge_transform(self._h, ctypes.byref(p.struct), ctypes.byref(g.struct),
                                              1 if to_gauge else 0, _ptr(x1), _ptr(x2), _ptr(y1), _ptr(y2),
                                              _stream(stream)))
        return y1, y2

    def residual_gauge(self, p: DeviceProblem, g: DeviceGauge, th1, th2, energy=False, stream=None):
        r1, r2 = torch.empty_like(th1), torch.empty_like(th2)
        e = ctypes.c_double(0.0)
        self._check(_lib().cc_residual_gauge(self._h, ctypes.byref(p.struct), ctypes.byref(g.struct), _ptr(th1),
                                             _ptr(th2), _ptr(r1), _ptr(r2), ctypes.byref(e) if energy else None,
                                             _stream(stream)))
        return (r1, r2, e.value) if energy else (r1, r2)

    def jvp_gauge(self, p: DeviceProblem, g: DeviceGauge, th1, th2, v1, v2, prec="fp64", stream=None):
        y1, y2 = torch.empty_like(v1), torch.empty_like(v2)
        pr = L.PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self._check(_lib().cc_jvp_gauge(self._h, ctypes.byref(p.struct), ctypes.byref(g.struct), _ptr(th1),
                                        _ptr(th2), _ptr(v1), _ptr(v2), _ptr(y1), _ptr(y2), pr, _stream(stream)))
        return y1, y2

    def solve_pnk_gauge(self, p: DeviceProblem, g: DeviceGauge, th1=None, th2=None, stream=None, **opts):
        o = pnk_opts(**opts)
        if th1 is None:
            th1, th2 = g.zeros_theta()
            o.init_mp2 = 1 if "init_mp2" not in opts else o.init_mp2
        info = cc_info()
        st = self._check(_lib().cc_solve_pnk_gauge(self._h, ctypes.byref(p.struct), ctypes.byref(g.struct),
                                                   ctypes.byref(o), _ptr(th1), _ptr(th2), ctypes.byref(info),
                                                   _stream(stream)),
                         ok=(L.CC_OK, L.CC_NOT_CONVERGED, L.CC_ERR_NAN))
        return th1, th2, dict(info.as_dict(), status=L.STATUS_NAMES[st])

    def solve_fp_diis_gauge(self, p: DeviceProblem, g: DeviceGauge, th1=None, th2=None, stream=None, **opts):
        o = fp_opts(**opts)
        if th1 is None:
            th1, th2 = g.zeros_theta()
        info = cc_info()
        st = self._check(_lib().cc_solve_fp_diis_gauge(self._h, ctypes.byref(p.struct), ctypes.byref(g.struct),
                                                       ctypes.byref(o), _ptr(th1), _ptr(th2), ctypes.byref(info),
                                                       _stream(stream)),
                         ok=(L.CC_OK, L.CC_NOT_CONVERGED, L.CC_ERR_NAN))
        return th1, th2, dict(info.as_dict(), status=L.STATUS_NAMES[st])

    def timing(self, enable: bool = True):
        self._check(_lib().cc_diag_timing(self._h, 1 if enable else 0))

    def contraction_flops(self, p: DeviceProblem, prec="fp64", stream=None):
        """(residual, J v) matrix-core flops as implemented: 2 M N K per
        contraction at its own sizes (cc_diag_contraction_flops)."""
        rf, jf = ctypes.c_double(0.0), ctypes.c_double(0.0)
        pr = L.PRECISIONS[prec] if isinstance(prec, str) else int(prec)
        self._check(_lib().cc_diag_contraction_flops(self._h, ctypes.byref(p.struct), pr, ctypes.byref(rf),
                                                     ctypes.byref(jf), _stream(stream)))
        return rf.value, jf.value

    def timing_read(self, slot: int):
        """(launch count, total ms) of a timing slot: 0 ladder contraction,
        1 residual, 2 J v, 3 A_F product, 4 inner A_F solve."""
        c, t = ctypes.c_int(0), ctypes.c_double(0.0)
        self._check(_lib().cc_diag_timing_read(self._h, slot, ctypes.byref(c), ctypes.byref(t)))
        return c.value, t.value

    def history(self):
        n = _lib().cc_last_history(self._h, None, 0)
        buf = (ctypes.c_double * (2 * max(n, 1)))()
        _lib().cc_last_history(self._h, buf, n)
        return np.array(buf[:2 * n]).reshape(n, 2)


def diag_gemm(A, B, C, a_strides, b_strides, c_strides, M, N, K, alpha=1.0, beta=0.0, prec="fp64", stream=None):
    """C = alpha A B + beta C through the library's matrix-core kernel."""
    st = _lib().cc_diag_gemm(M, N, K, _ptr(A), a_strides[0], a_strides[1], _ptr(B), b_strides[0], b_strides[1],
                             _ptr(C), c_strides[0], c_strides[1], alpha, beta,
                             L.PRECISIONS[prec] if isinstance(prec, str) else int(prec), _stream(stream))
    if st != L.CC_OK:
        raise CCError(st, "cc_diag_gemm failed")
    return C


def diag_gemm_batched(A, B, C, a_strides, b_strides, c_strides, M, N, K, nbatch, alpha=1.0, beta=0.0, prec="fp64",
                      precast=False, splitk=False, stream=None):
    """C[b] = alpha A[b] B[b] + beta C[b]; strides are (row, col, batch)
    element strides. precast rounds FP64 operands of an FP32/BF16 product
    once into a scratch copy first; splitk allows the split contraction."""
    st = _lib().cc_diag_gemm_batched(M, N, K, nbatch, _ptr(A), a_strides[0], a_strides[1], a_strides[2], _ptr(B),
                                     b_strides[0], b_strides[1], b_strides[2], _ptr(C), c_strides[0], c_strides[1],
                                     c_strides[2], alpha, beta,
                                     L.PRECISIONS[prec] if isinstance(prec, str) else int(prec),
                                     (1 if precast else 0) | (2 if splitk else 0), _stream(stream))
    if st != L.CC_OK:
        raise CCError(st, "cc_diag_gemm_batched failed")
    return C


def gemm_noalloc(A, B, C, a_strides, b_strides, c_strides, M, N, K, nbatch, alpha=1.0, beta=0.0, prec="fp64",
                 precast=False, splitk=False, stream=None):
    """cc_gemm_noalloc: diag_gemm_batched's product with its scratch in the
    library's fixed device array (no allocation; does not synchronise)."""
    st = _lib().cc_gemm_noalloc(M, N, K, nbatch, _ptr(A), a_strides[0], a_strides[1], a_strides[2], _ptr(B),
                                b_strides[0], b_strides[1], b_strides[2], _ptr(C), c_strides[0], c_strides[1],
                                c_strides[2], alpha, beta, L.PRECISIONS[prec] if isinstance(prec, str) else int(prec),
                                (1 if precast else 0) | (2 if splitk else 0), _stream(stream))
    if st != L.CC_OK:
        raise CCError(st, "cc_gemm_noalloc failed")
    return C


def occ_sets(nvir):
    """The occupied A_F kernel's position sets for nvir virtuals
    (cc_diag_occ_sets; host code, no GPU): arrays a, b, lane_t of shape
    (sets, 64)."""
    nb = (nvir + 7) // 8
    cap = 64 * nb * nb
    a = np.zeros(cap, dtype=np.int32)
    b = np.zeros(cap, dtype=np.int32)
    lt = np.zeros(cap, dtype=np.int32)
    n = ctypes.c_int(0)
    st = _lib().cc_diag_occ_sets(nvir, a.ctypes.data, b.ctypes.data, lt.ctypes.data, cap, ctypes.byref(n))
    if st != L.CC_OK:
        raise CCError(st, "cc_diag_occ_sets failed")
    k = 64 * n.value
    return a[:k].reshape(-1, 64), b[:k].reshape(-1, 64), lt[:k].reshape(-1, 64)


def hessenberg_eigenvalues(H) -> np.ndarray:
    """Eigenvalues of a real upper Hessenberg matrix by the library's host
    QR iteration (cc_diag_hessenberg_eigenvalues; no GPU needed)."""
    H = np.ascontiguousarray(H, dtype=np.float64)
    m = H.shape[0]
    re = np.zeros(m)
    im = np.zeros(m)
    st = _lib().cc_diag_hessenberg_eigenvalues(m, H.ctypes.data, re.ctypes.data, im.ctypes.data)
    if st != L.CC_OK:
        raise CCError(st, "cc_diag_hessenberg_eigenvalues failed")
    return re + 1j * im


def workspace_bytes(nocc, nvir, naux, lowp_flags=0, m_max=20, inner_restart=30, diis_size=0) -> int:
    return _lib().cc_workspace_bytes(nocc, nvir, naux, lowp_flags, m_max, inner_restart, diis_size)


class Server:
    """Continuous-batching PNK server on one GPU (cc_server_*)."""

    def __init__(self, device=0, mem_budget=0, max_slots=4):
        s = ctypes.c_void_p()
        st = _lib().cc_server_create(ctypes.byref(s), device, mem_budget, max_slots)
        if st != L.CC_OK:
            raise CCError(st, "cc_server_create failed")
        self._s = s
        self._shapes = {}

    def submit(self, problem, **opts) -> int:
        """problem: host arrays (gen.Problem or anything with f_oo, f_ov, f_vv, L)."""
        arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (problem.f_oo, problem.f_ov, problem.f_vv,
                                                                  problem.L)]
        ps = cc_problem(arrs[0].shape[0], arrs[2].shape[0], arrs[3].shape[0],
                        *[a.ctypes.data_as(ctypes.c_void_p) for a in arrs])
        rid = ctypes.c_uint64(0)
        st = _lib().cc_server_submit(self._s, ctypes.byref(ps), ctypes.byref(pnk_opts(**opts)), ctypes.byref(rid))
        if st != L.CC_OK:
            raise CCError(st, "submit failed")
        self._shapes[rid.value] = (arrs[0].shape[0], arrs[2].shape[0])
        return rid.value

    def poll(self, rid, want_amplitudes=True):
        done = ctypes.c_int(0)
        info = cc_info()
        o, v = self._shapes[rid]
        t1 = np.empty((o, v)) if want_amplitudes else None
        t2 = np.empty((o, o, v, v)) if want_amplitudes else None
        st = _lib().cc_server_poll(self._s, rid, ctypes.byref(done), ctypes.byref(info),
                                   t1.ctypes.data_as(ctypes.c_void_p) if t1 is not None else None,
                                   t2.ctypes.data_as(ctypes.c_void_p) if t2 is not None else None)
        if st == L.CC_ERR_ARG:
            raise CCError(st, f"unknown or already collected request {rid}")
        if not done.value:
            return None
        return dict(info.as_dict(), status=L.STATUS_NAMES.get(st, st), t1=t1, t2=t2)

    def drain(self):
        _lib().cc_server_drain(self._s)

    def stats(self):
        st = cc_server_stats()
        _lib().cc_server_get_stats(self._s, ctypes.byref(st))
        return st.as_dict()

    def times(self, rid):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _lib().cc_server_request_times(self._s, rid, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return a.value, b.value, c.value

    def close(self):
        if self._s:
            _lib().cc_server_destroy(self._s)
            self._s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
