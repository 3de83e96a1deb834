"""Fock preconditioner, GMRES, PNK and FP+DIIS on top of oracle.ccsd.

TEST INFRASTRUCTURE ONLY (CPU float64 oracle; never imported by the product
path).

* A_F (equation Preconditioner, working equations in Appendix C): the
  matrix of <Phi_mu|[F, X_nu]|Phi_0>. In the residual normalisation of
  oracle.ccsd this is exactly the Jacobian of the residual at t = 0 for a
  Hamiltonian without two-electron part, so the factor 4 of the appendix's
  normalisation is absent; a scale factor cancels in left preconditioning.
  The singles block (not in the paper, which is CCD) follows from the same
  definition and couples to the doubles through f_ov.
* GMRES: Arnoldi with modified Gram-Schmidt and Givens rotations for the
  Hessenberg least-squares problem (Saad & Schultz, SIAM J. Sci. Stat.
  Comput. 7 (1986) 856), as in the PNK algorithm of Appendix F.
* PNK (Appendix F algorithm, Section "Adaptive Forcing"): Newton steps
  from A_F^{-1} J delta = -A_F^{-1} r, solved by GMRES with A_F^{-1} applied
  by an inner GMRES, stopped by the Eisenstat-Walker forcing term
  eta_k = gamma (||r_k|| / ||r_{k-1}||)^alpha with gamma = 0.9,
  alpha = 1.5.
* FP / SFP (Section "Theory", equation Commutator_MO; Appendix D): the
  Jacobi update with the diagonal of the Fock matrix, optionally shifted,
  accelerated by DIIS (Pulay, Chem. Phys. Lett. 73 (1980) 393).

Readings where the paper is silent (each is listed with its reason in the
design notes): the unknowns are the closed-shell amplitudes, doubles with
t_ij^ab = t_ji^ba, so every preconditioned vector is projected onto that
space (the identity on it in exact arithmetic); the stopping test uses
||r||_inf; the forcing test uses the
preconditioned GMRES residual estimate |g_{m+1}| <= eta_k beta; eta_0 = 0.5
and the Eisenstat-Walker safeguards (choice 2 of Eisenstat & Walker, SIAM J.
Sci. Comput. 17 (1996) 16) with eta_max = 0.9; the update sums the basis
vectors actually built; the inner solve is GMRES(30) to relative residual
1e-12; DIIS error vectors are the Jacobi steps -D^{-1} r.
"""

from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import ccsd


# ----------------------------------------------------------------- A_F ----

def fock_apply(f_oo, f_ov, f_vv, x1, x2):
    """A_F x for x = (x1 [o][v], x2 [o][o][v][v])."""
    y2 = (np.einsum("ac,ijcb->ijab", f_vv, x2)
          + np.einsum("bc,ijac->ijab", f_vv, x2)
          - np.einsum("ki,kjab->ijab", f_oo, x2)
          - np.einsum("kj,ikab->ijab", f_oo, x2))
    y1 = (np.einsum("ac,ic->ia", f_vv, x1)
          - np.einsum("ki,ka->ia", f_oo, x1)
          + np.einsum("kc,ikac->ia", f_ov, 2.0 * x2 - np.transpose(x2, (0, 1, 3, 2))))
    return y1, y2


def fock_solve_exact(f_oo, f_ov, f_vv, b1, b2):
    """A_F^{-1} b through the eigenvectors of f_oo and f_vv (A_F is a
    Kronecker sum of those blocks plus the f_ov coupling of the singles)."""
    eo, Uo = np.linalg.eigh(f_oo)
    ev, Uv = np.linalg.eigh(f_vv)
    bh = np.einsum("ki,lj,ca,db,klcd->ijab", Uo, Uo, Uv, Uv, b2, optimize=True)
    den2 = ev[None, None, :, None] + ev[None, None, None, :] - eo[:, None, None, None] - eo[None, :, None, None]
    x2 = np.einsum("ik,jl,ac,bd,klcd->ijab", Uo, Uo, Uv, Uv, bh / den2, optimize=True)
    c1 = b1 - np.einsum("kc,ikac->ia", f_ov, 2.0 * x2 - np.transpose(x2, (0, 1, 3, 2)))
    ch = Uo.T @ c1 @ Uv
    x1 = Uo @ (ch / (ev[None, :] - eo[:, None])) @ Uv.T
    return x1, x2


# ----------------------------------------------------- vector helpers ----

def pack(x1, x2):
    return np.concatenate([np.ravel(x1), np.ravel(x2)])


def unpack(x, o, v):
    return x[:o * v].reshape(o, v), x[o * v:].reshape(o, o, v, v)


# --------------------------------------------------------------- GMRES ----

@dataclass
class GmresResult:
    x: np.ndarray
    iters: int
    relres: float
    converged: bool


def gmres(apply, b, rtol=1e-12, maxit=200, restart=30, x0=None):
    """Restarted GMRES(restart) for apply(x) = b, relative to ||b||_2."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return GmresResult(x, 0, 0.0, True)
    total = 0
    r = b - apply(x) if x0 is not None else b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta <= rtol * bnorm or total >= maxit:
            return GmresResult(x, total, beta / bnorm, beta <= rtol * bnorm)
        m = restart
        Q = [r / beta]
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        k_done = 0
        for k in range(m):
            w = apply(Q[k])
            total += 1
            for i in range(k + 1):
                H[i, k] = np.dot(Q[i], w)
                w = w - H[i, k] * Q[i]
            H[k + 1, k] = np.linalg.norm(w)
            for i in range(k):
                a, c = H[i, k], H[i + 1, k]
                H[i, k] = cs[i] * a + sn[i] * c
                H[i + 1, k] = -sn[i] * a + cs[i] * c
            rho = np.hypot(H[k, k], H[k + 1, k])
            cs[k] = H[k, k] / rho
            sn[k] = H[k + 1, k] / rho
            hk1 = H[k + 1, k]
            H[k, k] = rho
            H[k + 1, k] = 0.0
            g[k + 1] = -sn[k] * g[k]
            g[k] = cs[k] * g[k]
            k_done = k + 1
            if abs(g[k + 1]) <= rtol * bnorm or total >= maxit or hk1 == 0.0:
                break
            Q.append(w / hk1)
        y = np.linalg.solve(np.triu(H[:k_done, :k_done]), g[:k_done])
        for i in range(k_done):
            x = x + y[i] * Q[i]
        r = b - apply(x)


def fock_solve_gmres(f_oo, f_ov, f_vv, b1, b2, rtol=1e-12, maxit=200, restart=30):
    o, v = b1.shape
    res = gmres(lambda x: pack(*fock_apply(f_oo, f_ov, f_vv, *unpack(x, o, v))),
                pack(b1, b2), rtol=rtol, maxit=maxit, restart=restart)
    x1, x2 = unpack(res.x, o, v)
    return x1, x2, res


# ------------------------------------------------------------- solvers ----

@dataclass
class SolveInfo:
    e_corr: float = 0.0
    res_inf: float = np.inf
    res_2: float = np.inf
    converged: bool = False
    newton_iters: int = 0
    n_residual: int = 0
    n_jvp: int = 0
    n_afmv: int = 0
    n_inner_iters: int = 0
    seconds: float = 0.0
    history: list = field(default_factory=list)  # (n_residual, ||r||_2, ||r||_inf)


class _Problem:
    """The maps the solvers iterate on. ccd=True is the paper's CCD level:
    t1 is held at zero and the singles equations are dropped, i.e. every
    vector (amplitudes, residual, J v, A_F^-1 b) has its singles part set to
    zero. With t1 = 0 the doubles residual of the T1-dressed equations is the
    CCD residual."""

    def __init__(self, f_oo, f_ov, f_vv, L, ccd=False):
        self.f_oo, self.f_ov, self.f_vv, self.L = f_oo, f_ov, f_vv, L
        self.o, self.v = f_oo.shape[0], f_vv.shape[0]
        self.ccd = ccd

    def mask(self, x):
        if self.ccd:
            x = x.copy()
            x[: self.o * self.v] = 0.0
        return x

    def amplitude_space(self, x):
        """Orthogonal projection onto the space the unknowns live in: doubles
        with t_ij^ab = t_ji^ba (closed-shell amplitudes; the residual has the
        same symmetry), and zero singles at the CCD level. Every vector the
        solvers build from such amplitudes lies in it in exact arithmetic;
        the projection removes what rounding leaves outside it, where the
        Jacobian of the equations as written is not that of any amplitude
        (left in, it makes the Newton tail linear on hard problems)."""
        return self.mask(pair_symmetrize(x, self.o, self.v))

    def residual(self, x):
        return self.mask(pack(*ccsd.residual(self.f_oo, self.f_ov, self.f_vv, self.L, *unpack(x, self.o, self.v))))

    def jvp(self, x, q, mode="complex", r=None, delta=None):
        t1, t2 = unpack(x, self.o, self.v)
        v1, v2 = unpack(q, self.o, self.v)
        if mode == "complex":
            return self.mask(pack(*ccsd.jvp_complex_step(self.f_oo, self.f_ov, self.f_vv, self.L, t1, t2, v1, v2)))
        # forward difference (the paper's form), r = r(x) given
        p = self.residual(x + delta * q)
        return (p - r) / delta

    def energy(self, x):
        return float(ccsd.energy(self.f_oo, self.f_ov, self.f_vv, self.L, *unpack(x, self.o, self.v)))

    def precond(self, b, rtol, maxit, restart, info):
        # A_F has no doubles <- singles coupling (its doubles rows involve x2
        # only), so for b1 = 0 the doubles of A_F^-1 b are A_dd^-1 b2: the
        # CCD preconditioner once the singles are dropped
        res = gmres(lambda y: pack(*fock_apply(self.f_oo, self.f_ov, self.f_vv, *unpack(y, self.o, self.v))),
                    b, rtol=rtol, maxit=maxit, restart=restart)
        info.n_afmv += res.iters
        info.n_inner_iters += res.iters
        return self.amplitude_space(res.x)


def _make_problem(f_oo, f_ov, f_vv, L, ccd, gauge):
    if gauge is None:
        return _Problem(f_oo, f_ov, f_vv, L, ccd)
    from .gauge import GaugeProblem
    return GaugeProblem(f_oo, f_ov, f_vv, L, gauge[0], gauge[1], ccd)


def mp2_guess(f_oo, f_ov, f_vv, L, inner_rtol=1e-12, inner_maxit=200, inner_restart=30):
    """theta^0 = -A_F^{-1} r(0): the generalized MP2 amplitudes
    (equation inexact_newton_update at t = 0)."""
    P = _Problem(f_oo, f_ov, f_vv, L)
    info = SolveInfo()
    r0 = P.residual(np.zeros(P.o * P.v + P.o ** 2 * P.v ** 2))
    return -P.precond(r0, inner_rtol, inner_maxit, inner_restart, info)


def forcing_term(k, rn, rn_prev, eta_prev, tol, gamma=0.9, alpha=1.5,
                 eta0=0.5, eta_max=0.9):
    """Eisenstat-Walker forcing term (choice 2) with its safeguards."""
    if k == 0:
        eta = eta0
    else:
        eta = gamma * (rn / rn_prev) ** alpha
        sg = gamma * eta_prev ** alpha
        if sg > 0.1:
            eta = max(eta, sg)
    eta = min(eta, eta_max)
    eta = max(eta, 0.5 * tol / rn)
    return min(eta, eta_max)


def solve_pnk(f_oo, f_ov, f_vv, L, tol=1e-8, max_newton=100, m_max=20,
              gamma=0.9, alpha=1.5, eta0=0.5, eta_max=0.9, inner_rtol=1e-12,
              inner_maxit=200, inner_restart=30, jvp="complex", x0=None,
              precond=True, ccd=False, gauge=None):
    """PNK (precond=True) or unpreconditioned NK (precond=False), Algorithm 1
    and the method table; ccd=True at the CCD level (see _Problem).
    gauge=(W_o, W_v) iterates on the amplitudes of that non-orthogonal gauge
    (oracle.gauge) and returns them."""
    t_start = time.perf_counter()
    P = _make_problem(f_oo, f_ov, f_vv, L, ccd, gauge)
    info = SolveInfo()
    N = P.o * P.v + P.o ** 2 * P.v ** 2

    def Ainv(b):
        if not precond:
            # NK: no preconditioner, the identity on the amplitude space
            return P.amplitude_space(b)
        return P.precond(b, inner_rtol, inner_maxit, inner_restart, info)

    if x0 is None:
        # MP2-type start for every protocol (the numerics section uses it in
        # all examples): -A_F^-1 r(0), also for NK
        r0 = P.residual(np.zeros(N))
        info.n_residual += 1
        x = -P.precond(r0, inner_rtol, inner_maxit, inner_restart, info)
    else:
        x = P.mask(x0)
    rn_prev = None
    eta = eta0
    k = 0
    while True:
        r = P.residual(x)
        info.n_residual += 1
        rinf = float(np.max(np.abs(r)))
        rn = float(np.linalg.norm(r))
        info.history.append((info.n_residual + info.n_jvp, rn, rinf))
        info.res_inf, info.res_2 = rinf, rn
        if not np.isfinite(rn):
            break
        if rinf < tol:
            info.converged = True
            break
        if k >= max_newton:
            break
        eta = forcing_term(k, rn, rn_prev, eta, tol, gamma, alpha, eta0, eta_max)
        z = Ainv(r)
        beta = float(np.linalg.norm(z))
        Q = [z / beta]
        H = np.zeros((m_max + 1, m_max))
        cs = np.zeros(m_max)
        sn = np.zeros(m_max)
        g = np.zeros(m_max + 1)
        g[0] = beta
        m_done = 0
        delta = None
        if jvp == "fd":
            delta = np.sqrt(np.finfo(float).eps) * (1.0 + np.linalg.norm(x))
        for m in range(m_max):
            w = Ainv(P.jvp(x, Q[m], jvp, r=r, delta=delta))
            info.n_jvp += 1
            for i in range(m + 1):
                H[i, m] = np.dot(Q[i], w)
                w = w - H[i, m] * Q[i]
            hnext = float(np.linalg.norm(w))
            H[m + 1, m] = hnext
            for i in range(m):
                a, c = H[i, m], H[i + 1, m]
                H[i, m] = cs[i] * a + sn[i] * c
                H[i + 1, m] = -sn[i] * a + cs[i] * c
            rho = np.hypot(H[m, m], H[m + 1, m])
            cs[m] = H[m, m] / rho
            sn[m] = H[m + 1, m] / rho
            H[m, m] = rho
            H[m + 1, m] = 0.0
            g[m + 1] = -sn[m] * g[m]
            g[m] = cs[m] * g[m]
            m_done = m + 1
            if abs(g[m + 1]) <= eta * beta or hnext <= 1e-14 * beta:
                break
            if m + 1 < m_max:
                Q.append(w / hnext)
        y = np.linalg.solve(np.triu(H[:m_done, :m_done]), g[:m_done])
        for i in range(m_done):
            x = x - y[i] * Q[i]
        rn_prev = rn
        k += 1
    info.newton_iters = k
    info.e_corr = P.energy(x)
    info.seconds = time.perf_counter() - t_start
    t1, t2 = unpack(x, P.o, P.v)
    return t1.copy(), t2.copy(), info


def jacobi_denominators(f_oo, f_vv, shift=0.0):
    """D_i^a = f_aa - f_ii + s and D_ij^ab = f_aa + f_bb - f_ii - f_jj + s,
    from the diagonal of the Fock matrix in the current gauge."""
    fo = np.diag(f_oo)
    fv = np.diag(f_vv)
    d1 = fv[None, :] - fo[:, None] + shift
    d2 = (fv[None, None, :, None] + fv[None, None, None, :]
          - fo[:, None, None, None] - fo[None, :, None, None] + shift)
    return d1, d2


def solve_fp_diis(f_oo, f_ov, f_vv, L, tol=1e-8, max_iter=500, diis_size=8,
                  diis_start=2, level_shift=0.0, x0=None, init="mp2",
                  inner_rtol=1e-12, diverge=1e6, ccd=False, gauge=None):
    """(S)FP iteration t <- t - r(t)/D with DIIS over the last `diis_size`
    (amplitude, Jacobi step) pairs; diis_size = 0 disables DIIS; ccd=True at
    the CCD level (see _Problem). gauge=(W_o, W_v): the iteration on the
    amplitudes of that gauge, D from the diagonals of its Fock blocks (the
    random-gauge FP update)."""
    t_start = time.perf_counter()
    P = _make_problem(f_oo, f_ov, f_vv, L, ccd, gauge)
    info = SolveInfo()
    N = P.o * P.v + P.o ** 2 * P.v ** 2
    if gauge is not None:
        d1, d2 = jacobi_denominators(P.Fo, P.Fv, level_shift)
    else:
        d1, d2 = jacobi_denominators(f_oo, f_vv, level_shift)
    D = pack(d1, d2)
    if x0 is not None:
        x = P.mask(x0)
    elif init == "mp2":
        r0 = P.residual(np.zeros(N))
        info.n_residual += 1
        x = -P.precond(r0, inner_rtol, 200, 30, info)
    else:
        x = np.zeros(N)
    hist_x, hist_e = [], []
    it = 0
    while True:
        r = P.residual(x)
        info.n_residual += 1
        rinf = float(np.max(np.abs(r)))
        rn = float(np.linalg.norm(r))
        info.history.append((info.n_residual, rn, rinf))
        info.res_inf, info.res_2 = rinf, rn
        if not np.isfinite(rn) or rn > diverge:
            break
        if rinf < tol:
            info.converged = True
            break
        if it >= max_iter:
            break
        e = -r / D
        xn = x + e
        if diis_size > 0:
            hist_x.append(xn)
            hist_e.append(e)
            if len(hist_x) > diis_size:
                hist_x.pop(0)
                hist_e.pop(0)
            if it + 1 >= diis_start and len(hist_x) >= 2:
                m = len(hist_x)
                B = -np.ones((m + 1, m + 1))
                B[m, m] = 0.0
                for a_ in range(m):
                    for b_ in range(m):
                        B[a_, b_] = np.dot(hist_e[a_], hist_e[b_])
                rhs = np.zeros(m + 1)
                rhs[m] = -1.0
                c = np.linalg.lstsq(B, rhs, rcond=None)[0][:m]
                xn = sum(ci * xi for ci, xi in zip(c, hist_x))
        x = xn
        it += 1
    info.newton_iters = it
    info.e_corr = P.energy(x)
    info.seconds = time.perf_counter() - t_start
    t1, t2 = unpack(x, P.o, P.v)
    return t1.copy(), t2.copy(), info


def solve_ink(f_oo, f_ov, f_vv, L, tol=1e-8, max_iter=200, inner_rtol=1e-12,
              inner_maxit=200, inner_restart=30, x0=None, ccd=False, diverge=1e6, gauge=None):
    """INK (method table): the Newton update with A_F in place of the
    Jacobian, A_F dt = -r(t) (equation inexact_newton_update), solved by
    GMRES; t <- t + dt until ||r||_inf < tol. Starts from the MP2 amplitudes
    -A_F^-1 r(0) unless x0 is given. In the canonical gauge A_F is the
    diagonal of orbital-energy differences and INK is the plain FP
    iteration. gauge=(W_o, W_v) iterates on the amplitudes of that gauge
    with its A_F."""
    t_start = time.perf_counter()
    P = _make_problem(f_oo, f_ov, f_vv, L, ccd, gauge)
    info = SolveInfo()
    N = P.o * P.v + P.o ** 2 * P.v ** 2
    if x0 is not None:
        x = P.mask(x0)
    else:
        r0 = P.residual(np.zeros(N))
        info.n_residual += 1
        x = -P.precond(r0, inner_rtol, inner_maxit, inner_restart, info)
    it = 0
    while True:
        r = P.residual(x)
        info.n_residual += 1
        rinf = float(np.max(np.abs(r)))
        rn = float(np.linalg.norm(r))
        info.history.append((info.n_residual, rn, rinf))
        info.res_inf, info.res_2 = rinf, rn
        if not np.isfinite(rn) or rn > diverge:
            break
        if rinf < tol:
            info.converged = True
            break
        if it >= max_iter:
            break
        x = x - P.precond(r, inner_rtol, inner_maxit, inner_restart, info)
        it += 1
    info.newton_iters = it
    info.e_corr = P.energy(x)
    info.seconds = time.perf_counter() - t_start
    t1, t2 = unpack(x, P.o, P.v)
    return t1.copy(), t2.copy(), info


def pair_symmetrize(x, o, v):
    """Orthogonal projection onto pair-symmetric vectors: doubles
    (x_ij^ab + x_ji^ba) / 2, singles unchanged."""
    x1, x2 = unpack(x, o, v)
    return pack(x1, 0.5 * (x2 + np.transpose(x2, (1, 0, 3, 2))))


def fp_jacobian_spectral_radius(f_oo, f_ov, f_vv, L, t1, t2, shift=0.0, m=30, seed=0, ccd=False, q0=None):
    """Spectral radius of the Jacobian G = I - diag(D + shift)^-1 J(t) of the
    (S)FP map t -> t - r(t) / (D + shift) at t, with D the Jacobi
    denominators of the current gauge (Section "Regularization" ties FP's
    convergence to this radius being below one; Appendix D, the shift as a
    Ridge term). G acts on pair-symmetric vectors (the amplitude space; the
    projection is applied after every product). Arnoldi with modified
    Gram-Schmidt for m steps from q0 (projected), else a seeded
    pair-symmetric start; returns the
    largest modulus of the Ritz values (exact once the Krylov space is
    invariant) and the Ritz values."""
    P = _Problem(f_oo, f_ov, f_vv, L, ccd)
    o, v = P.o, P.v
    x = pack(t1, t2)
    d1, d2 = jacobi_denominators(f_oo, f_vv, shift)
    D = pack(d1, d2)
    if q0 is None:
        q0 = np.random.default_rng(seed).standard_normal(x.size)
    q = P.mask(pair_symmetrize(np.asarray(q0, dtype=float), o, v))
    Q = [q / np.linalg.norm(q)]
    H = np.zeros((m + 1, m))
    k = 0
    for k in range(m):
        w = Q[k] - P.jvp(x, Q[k]) / D
        w = P.mask(pair_symmetrize(w, o, v))
        for i in range(k + 1):
            H[i, k] = np.dot(Q[i], w)
            w = w - H[i, k] * Q[i]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] <= 1e-12 * max(1.0, abs(H[k, k])):
            k += 1
            break
        Q.append(w / H[k + 1, k])
    else:
        k = m
    ritz = np.linalg.eigvals(H[:k, :k])
    return float(np.max(np.abs(ritz))), ritz
