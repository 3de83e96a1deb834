"""Amplitude equations in a non-orthogonal orbital gauge.

TEST INFRASTRUCTURE ONLY. Part of the CPU float64 oracle; only the tests,
the smoke check and the benchmark's CPU baseline may import it.

Source: Appendix A, "Random gauge representation" (the transformed
amplitudes theta, the projectors P, Q, P-bar, Q-bar, the transformed
integrals pi, A, B, X, Y, the Fock blocks oF, vF and the random-gauge CCD
residual with its FP update).

The gauge. Within each orbital block, gauge functions that span the same
space as the orthonormal orbitals phi but need not be orthonormal:
chi_occ = phi_occ W_o and chi_vir = phi_vir W_v, with W_o (o x m_o) and W_v
(v x m_v) of full row rank. They overlap as S = W^T W. With m = o (v) and W
invertible the gauge is non-redundant; with m > o (v) it is redundant (more
functions than the space they span, as projected atomic orbitals are) and S
is singular. In the appendix's notation the gauge functions are the basis,
the orbital coefficients in it are C = W^+ = W^T (W W^T)^{-1} (so W C = 1 and
C^T S C = 1; W^+ = W^{-1} when W is square), the gauge map is U = C and
U-bar = S U = W^T, and the appendix's projector onto the gauge space is
Pi = U-bar C^T = W^T (W W^T)^{-1} W per block: the orthogonal projector, in
gauge-index space, onto the range of U-bar. For a redundant gauge only that
range holds amplitudes: theta and r(theta) lie in it, components outside it
do not change t(theta), and the Jacobian of r(theta) is singular there.

* Amplitudes: theta = U-bar^(x4) t, i.e.
  theta[mu, nu, lam, sig] = sum W[i, mu] W[j, nu] W[a, lam] W[b, sig] t[i, j, a, b]
  (covariant components); singles theta1 = W_o^T t1 W_v.
* Residual: the first line of the random-gauge residual equation,
  r(theta) = U-bar^(x4) r(t) with t the back-transform of theta
  (t = C^(x4) theta, C = W^+). `residual` is that definition.
  `residual_ccd_explicit` writes the same CCD residual out in the gauge
  quantities of the appendix (Y + A theta + theta B + theta pi theta + the
  symmetrised Fock, J and K terms), so the two pin each other.
* Fock blocks: the one-body part of the residual acts on a virtual index
  of theta through Fv = W_v^T f_vv C_v^T and on an occupied index
  through Fo = W_o^T f_oo C_o^T (m x m; W^T f W^{-T} for a square gauge). Reading: the appendix's f-bar is the
  Fock matrix in the gauge basis, <chi|f|chi> = W^T f W, which the
  projector products Q-bar f-bar Q and P-bar f-bar P turn into these
  similarity transforms. (The printed f-bar = U f U^T with U = C agrees
  with this only for orthogonal W.)
* A_F in the gauge: the Kronecker sum of Fv over the virtual indices and
  -Fo over the occupied ones, i.e. U-bar^(x4) A_F C^(x4); not symmetric
  when W is not orthogonal.
* FP in the gauge: the Jacobi step with the diagonals of Fo and Fv (the
  appendix's Delta).

Readings where the appendix is garbled (index placement of pi in the
quadratic terms; J-bar lacks one of the two t.pi terms; K-bar repeats an
index): the explicit form below follows the corrected MO equations of
oracle.ccsd term by term, each MO contraction becoming a contraction of a
covariant with a contravariant gauge index.
"""

from __future__ import annotations

import numpy as np

from . import ccsd
from .solvers import _Problem, gmres, pack, unpack


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def forward(Wo, Wv, x1, x2):
    """theta = U-bar^(x4) x: singles W_o^T x1 W_v, doubles on all four
    indices (the transformed amplitudes and residuals)."""
    y1 = _es("iM,aL,ia->ML", Wo, Wv, x1)
    y2 = _es("iM,jN,aL,bS,ijab->MNLS", Wo, Wo, Wv, Wv, x2)
    return y1, y2


def coefficients(W):
    """C = W^+ = W^T (W W^T)^{-1} (m x n): the orbital coefficients of a
    block in its gauge functions; W^{-1} when W is square and invertible."""
    return W.T @ np.linalg.inv(W @ W.T)


def projector(W):
    """Pi = W^T (W W^T)^{-1} W (m x m): projector onto the range of
    U-bar = W^T, the gauge-index space amplitudes live in (the identity for
    a non-redundant gauge)."""
    return W.T @ np.linalg.inv(W @ W.T) @ W


def backward(Wo, Wv, y1, y2):
    """x = C^(x4) y with C = W^+: the orbital amplitudes of gauge
    amplitudes y (the inverse of `forward` on its range)."""
    Co = coefficients(Wo)
    Cv = coefficients(Wv)
    x1 = _es("Mi,La,ML->ia", Co, Cv, y1)
    x2 = _es("Mi,Nj,La,Sb,MNLS->ijab", Co, Co, Cv, Cv, y2)
    return x1, x2


def fock_blocks(f_oo, f_vv, Wo, Wv):
    """(Fo, Fv): the gauge's occupied and virtual Fock blocks,
    W^T f C^T per block (m x m; W^T f W^{-T} when W is square)."""
    Fo = Wo.T @ f_oo @ coefficients(Wo).T
    Fv = Wv.T @ f_vv @ coefficients(Wv).T
    return Fo, Fv


def residual(f_oo, f_ov, f_vv, L, Wo, Wv, th1, th2):
    """r(theta) = U-bar^(x4) r(t(theta)) (the definition)."""
    t1, t2 = backward(Wo, Wv, th1, th2)
    r1, r2 = ccsd.residual(f_oo, f_ov, f_vv, L, t1, t2)
    return forward(Wo, Wv, r1, r2)


def energy(f_oo, f_ov, f_vv, L, Wo, Wv, th1, th2):
    """The correlation energy is gauge invariant: E(t(theta))."""
    t1, t2 = backward(Wo, Wv, th1, th2)
    return ccsd.energy(f_oo, f_ov, f_vv, L, t1, t2)


def jvp_complex_step(f_oo, f_ov, f_vv, L, Wo, Wv, th1, th2, v1, v2, h=1e-30):
    """J(theta) v by the complex step (exact to rounding)."""
    r1, r2 = residual(f_oo, f_ov, f_vv, L, Wo, Wv, th1 + 1j * h * v1, th2 + 1j * h * v2)
    return r1.imag / h, r2.imag / h


def fock_apply(f_ov, Wo, Wv, Fo, Fv, x1, x2):
    """A_F in the gauge applied to x = (x1, x2): Fv on each virtual index,
    -Fo on each occupied index; the singles couple to the doubles through
    f_ov as in the orbital basis (transformed along)."""
    y2 = (_es("ac,ijcb->ijab", Fv, x2)
          + _es("bc,ijac->ijab", Fv, x2)
          - _es("ik,kjab->ijab", Fo, x2)
          - _es("jk,ikab->ijab", Fo, x2))
    y1 = _es("ac,ic->ia", Fv, x1) - _es("ik,ka->ia", Fo, x1)
    if np.any(f_ov != 0.0):
        _, t2 = backward(Wo, Wv, np.zeros_like(x1), x2)
        c1 = _es("kc,ikac->ia", f_ov, 2.0 * t2 - np.transpose(t2, (0, 1, 3, 2)))
        y1 = y1 + forward(Wo, Wv, c1, np.zeros_like(t2))[0]
    return y1, y2


def residual_ccd_explicit(f_oo, f_vv, L, Wo, Wv, th2):
    """The random-gauge CCD residual (t1 = 0) written out in the appendix's
    gauge quantities; doubles only. Covariant gauge indices come from
    W^T (U-bar), contravariant ones from C = W^+."""
    o = f_oo.shape[0]
    # contravariant gauge indices: C = W^+, [gauge][orbital]
    Co = coefficients(Wo)
    Cv = coefficients(Wv)
    Loo, Lov, Lvv = L[:, :o, :o], L[:, :o, o:], L[:, o:, o:]
    Lvo = L[:, o:, :o]
    ovov = _es("Pia,Pjb->iajb", Lov, Lov)
    oooo = _es("Pki,Plj->kilj", Loo, Loo)
    vvvv = _es("Pac,Pbd->acbd", Lvv, Lvv)
    voov = _es("Pai,Pkc->aikc", Lvo, Lov)
    oovv = _es("Pki,Pac->kiac", Loo, Lvv)
    th = th2
    Th = 2.0 * th - np.transpose(th, (0, 1, 3, 2))
    # transformed integrals (Y, A, B all-covariant / mixed; pi contravariant)
    Y = _es("iM,jN,aL,bS,iajb->MNLS", Wo, Wo, Wv, Wv, ovov)
    A = _es("iM,jN,Ak,Bl,kilj->MNAB", Wo, Wo, Co, Co, oooo)
    B = _es("Ac,Bd,aL,bS,acbd->ABLS", Cv, Cv, Wv, Wv, vvvv)
    pi = _es("Gk,Dl,Ac,Bd,kcld->GDAB", Co, Co, Cv, Cv, ovov)  # (kc|ld) as [k][l][c][d]
    X_J = _es("aL,iM,Ak,Gc,aikc->LMAG", Wv, Wo, Co, Cv, voov)
    X_K = _es("Ak,iM,aL,Gc,kiac->AMLG", Co, Wo, Wv, Cv, oovv)
    Fo, Fv = fock_blocks(f_oo, f_vv, Wo, Wv)
    vG = Fv - _es("GDLB,GDAB->LA", Th, pi)
    oG = Fo + _es("MBGD,ABGD->MA", Th, pi)
    Jb = X_J + 0.5 * _es("ABGD,MBLD->LMAG", pi, Th) - 0.5 * _es("ABDG,MBLD->LMAG", pi, th)
    Kb = X_K - 0.5 * _es("ABDG,MBDL->AMLG", pi, th)
    r = (Y
         + _es("MNAB,ABLS->MNLS", A, th)
         + _es("MNAB,ABLS->MNLS", th, B)
         + _es("MNAB,GDAB,GDLS->MNLS", th, pi, th))
    x = (_es("SA,MNLA->MNLS", vG, th)
         - _es("NA,MALS->MNLS", oG, th)
         + _es("LMAG,NASG->MNLS", Jb, Th)
         - _es("AMLG,ANGS->MNLS", Kb, th)
         - _es("AMSG,ANLG->MNLS", Kb, th))
    return r + x + np.transpose(x, (1, 0, 3, 2))


class GaugeProblem(_Problem):
    """The solvers' maps on gauge amplitudes theta: the residual and its
    Jacobian by the definition above, A_F in the gauge (GMRES, since it is
    not symmetric), the energy of t(theta)."""

    def __init__(self, f_oo, f_ov, f_vv, L, Wo, Wv, ccd=False):
        super().__init__(f_oo, f_ov, f_vv, L, ccd)
        self.Wo, self.Wv = Wo, Wv
        self.Fo, self.Fv = fock_blocks(f_oo, f_vv, Wo, Wv)
        # vectors are gauge vectors: m_o gauge functions for the occupied
        # block, m_v for the virtual one
        self.o, self.v = Wo.shape[1], Wv.shape[1]

    def residual(self, x):
        th1, th2 = unpack(x, self.o, self.v)
        return self.mask(pack(*residual(self.f_oo, self.f_ov, self.f_vv, self.L, self.Wo, self.Wv, th1, th2)))

    def jvp(self, x, q, mode="complex", r=None, delta=None):
        if mode != "complex":
            return super().jvp(x, q, mode, r, delta)
        th1, th2 = unpack(x, self.o, self.v)
        v1, v2 = unpack(q, self.o, self.v)
        return self.mask(pack(*jvp_complex_step(self.f_oo, self.f_ov, self.f_vv, self.L, self.Wo, self.Wv,
                                                th1, th2, v1, v2)))

    def energy(self, x):
        th1, th2 = unpack(x, self.o, self.v)
        return float(energy(self.f_oo, self.f_ov, self.f_vv, self.L, self.Wo, self.Wv, th1, th2))

    def precond(self, b, rtol, maxit, restart, info):
        res = gmres(lambda y: pack(*fock_apply(self.f_ov, self.Wo, self.Wv, self.Fo, self.Fv,
                                                *unpack(y, self.o, self.v))),
                    b, rtol=rtol, maxit=maxit, restart=restart)
        info.n_afmv += res.iters
        info.n_inner_iters += res.iters
        # gauge amplitudes keep the pair symmetry: the same W maps i and j,
        # and a and b
        return self.amplitude_space(res.x)
