"""Closed-shell CCSD residual and energy from density-fitted integrals.

TEST INFRASTRUCTURE ONLY. This is the CPU float64 oracle that the GPU path
is checked against. Only the tests, the smoke check and the benchmark's CPU
baseline may import it; the product path never does.

What is computed (Section "Theory", equations CC_ampl and CC_energy): the
projected amplitude equations r_mu(t) = <Phi_mu| e^{-T} H e^{T} |Phi_0> = 0
over all singles and doubles and the energy <Phi_0| e^{-T} H e^{T} |Phi_0>.
The paper writes them out only at the CCD level (Appendix A, "Molecular
orbital representation"); singles are added here through the
T1-similarity-transformed Hamiltonian (Koch et al., J. Chem. Phys. 100
(1994) 4393): with T1 folded into H the doubles keep the CCD form, built
from dressed integrals. Readings of the paper's garbled CCD intermediates:

* g_c^a: the omega.t term enters with a minus sign (it does in the
  random-gauge form of the same appendix);
* K: the (1/2) v.t term enters with a minus sign (likewise);
* K_{kc}^{ka} in the residual is read as K_{ic}^{ka} (and ^{kb}).

Every formula below is pinned by the brute-force determinant-space
evaluation in oracle.brute (same definition, no shared code).

Conventions. Indices i,j,k,l occupied (0..o-1), a,b,c,d virtual. Chemists'
integrals (pq|rs) = sum_P L[P,p,q] L[P,r,s]. Amplitudes
T = sum t1[i,a] E_ai + 1/2 sum t2[i,j,a,b] E_ai E_bj with E_pq the spin-summed
excitation operator and t2[i,j,a,b] = t2[j,i,b,a]. Residual components are
the projections onto a+_{a alpha} a_{i alpha} |Phi_0> and
a+_{a alpha} a_{i alpha} a+_{b beta} a_{j beta} |Phi_0>.

All functions accept complex arrays and use no conjugation, so a
complex-step derivative of the residual is exact to rounding.
"""

from __future__ import annotations

import numpy as np


def _es(spec, *ops):
    return np.einsum(spec, *ops, optimize=True)


def fock_matrix(f_oo, f_ov, f_vv):
    o, v = f_oo.shape[0], f_vv.shape[0]
    f = np.zeros((o + v, o + v), dtype=np.result_type(f_oo, f_ov, f_vv))
    f[:o, :o] = f_oo
    f[:o, o:] = f_ov
    f[o:, :o] = f_ov.T
    f[o:, o:] = f_vv
    return f


def two_electron_fock(L, nocc):
    """G[L]_pq = sum_k 2 (pq|kk) - (pk|kq), the closed-shell mean field of
    the doubly occupied orbitals 0..nocc-1."""
    o = nocc
    d = _es("Pkk->P", L[:, :o, :o])
    coul = 2.0 * _es("Ppq,P->pq", L, d)
    exch = _es("Ppk,Pkq->pq", L[:, :, :o], L[:, :o, :])
    return coul - exch


def core_hamiltonian(f, L, nocc):
    """One-electron operator h with f = h + G[L]."""
    return f - two_electron_fock(L, nocc)


def t1_similarity(nocc, t1):
    """(1 - tau, 1 + tau) with tau[o+a, i] = t1[i, a]: e^{-T1} E_pq e^{T1}
    = sum_rs (1-tau)_{rp} (1+tau)_{qs} E_rs, so every one-index quantity X
    dresses as (1 - tau) X (1 + tau)."""
    o, v = t1.shape
    n = o + v
    tau = np.zeros((n, n), dtype=t1.dtype)
    tau[o:, :o] = t1.T
    eye = np.eye(n, dtype=t1.dtype)
    return eye - tau, eye + tau


def dress(X, nocc, t1):
    """(1 - tau) X (1 + tau) for an n x n matrix or a stack [P][n][n]."""
    left, right = t1_similarity(nocc, t1)
    if X.ndim == 2:
        return left @ X @ right
    return _es("rp,Ppq,qs->Prs", left, X, right)


def dressed_quantities(f_oo, f_ov, f_vv, L, t1):
    """Dressed DF factors Lt and the dressed Fock matrix Ft (n x n)."""
    o = f_oo.shape[0]
    f = fock_matrix(f_oo, f_ov, f_vv)
    h = core_hamiltonian(f, L, o)
    Lt = dress(L, o, t1)
    ht = dress(h, o, t1)
    Ft = ht + two_electron_fock(Lt, o)
    return Lt, Ft


def residual(f_oo, f_ov, f_vv, L, t1, t2):
    """CCSD residual (r1 [o][v], r2 [o][o][v][v]) at amplitudes (t1, t2)."""
    o = f_oo.shape[0]
    Lt, Ft = dressed_quantities(f_oo, f_ov, f_vv, L, t1)
    Loo = Lt[:, :o, :o]   # [P,k,i]  creator index first
    Lov = Lt[:, :o, o:]   # [P,k,c]  (equal to the undressed block)
    Lvo = Lt[:, o:, :o]   # [P,a,i]
    Lvv = Lt[:, o:, o:]   # [P,a,c]
    F_oo = Ft[:o, :o]
    F_ov = Ft[:o, o:]
    F_vo = Ft[o:, :o]
    F_vv = Ft[o:, o:]

    # dressed integral blocks (pq|rs)~ = sum_P Lt[P,p,q] Lt[P,r,s]
    aibj = _es("Pai,Pbj->aibj", Lvo, Lvo)
    acbd = _es("Pac,Pbd->acbd", Lvv, Lvv)
    kilj = _es("Pki,Plj->kilj", Loo, Loo)
    kcld = _es("Pkc,Pld->kcld", Lov, Lov)
    aikc = _es("Pai,Pkc->aikc", Lvo, Lov)
    kiac = _es("Pki,Pac->kiac", Loo, Lvv)
    ackd = _es("Pac,Pkd->ackd", Lvv, Lov)
    kilc = _es("Pki,Plc->kilc", Loo, Lov)

    u = 2.0 * t2 - np.transpose(t2, (0, 1, 3, 2))

    # singles
    r1 = (F_vo.T
          + _es("ackd,ikcd->ia", ackd, u)
          - _es("kilc,klac->ia", kilc, u)
          + _es("kc,ikac->ia", F_ov, u))

    # doubles intermediates
    W = kilj.transpose(0, 2, 1, 3) + _es("kcld,ijcd->klij", kcld, t2)  # W[k,l,i,j]
    Gv = F_vv - _es("kcld,klbd->bc", kcld, u)
    Go = F_oo + _es("kcld,jlcd->kj", kcld, u)
    J = (aikc + 0.5 * _es("kcld,ilad->aikc", kcld, u)
         - 0.5 * _es("kdlc,ilad->aikc", kcld, t2))
    K = kiac - 0.5 * _es("kdlc,ilda->kiac", kcld, t2)

    r2 = (np.transpose(aibj, (1, 3, 0, 2))
          + _es("acbd,ijcd->ijab", acbd, t2)
          + _es("klij,klab->ijab", W, t2))
    x = (_es("bc,ijac->ijab", Gv, t2)
         - _es("kj,ikab->ijab", Go, t2)
         + _es("aikc,jkbc->ijab", J, u)
         - _es("kiac,kjcb->ijab", K, t2)
         - _es("kibc,kjac->ijab", K, t2))
    r2 = r2 + x + np.transpose(x, (1, 0, 3, 2))
    return r1, r2


def energy(f_oo, f_ov, f_vv, L, t1, t2):
    """Correlation energy E_CC - E_ref at (t1, t2)."""
    o = f_oo.shape[0]
    Lov = L[:, :o, o:]
    iajb = _es("Pia,Pjb->iajb", Lov, Lov)
    tau = t2 + _es("ia,jb->ijab", t1, t1)
    return (2.0 * _es("ia,ia->", f_ov, t1)
            + _es("iajb,ijab->", iajb, 2.0 * tau - np.transpose(tau, (0, 1, 3, 2))))


def jvp_complex_step(f_oo, f_ov, f_vv, L, t1, t2, v1, v2, h=1e-30):
    """J(t) v = Im r(t + i h v) / h (Squire & Trapp, SIAM Rev. 40 (1998)
    110): the directional derivative to rounding, since r is a polynomial
    evaluated without conjugation."""
    r1, r2 = residual(f_oo, f_ov, f_vv, L, t1 + 1j * h * v1, t2 + 1j * h * v2)
    return r1.imag / h, r2.imag / h


def jvp_central(f_oo, f_ov, f_vv, L, t1, t2, v1, v2, h=None):
    """Central difference [r(t + h v) - r(t - h v)] / (2 h)."""
    if h is None:
        nv = np.sqrt(np.vdot(v1, v1).real + np.vdot(v2, v2).real)
        nt = np.sqrt(np.vdot(t1, t1).real + np.vdot(t2, t2).real)
        h = 1e-5 * max(1.0, nt) / max(nv, 1e-300)
    p1, p2 = residual(f_oo, f_ov, f_vv, L, t1 + h * v1, t2 + h * v2)
    m1, m2 = residual(f_oo, f_ov, f_vv, L, t1 - h * v1, t2 - h * v2)
    return (p1 - m1) / (2 * h), (p2 - m2) / (2 * h)


def jvp_forward(f_oo, f_ov, f_vv, L, t1, t2, v1, v2, delta):
    """Forward difference of Eq. jacobian_vector_product_via_finite_difference."""
    p1, p2 = residual(f_oo, f_ov, f_vv, L, t1 + delta * v1, t2 + delta * v2)
    r1, r2 = residual(f_oo, f_ov, f_vv, L, t1, t2)
    return (p1 - r1) / delta, (p2 - r2) / delta
