"""Brute-force coupled-cluster quantities in the space of Slater determinants.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle; never imported by the
product path).

This evaluates the definitions of equations CC_ampl and CC_energy (Section
"Theory") literally for tiny systems: all determinants with `nocc` alpha and
`nocc` beta electrons in n spatial orbitals are enumerated, the spin-summed
excitation operators E_pq are built as matrices with Jordan-Wigner signs,
H, T, e^{+-T} are formed from them (T is nilpotent, so the exponential is a
finite Taylor sum), and the residual is read off as the overlap of
e^{-T} H e^{T} |Phi_0> with the excited determinants X_mu |Phi_0>. It shares
no formula with oracle.ccsd: agreement pins the working equations there.
"""

from __future__ import annotations

from itertools import combinations

import numpy as np


def _bits(occ):
    s = 0
    for p in occ:
        s |= 1 << p
    return s


def _apply_excitation(string, p, q):
    """a+_p a_q on one spin string (bit mask). Returns (sign, new) or None."""
    if not (string >> q) & 1:
        return None
    sign = -1.0 if bin(string & ((1 << q) - 1)).count("1") % 2 else 1.0
    s = string & ~(1 << q)
    if (s >> p) & 1:
        return None
    sign *= -1.0 if bin(s & ((1 << p) - 1)).count("1") % 2 else 1.0
    return sign, s | (1 << p)


class DeterminantSpace:
    """Determinants |alpha string, beta string> with nocc electrons of each
    spin in n orbitals. Orbitals 0..nocc-1 are occupied in Phi_0."""

    def __init__(self, n, nocc):
        self.n = n
        self.nocc = nocc
        strings = [_bits(c) for c in combinations(range(n), nocc)]
        self.dets = [(a, b) for a in strings for b in strings]
        self.index = {d: k for k, d in enumerate(self.dets)}
        self.dim = len(self.dets)
        ref = _bits(range(nocc))
        self.ref = np.zeros(self.dim)
        self.ref[self.index[(ref, ref)]] = 1.0
        self.Ea = [[self._spin_op(p, q, 0) for q in range(n)] for p in range(n)]
        self.Eb = [[self._spin_op(p, q, 1) for q in range(n)] for p in range(n)]
        self.E = [[self.Ea[p][q] + self.Eb[p][q] for q in range(n)] for p in range(n)]

    def _spin_op(self, p, q, spin):
        # Jordan-Wigner order: all alpha orbitals, then all beta orbitals.
        # a+_{p beta} a_{q beta} passes every alpha electron twice, so only
        # the beta string contributes to the sign.
        M = np.zeros((self.dim, self.dim))
        for col, (a, b) in enumerate(self.dets):
            s = a if spin == 0 else b
            r = _apply_excitation(s, p, q)
            if r is None:
                continue
            sign, s2 = r
            row = self.index[(s2, b) if spin == 0 else (a, s2)]
            M[row, col] += sign
        return M

    def hamiltonian(self, h, eri):
        """H = sum h_pq E_pq + 1/2 sum (pq|rs) (E_pq E_rs - delta_qr E_ps)."""
        n = self.n
        H = np.zeros((self.dim, self.dim))
        for p in range(n):
            for q in range(n):
                H += h[p, q] * self.E[p][q]
        for p in range(n):
            for q in range(n):
                Epq = self.E[p][q]
                for r in range(n):
                    for s in range(n):
                        g = eri[p, q, r, s]
                        if g == 0.0:
                            continue
                        term = Epq @ self.E[r][s]
                        if q == r:
                            term = term - self.E[p][s]
                        H += 0.5 * g * term
        return H

    def cluster_operator(self, t1, t2):
        """T = sum t1[i,a] E_ai + 1/2 sum t2[i,j,a,b] E_ai E_bj."""
        o = self.nocc
        v = self.n - o
        T = np.zeros((self.dim, self.dim))
        for i in range(o):
            for a in range(v):
                T += t1[i, a] * self.E[o + a][i]
        for i in range(o):
            for j in range(o):
                for a in range(v):
                    for b in range(v):
                        if t2[i, j, a, b] != 0.0:
                            T += 0.5 * t2[i, j, a, b] * (self.E[o + a][i] @ self.E[o + b][j])
        return T


def _exp_apply(T, vec, sign):
    out = vec.copy()
    term = vec.copy()
    k = 1
    while True:
        term = sign * (T @ term) / k
        if not np.any(term):
            break
        out = out + term
        k += 1
        if k > 64:
            raise RuntimeError("cluster operator is not nilpotent")
    return out


def brute_force(h, eri, nocc, t1, t2):
    """Residual (r1, r2) and correlation energy, from the definition.

    h: n x n one-electron matrix; eri[p,q,r,s] = (pq|rs)."""
    n = h.shape[0]
    o = nocc
    v = n - o
    sp = DeterminantSpace(n, o)
    H = sp.hamiltonian(h, eri)
    T = sp.cluster_operator(t1, t2)
    psi = _exp_apply(T, sp.ref, +1.0)
    chi = _exp_apply(T, H @ psi, -1.0)
    r1 = np.zeros((o, v))
    r2 = np.zeros((o, o, v, v))
    for i in range(o):
        for a in range(v):
            mu = sp.Ea[o + a][i] @ sp.ref
            r1[i, a] = mu @ chi
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    mu = sp.Ea[o + a][i] @ (sp.Eb[o + b][j] @ sp.ref)
                    r2[i, j, a, b] = mu @ chi
    e_ref = sp.ref @ H @ sp.ref
    e_corr = sp.ref @ chi - e_ref
    return r1, r2, e_corr


def fci_ground_energy(h, eri, nocc):
    """Lowest eigenvalue of H, minus E_ref, within the spin-flip symmetry
    sector of Phi_0 (which holds the singlets). The operator that swaps
    alpha and beta labels maps |a-string, b-string> to
    (-1)^(nocc*nocc) |b-string, a-string> and leaves Phi_0 with that same
    sign, so the sector is the +1 eigenspace of sign * swap."""
    n = h.shape[0]
    sp = DeterminantSpace(n, nocc)
    H = sp.hamiltonian(h, eri)
    P = np.zeros((sp.dim, sp.dim))
    sgn = -1.0 if (nocc * nocc) % 2 else 1.0
    for k, (a, b) in enumerate(sp.dets):
        P[sp.index[(b, a)], k] = sgn
    S = sgn * P
    w, V = np.linalg.eigh(0.5 * (S + S.T))
    B = V[:, w > 0.5]
    evals = np.linalg.eigvalsh(B.T @ H @ B)
    e_ref = sp.ref @ H @ sp.ref
    return evals[0] - e_ref, evals - e_ref
