"""Pins of the CPU oracle against things other than itself.

Each test checks the oracle against a definition, a closed form, an
invariant or the paper's own constants, so that a dropped term, a wrong
sign or index or a transposed operand in oracle/ fails at least one of them.
"""

import json
import os

import numpy as np
import pytest

from gen import (haar_orthogonal, make_config, make_general, make_problem,
                 random_amplitudes)
from oracle import brute, ccsd, solvers

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _args(p):
    return p.f_oo, p.f_ov, p.f_vv, p.L


def _eri(L):
    return np.einsum("Ppq,Prs->pqrs", L, L)


# ---------------------------------------------------------------- T1 -----
@pytest.mark.parametrize("o,v,naux,seed", [(1, 1, 3, 1), (1, 3, 4, 2), (2, 2, 5, 3),
                                           (2, 3, 6, 4), (3, 2, 4, 5)])
def test_residual_equals_determinant_space_definition(o, v, naux, seed):
    """Equation CC_ampl / CC_energy evaluated literally in the determinant
    space equals the T1-dressed working equations (f_ov != 0, random t)."""
    p = make_general(o, v, naux, seed)
    t1, t2 = random_amplitudes(o, v, seed + 100, scale=0.1)
    h = ccsd.core_hamiltonian(p.fock(), p.L, o)
    r1b, r2b, eb = brute.brute_force(h, _eri(p.L), o, t1, t2)
    r1, r2 = ccsd.residual(*_args(p), t1, t2)
    e = ccsd.energy(*_args(p), t1, t2)
    assert np.abs(r2b).max() > 1e-2 and np.abs(r1b).max() > 1e-2
    assert np.allclose(r1, r1b, atol=1e-12, rtol=0)
    assert np.allclose(r2, r2b, atol=1e-12, rtol=0)
    assert abs(e - eb) < 1e-12


def test_residual_pair_symmetry():
    p = make_general(2, 3, 5, 8)
    t1, t2 = random_amplitudes(2, 3, 9)
    _, r2 = ccsd.residual(*_args(p), t1, t2)
    assert np.allclose(r2, np.transpose(r2, (1, 0, 3, 2)), atol=1e-14)


# ---------------------------------------------------------------- T3 -----
def _mp2_closed_form(p):
    """MP2 amplitudes t = (ia|jb) / (e_i + e_j - e_a - e_b) and energy
    sum (ia|jb)(2 t_ij^ab - t_ij^ba), by loops, for a diagonal Fock."""
    o, v = p.nocc, p.nvir
    eo, ev = np.diag(p.f_oo), np.diag(p.f_vv)
    t = np.zeros((o, o, v, v))
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    g = float(np.dot(p.L[:, i, o + a], p.L[:, j, o + b]))
                    t[i, j, a, b] = g / (eo[i] + eo[j] - ev[a] - ev[b])
    e = 0.0
    for i in range(o):
        for j in range(o):
            for a in range(v):
                for b in range(v):
                    g = float(np.dot(p.L[:, i, o + a], p.L[:, j, o + b]))
                    e += g * (2 * t[i, j, a, b] - t[i, j, b, a])
    return t, e


def test_mp2_first_step_closed_form():
    p = make_problem(3, 7, 12, 21, gauge="canonical")
    x = solvers.mp2_guess(*_args(p))
    t1, t2 = solvers.unpack(x, 3, 7)
    tm, em = _mp2_closed_form(p)
    assert np.abs(t1).max() < 1e-14
    assert np.allclose(t2, tm, atol=1e-13, rtol=0)
    assert abs(ccsd.energy(*_args(p), t1, t2) - em) < 1e-13
    # the same generalized-MP2 energy in a Haar-rotated gauge
    q = make_problem(3, 7, 12, 21, gauge="haar")
    y = solvers.mp2_guess(*_args(q))
    assert abs(ccsd.energy(*_args(q), *solvers.unpack(y, 3, 7)) - em) < 1e-12


# ---------------------------------------------------------------- T4 -----
def _rotate_problem(p, Uo, Uv):
    o = p.nocc
    U = np.zeros((p.L.shape[1],) * 2)
    U[:o, :o] = Uo
    U[o:, o:] = Uv
    L = np.einsum("pr,Prs,qs->Ppq", U, p.L, U)
    return Uo @ p.f_oo @ Uo.T, Uo @ p.f_ov @ Uv.T, Uv @ p.f_vv @ Uv.T, L


def test_gauge_covariance_of_residual_and_energy():
    p = make_general(3, 4, 6, 31)
    t1, t2 = random_amplitudes(3, 4, 32)
    rng = np.random.default_rng(33)
    Uo, Uv = haar_orthogonal(rng, 3), haar_orthogonal(rng, 4)
    q = _rotate_problem(p, Uo, Uv)
    s1 = Uo @ t1 @ Uv.T
    s2 = np.einsum("ik,jl,ac,bd,klcd->ijab", Uo, Uo, Uv, Uv, t2)
    r1, r2 = ccsd.residual(*_args(p), t1, t2)
    q1, q2 = ccsd.residual(*q, s1, s2)
    assert np.allclose(q1, Uo @ r1 @ Uv.T, atol=1e-13)
    assert np.allclose(q2, np.einsum("ik,jl,ac,bd,klcd->ijab", Uo, Uo, Uv, Uv, r2), atol=1e-13)
    assert abs(ccsd.energy(*q, s1, s2) - ccsd.energy(*_args(p), t1, t2)) < 1e-13


def test_pnk_history_is_gauge_invariant():
    """The paper's claim that PNK convergence is gauge invariant, made
    exact: 2-norm residual histories and step counts agree across gauges."""
    pc = make_problem(3, 8, 16, 41, gauge="canonical")
    ph = make_problem(3, 8, 16, 41, gauge="haar")
    _, _, ic = solvers.solve_pnk(*_args(pc), tol=1e-10)
    _, _, ih = solvers.solve_pnk(*_args(ph), tol=1e-10)
    assert ic.converged and ih.converged
    assert ic.n_jvp == ih.n_jvp and ic.newton_iters == ih.newton_iters
    hc = np.array([h[1] for h in ic.history])
    hh = np.array([h[1] for h in ih.history])
    assert np.allclose(hc, hh, rtol=1e-6, atol=1e-12)
    assert abs(ic.e_corr - ih.e_corr) < 1e-11


# ---------------------------------------------------------------- T5 -----
def test_jvp_complex_step_matches_central_difference():
    p = make_general(3, 5, 8, 51)
    t1, t2 = random_amplitudes(3, 5, 52, scale=0.1)
    v1, v2 = random_amplitudes(3, 5, 53, scale=1.0)
    j1, j2 = ccsd.jvp_complex_step(*_args(p), t1, t2, v1, v2)
    c1, c2 = ccsd.jvp_central(*_args(p), t1, t2, v1, v2)
    num = np.sqrt(np.sum((j1 - c1) ** 2) + np.sum((j2 - c2) ** 2))
    den = np.sqrt(np.sum(j1 ** 2) + np.sum(j2 ** 2))
    assert num / den < 1e-7
    # linearity in v (complex step is exact for a polynomial residual)
    k1, k2 = ccsd.jvp_complex_step(*_args(p), t1, t2, 2 * v1, 2 * v2)
    assert np.allclose(k2, 2 * j2, rtol=1e-13, atol=1e-15)


# ---------------------------------------------------------------- T6 -----
def test_fock_operator_is_jacobian_at_zero_without_two_electron_part():
    p = make_general(3, 4, 5, 61)
    x1, x2 = random_amplitudes(3, 4, 62, scale=1.0)
    z1, z2 = np.zeros((3, 4)), np.zeros((3, 3, 4, 4))
    j1, j2 = ccsd.jvp_complex_step(p.f_oo, p.f_ov, p.f_vv, np.zeros_like(p.L), z1, z2, x1, x2)
    a1, a2 = solvers.fock_apply(p.f_oo, p.f_ov, p.f_vv, x1, x2)
    assert np.allclose(a1, j1, atol=1e-14) and np.allclose(a2, j2, atol=1e-14)


def test_fock_operator_inverse_gmres_equals_eigendecomposition():
    p = make_general(3, 6, 5, 63)
    b1, b2 = random_amplitudes(3, 6, 64, scale=1.0)
    e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, b1, b2)
    g1, g2, res = solvers.fock_solve_gmres(p.f_oo, p.f_ov, p.f_vv, b1, b2, rtol=1e-13)
    assert res.converged
    assert np.allclose(g1, e1, atol=1e-11) and np.allclose(g2, e2, atol=1e-11)
    y1, y2 = solvers.fock_apply(p.f_oo, p.f_ov, p.f_vv, e1, e2)
    assert np.allclose(y1, b1, atol=1e-12) and np.allclose(y2, b2, atol=1e-12)


def test_fock_doubles_block_is_symmetric():
    p = make_general(2, 3, 4, 65)
    o, v = 2, 3
    N2 = o * o * v * v
    A = np.zeros((N2, N2))
    for k in range(N2):
        e = np.zeros(N2)
        e[k] = 1.0
        _, y2 = solvers.fock_apply(p.f_oo, p.f_ov, p.f_vv, np.zeros((o, v)), e.reshape(o, o, v, v))
        A[:, k] = y2.ravel()
    assert np.allclose(A, A.T, atol=1e-15)


def test_fock_operator_spectrum_is_a_kronecker_sum_of_the_singles_block():
    """With f_ov = 0, A_F is block diagonal and its doubles block is the
    Kronecker sum of the singles block with itself: its eigenvalues are all
    sums lam_p + lam_q of singles eigenvalues, so its spectrum spans exactly
    twice the singles range (the fact behind the factor 2 on the singles in
    the device's symmetric inner solve). Built column by column from the
    oracle's A_F in a rotated gauge."""
    p = make_problem(2, 3, 8, 66, gauge="haar")
    o, v = 2, 3
    n1, n2 = o * v, o * o * v * v
    A = np.zeros((n1 + n2, n1 + n2))
    for k in range(n1 + n2):
        e = np.zeros(n1 + n2)
        e[k] = 1.0
        y1, y2 = solvers.fock_apply(p.f_oo, p.f_ov, p.f_vv, e[:n1].reshape(o, v), e[n1:].reshape(o, o, v, v))
        A[:, k] = np.concatenate([y1.ravel(), y2.ravel()])
    assert np.abs(A[:n1, n1:]).max() == 0.0 and np.abs(A[n1:, :n1]).max() == 0.0
    lam1 = np.linalg.eigvalsh(A[:n1, :n1])
    lam2 = np.linalg.eigvalsh(A[n1:, n1:])
    sums = np.sort((lam1[:, None] + lam1[None, :]).ravel())
    assert np.allclose(lam2, sums, atol=1e-12)
    assert abs(lam2[0] - 2 * lam1[0]) < 1e-12 and abs(lam2[-1] - 2 * lam1[-1]) < 1e-12
    # the singles eigenvalues are the orbital-energy gaps eps_a - eps_i
    gaps = np.sort((np.linalg.eigvalsh(p.f_vv)[None, :] - np.linalg.eigvalsh(p.f_oo)[:, None]).ravel())
    assert np.allclose(lam1, gaps, atol=1e-12)


# ---------------------------------------------------------------- T7 -----
@pytest.mark.parametrize("seed", [71, 72])
def test_ccsd_equals_fci_for_one_occupied_orbital(seed):
    p = make_general(1, 5, 7, seed, sigma=0.15, fov_scale=0.1)
    _, _, info = solvers.solve_pnk(*_args(p), tol=1e-12)
    h = ccsd.core_hamiltonian(p.fock(), p.L, 1)
    efci, _ = brute.fci_ground_energy(h, _eri(p.L), 1)
    assert info.converged
    assert abs(info.e_corr - efci) < 1e-11


# ---------------------------------------------------------------- T8 -----
def test_thouless_solution_without_two_electron_part():
    """With L = 0 the exact state is the determinant of the lowest nocc
    eigenvectors C of f: t1 = C_v C_o^{-1}, t2 = 0, E = 2 (sum lambda - tr f_oo)."""
    p = make_general(3, 5, 4, 81, fov_scale=0.2)
    t1, t2, info = solvers.solve_pnk(p.f_oo, p.f_ov, p.f_vv, np.zeros_like(p.L), tol=1e-12)
    lam, C = np.linalg.eigh(p.fock())
    Co, Cv = C[:3, :3], C[3:, :3]
    assert info.converged
    assert np.allclose(t1, (Cv @ np.linalg.inv(Co)).T, atol=1e-11)
    assert np.abs(t2).max() < 1e-11
    assert abs(info.e_corr - 2 * (lam[:3].sum() - np.trace(p.f_oo))) < 1e-11


# ---------------------------------------------------------------- T9 -----
def test_pnk_and_fp_diis_reach_the_same_root_c1():
    p = make_config("c1_canonical")
    a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-11)
    b1, b2, ib = solvers.solve_fp_diis(*_args(p), tol=1e-11)
    assert ia.converged and ib.converged
    assert abs(ia.e_corr - ib.e_corr) < 1e-10
    assert np.abs(a2 - b2).max() < 1e-10 and np.abs(a1 - b1).max() < 1e-10
    # PNK needs fewer residual evaluations than FP+DIIS (paper, Fig. 4)
    assert ia.n_residual + ia.n_jvp < ib.n_residual


def test_forward_difference_pnk_converges_like_exact_jvp():
    p = make_problem(3, 8, 16, 91, gauge="haar")
    _, _, ie = solvers.solve_pnk(*_args(p), tol=1e-9)
    _, _, idf = solvers.solve_pnk(*_args(p), tol=1e-9, jvp="fd")
    assert ie.converged and idf.converged
    assert abs(ie.e_corr - idf.e_corr) < 1e-9


def test_fp_diverges_or_slows_in_rotated_gauge_while_pnk_does_not():
    """Jacobi denominators taken from the diagonal of a rotated Fock matrix
    (FP AO) lose accuracy; PNK's count stays the same."""
    pc = make_problem(3, 8, 16, 93, gauge="canonical")
    ph = make_problem(3, 8, 16, 93, gauge="haar")
    _, _, fc = solvers.solve_fp_diis(*_args(pc), tol=1e-9, diis_size=0, max_iter=300)
    _, _, fh = solvers.solve_fp_diis(*_args(ph), tol=1e-9, diis_size=0, max_iter=300)
    assert fc.converged
    assert (not fh.converged) or fh.n_residual > fc.n_residual


# ------------------------------------------------- protocols, CCD ------
@pytest.mark.parametrize("o,v,naux,seed", [(2, 3, 6, 94), (2, 4, 5, 95)])
def test_ccd_root_zeroes_the_determinant_space_doubles(o, v, naux, seed):
    """The CCD level (t1 held at 0, singles equations dropped): PNK's root
    makes the doubles projections of exp(-T2) H exp(T2) vanish when they are
    evaluated literally in the determinant space, and its energy is the
    determinant-space one; the singles projections do not vanish (it is not
    the CCSD root)."""
    p = make_general(o, v, naux, seed, sigma=0.15, fov_scale=0.05)
    t1, t2, info = solvers.solve_pnk(*_args(p), tol=1e-12, ccd=True)
    assert info.converged and not np.any(t1)
    h = ccsd.core_hamiltonian(p.fock(), p.L, o)
    r1b, r2b, eb = brute.brute_force(h, _eri(p.L), o, t1, t2)
    assert np.abs(r2b).max() < 1e-11
    assert np.abs(r1b).max() > 1e-6
    assert abs(eb - info.e_corr) < 1e-12


def test_ink_is_the_fixed_point_iteration_in_the_canonical_gauge():
    """With a diagonal Fock matrix A_F is the diagonal of orbital-energy
    differences, so INK (A_F dt = -r) takes the same steps as plain FP
    (t <- t - r / D, no DIIS, no shift), from the same MP2 start."""
    p = make_problem(3, 8, 16, 96, gauge="canonical")
    _, _, ink = solvers.solve_ink(*_args(p), tol=1e-9)
    _, _, fp = solvers.solve_fp_diis(*_args(p), tol=1e-9, diis_size=0)
    assert ink.converged and fp.converged
    assert ink.n_residual == fp.n_residual
    assert abs(ink.e_corr - fp.e_corr) < 1e-12
    hi = np.array([h[2] for h in ink.history])
    hf = np.array([h[2] for h in fp.history])
    assert np.allclose(hi, hf, rtol=1e-6, atol=0)  # GMRES to 1e-12 vs an exact division


@pytest.mark.parametrize("ccd", [False, True])
def test_protocols_reach_one_root_in_a_rotated_gauge(ccd):
    """NK, PNK, INK and SFP+DIIS (the method table) land on the same
    amplitudes and energy at the CCSD and at the CCD level; INK and NK are
    gauge invariant, so INK's history is that of the canonical problem."""
    p = make_problem(3, 7, 14, 97, gauge="haar")
    runs = {
        "pnk": solvers.solve_pnk(*_args(p), tol=1e-10, ccd=ccd),
        "nk": solvers.solve_pnk(*_args(p), tol=1e-10, precond=False, ccd=ccd, max_newton=200),
        "ink": solvers.solve_ink(*_args(p), tol=1e-10, ccd=ccd),
        "sfp": solvers.solve_fp_diis(*_args(p), tol=1e-10, level_shift=0.2, ccd=ccd),
    }
    ref1, ref2, ref = runs["pnk"]
    for name, (t1, t2, info) in runs.items():
        assert info.converged, name
        assert abs(info.e_corr - ref.e_corr) < 1e-9, name
        assert np.abs(t2 - ref2).max() < 1e-8 and np.abs(t1 - ref1).max() < 1e-8, name
    pc = make_problem(3, 7, 14, 97, gauge="canonical")
    _, _, inkc = solvers.solve_ink(*_args(pc), tol=1e-10, ccd=ccd)
    assert inkc.n_residual == runs["ink"][2].n_residual
    assert abs(inkc.e_corr - ref.e_corr) < 1e-9


# ------------------------------------------------------ forcing term -----
# Eisenstat & Walker (SIAM J. Sci. Comput. 17 (1996) 16), choice 2, with the
# paper's gamma = 0.9, alpha = 1.5 (Section "Adaptive Forcing"), eta_0 = 0.5,
# eta_max = 0.9, the safeguard max(eta, gamma eta_prev^alpha) when
# gamma eta_prev^alpha > 0.1, and the floor 0.5 tol / ||r_k||. Expected values
# are decimal evaluations of those definitions:
#   0.9 * 0.5**1.5  = 0.31819805153394637   (ratio ||r_k|| / ||r_{k-1}|| = 0.5)
#   0.9 * 0.8**1.5  = 0.64398757751993940   (safeguard from eta_prev = 0.8)
#   0.9 * 0.4**1.5  = 0.22768399153212330   (safeguard from eta_prev = 0.4)
#   0.9 * 0.2**1.5  = 0.08049844718999243   (below 0.1: safeguard off)
#   0.9 * 0.01**1.5 = 0.0009                (ratio 0.01)
#   0.9 * 2**1.5    = 2.545584412271571     (ratio 2: above the cap)
@pytest.mark.parametrize("k,rn,rn_prev,eta_prev,tol,expected", [
    (0, 3.0, None, 0.5, 1e-8, 0.5),                       # first step: eta_0
    (1, 0.5, 1.0, 0.8, 1e-12, 0.6439875775199394),        # safeguard above the plain term
    (1, 0.5, 1.0, 0.2, 1e-12, 0.31819805153394637),       # safeguard off (0.0805 <= 0.1)
    (1, 0.5, 1.0, 0.4, 1e-12, 0.31819805153394637),       # safeguard on but smaller
    (1, 0.01, 1.0, 0.4, 1e-12, 0.2276839915321233),       # safeguard lifts 0.0009
    (1, 0.01, 1.0, 0.2, 1e-12, 0.0009),                   # plain term, small
    (1, 2.0, 1.0, 0.2, 1e-12, 0.9),                       # cap eta_max
    (1, 0.01, 1.0, 1.0, 1e-12, 0.9),                      # safeguard 0.9 itself, at the cap
    (1, 2e-8, 2e-6, 0.05, 1e-8, 0.25),                    # floor 0.5 * 1e-8 / 2e-8
    (1, 4e-9, 4e-7, 0.05, 1e-8, 0.9),                     # floor 1.25 capped at eta_max
])
def test_forcing_term_branches(k, rn, rn_prev, eta_prev, tol, expected):
    eta = solvers.forcing_term(k, rn, rn_prev, eta_prev, tol)
    assert eta == pytest.approx(expected, rel=1e-13, abs=0.0)


# ---------------------------------------------------------- constants ----
def test_paper_constants():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        g = json.load(fh)
    # safeguard inactive (gamma * eta_prev^alpha < 0.1): eta = gamma (ratio)^alpha
    eta = solvers.forcing_term(1, 0.1, 1.0, 0.01, 1e-12)
    assert eta == pytest.approx(g["ew_gamma"] * 0.1 ** g["ew_alpha"], rel=1e-14)
    assert g["convergence_threshold"] == 1e-8
    M = np.array(g["conclusion_matrix"])
    lam = np.linalg.eigvalsh(M)
    assert abs(M[0, 0] - M[1, 1]) == pytest.approx(g["conclusion_diag_gap"], abs=1e-12)
    assert abs(lam[1] - lam[0]) == pytest.approx(g["conclusion_spectral_gap_approx"], rel=1e-3)


# ------------------------------------------------------- level shift -----
def _dense_fp_jacobian_sym(p, t1, t2, shift):
    """G = I - diag(D + s)^-1 J on pair-symmetric vectors, built column by
    column from complex-step products on an orthonormal basis of that space."""
    o, v = p.nocc, p.nvir
    n = o * v + o * o * v * v
    cols = []
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        s = solvers.pair_symmetrize(e, o, v)
        if np.linalg.norm(s) > 0:
            cols.append(s)
    U, sv, _ = np.linalg.svd(np.array(cols).T, full_matrices=False)
    rank = int(np.sum(sv > 1e-10 * sv[0]))
    B = U[:, :rank]  # orthonormal basis of the pair-symmetric space
    d1, d2 = solvers.jacobi_denominators(p.f_oo, p.f_vv, shift)
    D = solvers.pack(d1, d2)
    G = np.zeros((rank, rank))
    for c in range(rank):
        q1, q2 = solvers.unpack(B[:, c], o, v)
        j1, j2 = ccsd.jvp_complex_step(*_args(p), t1, t2, q1, q2)
        G[:, c] = B.T @ (B[:, c] - solvers.pack(j1, j2) / D)
    return G


@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_fp_spectral_radius_equals_the_dense_jacobian(shift):
    """Arnoldi over the whole pair-symmetric space finds the eigenvalues of
    the dense FP Jacobian built from unit-vector products."""
    p = make_problem(2, 3, 6, 98, gauge="haar")
    t1, t2, info = solvers.solve_pnk(*_args(p), tol=1e-10)
    assert info.converged
    G = _dense_fp_jacobian_sym(p, t1, t2, shift)
    rho_dense = np.max(np.abs(np.linalg.eigvals(G)))
    rho, _ = solvers.fp_jacobian_spectral_radius(*_args(p), t1, t2, shift=shift, m=G.shape[0])
    assert abs(rho - rho_dense) < 1e-9 * max(1.0, rho_dense)


@pytest.mark.parametrize("shift", [0.0, 0.5])
def test_fp_contraction_rate_is_the_spectral_radius(shift):
    """The FP Jacobian at the root decides (S)FP's local behaviour: started
    close to the root, plain shifted FP (no DIIS) contracts by a factor that
    tends to the spectral radius; the last step's ratio matches it. A shift
    where none is needed raises the radius (slower steps)."""
    p = make_problem(3, 8, 16, 99, gauge="canonical")
    t1, t2, info = solvers.solve_pnk(*_args(p), tol=1e-11)
    rho, _ = solvers.fp_jacobian_spectral_radius(*_args(p), t1, t2, shift=shift, m=60)
    rho0, _ = solvers.fp_jacobian_spectral_radius(*_args(p), t1, t2, shift=0.0, m=60)
    assert rho < 1.0 and (shift == 0.0 or rho > rho0)
    x0 = solvers.pack(t1, t2) + 1e-4 * solvers.pair_symmetrize(
        np.random.default_rng(5).standard_normal(3 * 8 + 9 * 64), 3, 8)
    _, _, fp = solvers.solve_fp_diis(*_args(p), tol=1e-13, diis_size=0, level_shift=shift, x0=x0, max_iter=400)
    h = np.array([r[1] for r in fp.history])
    assert fp.converged and abs(h[-1] / h[-2] - rho) < 0.02


# ------------------------------------------------- non-orthogonal gauge ----
def _gauge_problem(seed=1101, o=3, v=7, naux=20, cond=4.0, kind="haar"):
    from gen import nonorthogonal_gauge
    p = make_general(o, v, naux, seed) if kind == "general" else make_problem(o, v, naux, seed, gauge=kind)
    Wo, Wv = nonorthogonal_gauge(o, v, seed + 7, cond)
    return p, Wo, Wv


def test_gauge_matrices_have_the_requested_condition_number():
    from gen import nonorthogonal_gauge
    Wo, Wv = nonorthogonal_gauge(5, 12, 3, 6.0)
    assert abs(np.linalg.cond(Wo) - 6.0) < 1e-9 and abs(np.linalg.cond(Wv) - 6.0) < 1e-9
    Wo, Wv = nonorthogonal_gauge(5, 12, 3, 1.0)
    assert np.abs(Wo.T @ Wo - np.eye(5)).max() < 1e-13 and np.abs(Wv.T @ Wv - np.eye(12)).max() < 1e-13


def test_gauge_orthogonal_case_is_a_rotation_of_the_hamiltonian():
    """For orthogonal W the gauge amplitudes are those of the rotated
    orbitals phi W: the gauge residual equals the orbital-basis residual of
    the Hamiltonian rotated by U = W^T (f -> U f U^T, L^P -> U L^P U^T),
    singles and f_ov included."""
    from oracle import gauge
    p, Wo, Wv = _gauge_problem(kind="general", cond=1.0)
    o, v = p.f_oo.shape[0], p.f_vv.shape[0]
    U = np.zeros((o + v, o + v))
    U[:o, :o], U[o:, o:] = Wo.T, Wv.T
    f = U @ p.fock() @ U.T
    Lr = np.einsum("pr,Prs,qs->Ppq", U, p.L, U)
    th1, th2 = random_amplitudes(o, v, 31, scale=0.1)
    r1, r2 = gauge.residual(*_args(p), Wo, Wv, th1, th2)
    q1, q2 = ccsd.residual(f[:o, :o], f[:o, o:], f[o:, o:], Lr, th1, th2)
    assert np.abs(r1 - q1).max() < 1e-12 and np.abs(r2 - q2).max() < 1e-12
    e = gauge.energy(*_args(p), Wo, Wv, th1, th2)
    assert abs(e - ccsd.energy(f[:o, :o], f[:o, o:], f[o:, o:], Lr, th1, th2)) < 1e-13


@pytest.mark.parametrize("cond", [2.0, 8.0])
def test_gauge_residual_equals_the_appendix_random_gauge_equations(cond):
    """The definition r(theta) = U-bar^(x4) r(t) equals the random-gauge CCD
    residual written out in the appendix's transformed integrals, Fock
    blocks and intermediates, for a non-orthogonal gauge."""
    from oracle import gauge
    p, Wo, Wv = _gauge_problem(cond=cond)
    o, v = p.f_oo.shape[0], p.f_vv.shape[0]
    _, t2 = random_amplitudes(o, v, 32, scale=0.1)
    _, th2 = gauge.forward(Wo, Wv, np.zeros((o, v)), t2)
    _, r2 = gauge.residual(*_args(p), Wo, Wv, np.zeros((o, v)), th2)
    x2 = gauge.residual_ccd_explicit(p.f_oo, p.f_vv, p.L, Wo, Wv, th2)
    assert np.abs(r2 - x2).max() < 1e-12 * max(1.0, np.abs(r2).max())


def test_gauge_fock_operator_is_the_jacobian_without_two_electron_part():
    """A_F in the gauge (Kronecker sum of Fv and -Fo, f_ov coupling) is the
    Jacobian of the gauge residual at theta = 0 when L = 0; it is not
    symmetric for a non-orthogonal gauge."""
    from oracle import gauge
    p, Wo, Wv = _gauge_problem(kind="general")
    o, v = p.f_oo.shape[0], p.f_vv.shape[0]
    Fo, Fv = gauge.fock_blocks(p.f_oo, p.f_vv, Wo, Wv)
    x1, x2 = random_amplitudes(o, v, 33)
    j1, j2 = gauge.jvp_complex_step(p.f_oo, p.f_ov, p.f_vv, np.zeros_like(p.L), Wo, Wv,
                                    np.zeros((o, v)), np.zeros((o, o, v, v)), x1, x2)
    a1, a2 = gauge.fock_apply(p.f_ov, Wo, Wv, Fo, Fv, x1, x2)
    assert np.abs(j1 - a1).max() < 1e-13 and np.abs(j2 - a2).max() < 1e-13
    assert np.abs(Fv - Fv.T).max() > 1e-3 and np.abs(Fo - Fo.T).max() > 1e-3


def test_gauge_fp_in_a_diagonal_gauge_follows_the_orbital_fp():
    """A diagonal gauge W = diag(s) leaves the diagonals of the Fock blocks
    unchanged, so the gauge FP step (no DIIS) is the orbital FP step
    transformed: after k steps theta_k = U-bar^(x4) t_k."""
    from oracle import gauge
    p = make_problem(3, 7, 20, 1102, gauge="canonical")
    rng = np.random.default_rng(4)
    Wo, Wv = np.diag(rng.uniform(0.5, 2.0, 3)), np.diag(rng.uniform(0.5, 2.0, 7))
    a1, a2, ia = solvers.solve_fp_diis(*_args(p), tol=1e-30, diis_size=0, max_iter=4, gauge=(Wo, Wv))
    b1, b2, ib = solvers.solve_fp_diis(*_args(p), tol=1e-30, diis_size=0, max_iter=4)
    c1, c2 = gauge.forward(Wo, Wv, b1, b2)
    assert ia.newton_iters == ib.newton_iters == 4
    assert np.abs(a1 - c1).max() < 1e-13 and np.abs(a2 - c2).max() < 1e-13


def test_gauge_pnk_lands_on_the_transformed_root():
    """PNK on the gauge amplitudes (A_F of the gauge, solved by GMRES)
    converges to U-bar^(x4) t* with the orbital-basis energy."""
    from gen import nonorthogonal_gauge
    from oracle import gauge
    p = make_problem(4, 16, 48, 1001, gauge="haar")
    Wo, Wv = nonorthogonal_gauge(4, 16, 2002, 4.0)
    a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-11, gauge=(Wo, Wv))
    b1, b2, ib = solvers.solve_pnk(*_args(p), tol=1e-11)
    c1, c2 = gauge.forward(Wo, Wv, b1, b2)
    assert ia.converged and ib.converged
    assert np.abs(a1 - c1).max() < 1e-9 and np.abs(a2 - c2).max() < 1e-9
    assert abs(ia.e_corr - ib.e_corr) < 1e-10


def test_gauge_ink_is_the_orbital_ink_transformed():
    """INK's update t <- t - A_F^-1 r(t) is covariant: in any invertible
    gauge its iterates are the transformed orbital-basis iterates (A_F of the
    gauge is the similarity transform of A_F), at the CCD level too."""
    from gen import nonorthogonal_gauge
    from oracle import gauge
    p = make_problem(3, 7, 20, 1105, gauge="haar")
    Wo, Wv = nonorthogonal_gauge(3, 7, 2005, 4.0)
    for ccd in (False, True):
        a1, a2, ia = solvers.solve_ink(*_args(p), tol=1e-30, max_iter=3, ccd=ccd, gauge=(Wo, Wv))
        b1, b2, ib = solvers.solve_ink(*_args(p), tol=1e-30, max_iter=3, ccd=ccd)
        c1, c2 = gauge.forward(Wo, Wv, b1, b2)
        assert ia.newton_iters == ib.newton_iters == 3
        assert np.abs(a2 - c2).max() < 1e-10 and np.abs(a1 - c1).max() < 1e-10


# ------------------------------------------------------ redundant gauge ----
# Gauges with more functions than the block has orbitals (W_o: o x m_o,
# W_v: v x m_v, full row rank; the appendix's projectors for a rectangular
# U), as projected atomic orbitals are for the virtual space.
def _redundant(seed=1201, o=2, v=4, m_o=3, m_v=6, naux=12, cond=3.0, kind="haar"):
    from gen import redundant_gauge
    p = make_general(o, v, naux, seed) if kind == "general" else make_problem(o, v, naux, seed, gauge=kind)
    Wo, Wv = redundant_gauge(o, v, m_o, m_v, seed + 7, cond)
    return p, Wo, Wv


def test_redundant_gauge_coefficients_and_projector():
    """C = W^+ satisfies W C = 1; Pi = W^T (W W^T)^-1 W is the orthogonal
    projector of rank n onto the range of U-bar = W^T, and gauge amplitudes
    of orbital amplitudes lie in that range on every index; for a square W,
    C is W^-1 and Pi the identity."""
    from gen import nonorthogonal_gauge
    from oracle import gauge
    p, Wo, Wv = _redundant()
    for W, n in ((Wo, 2), (Wv, 4)):
        C = gauge.coefficients(W)
        Pi = gauge.projector(W)
        assert np.abs(W @ C - np.eye(n)).max() < 1e-13
        assert np.abs(Pi @ Pi - Pi).max() < 1e-13 and np.abs(Pi - Pi.T).max() < 1e-13
        assert np.linalg.matrix_rank(Pi, tol=1e-10) == n
    t1, t2 = random_amplitudes(2, 4, 41)
    th1, th2 = gauge.forward(Wo, Wv, t1, t2)
    Po, Pv = gauge.projector(Wo), gauge.projector(Wv)
    assert np.abs(np.einsum("MA,NB,LC,SD,ABCD->MNLS", Po, Po, Pv, Pv, th2) - th2).max() < 1e-13
    b1, b2 = gauge.backward(Wo, Wv, th1, th2)
    assert np.abs(b1 - t1).max() < 1e-13 and np.abs(b2 - t2).max() < 1e-13
    Wq, _ = nonorthogonal_gauge(3, 5, 7, 4.0)
    assert np.abs(gauge.coefficients(Wq) - np.linalg.inv(Wq)).max() < 1e-12


@pytest.mark.parametrize("in_range", [True, False])
def test_redundant_gauge_residual_equals_the_appendix_equations(in_range):
    """The definition r(theta) = U-bar^(x4) r(C^(x4) theta) equals the
    random-gauge CCD equations written out in the appendix's transformed
    quantities, for a redundant gauge. Those equations carry theta's free
    (covariant) indices through unchanged, so they presume theta in the range
    of U-bar^(x4); the definition sees only the projection Pi^(x4) theta, and
    for theta with components outside the range it equals the explicit
    equations at that projection."""
    from oracle import gauge
    p, Wo, Wv = _redundant(cond=5.0)
    _, t2 = random_amplitudes(2, 4, 42, scale=0.1)
    _, th2 = gauge.forward(Wo, Wv, np.zeros((2, 4)), t2)
    proj = th2
    if not in_range:
        rng = np.random.default_rng(43)
        extra = rng.standard_normal(th2.shape)
        th2 = th2 + 0.05 * (extra + np.transpose(extra, (1, 0, 3, 2)))
        Po, Pv = gauge.projector(Wo), gauge.projector(Wv)
        proj = np.einsum("MA,NB,LC,SD,ABCD->MNLS", Po, Po, Pv, Pv, th2)
        assert np.abs(proj - th2).max() > 1e-3
    _, r2 = gauge.residual(*_args(p), Wo, Wv, np.zeros((3, 6)), th2)
    x2 = gauge.residual_ccd_explicit(p.f_oo, p.f_vv, p.L, Wo, Wv, proj)
    assert np.abs(r2 - x2).max() < 1e-12 * max(1.0, np.abs(r2).max())


def test_redundant_gauge_jacobian_has_the_orbital_spectrum_and_a_null_space():
    """J_theta = U-bar^(x4) J C^(x4) with C^(x4) U-bar^(x4) = 1: its nonzero
    eigenvalues are those of the orbital-basis Jacobian J, and the rest of the
    gauge space (dimension m_o m_v + m_o^2 m_v^2 - (o v + o^2 v^2)) is null.
    Dense matrices from complex-step products on unit vectors (o=1, v=2,
    m_o=2, m_v=3)."""
    from gen import redundant_gauge
    from oracle import gauge
    p = make_general(1, 2, 5, 1202)
    Wo, Wv = redundant_gauge(1, 2, 2, 3, 1203, 3.0)
    t1, t2 = random_amplitudes(1, 2, 44, scale=0.1)
    th1, th2 = gauge.forward(Wo, Wv, t1, t2)

    def dense(fn, n, shape1, shape2):
        cols = []
        for k in range(n):
            e = np.zeros(n)
            e[k] = 1.0
            e1 = e[: np.prod(shape1)].reshape(shape1)
            e2 = e[np.prod(shape1):].reshape(shape2)
            j1, j2 = fn(e1, e2)
            cols.append(np.concatenate([j1.ravel(), j2.ravel()]))
        return np.array(cols).T

    ng = 2 * 3 + 4 * 9
    Jg = dense(lambda a, b: gauge.jvp_complex_step(*_args(p), Wo, Wv, th1, th2, a, b), ng, (2, 3), (2, 2, 3, 3))
    Jo = dense(lambda a, b: ccsd.jvp_complex_step(*_args(p), t1, t2, a, b), 2 + 4, (1, 2), (1, 1, 2, 2))
    eg = np.linalg.eigvals(Jg)
    eo = np.linalg.eigvals(Jo)
    scale = np.abs(eo).max()
    nonzero = eg[np.abs(eg) > 1e-9 * scale]
    assert len(nonzero) == len(eo) and np.linalg.matrix_rank(Jg, tol=1e-9 * scale) == 6
    assert np.allclose(np.sort_complex(nonzero), np.sort_complex(eo), rtol=1e-8, atol=1e-10 * scale)


def test_redundant_gauge_gmres_inverts_the_singular_fock_operator_on_its_range():
    """A_F of a redundant gauge is singular (its null space is that of
    C^(x4)); GMRES from zero on a right-hand side in its range converges to
    the one solution in the range, U-bar^(x4) A_F^-1 C^(x4) b."""
    from oracle import gauge
    p, Wo, Wv = _redundant(o=3, v=5, m_o=4, m_v=8, naux=16)
    Fo, Fv = gauge.fock_blocks(p.f_oo, p.f_vv, Wo, Wv)
    t1, t2 = random_amplitudes(3, 5, 45, scale=1.0)
    b1, b2 = gauge.forward(Wo, Wv, t1, t2)
    res = solvers.gmres(lambda y: solvers.pack(*gauge.fock_apply(p.f_ov, Wo, Wv, Fo, Fv, *solvers.unpack(y, 4, 8))),
                        solvers.pack(b1, b2), rtol=1e-12, maxit=400)
    assert res.converged
    e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, *gauge.backward(Wo, Wv, b1, b2))
    x1, x2 = gauge.forward(Wo, Wv, e1, e2)
    g1, g2 = solvers.unpack(res.x, 4, 8)
    assert np.abs(g2 - x2).max() < 1e-10 * np.abs(x2).max() and np.abs(g1 - x1).max() < 1e-10 * np.abs(x1).max()


def test_redundant_gauge_pnk_lands_on_the_transformed_root():
    """PNK on the amplitudes of a redundant gauge (the Newton systems are
    singular but consistent; GMRES's Krylov spaces stay in the range)
    converges to U-bar^(x4) t* with the orbital-basis energy, its iterate in
    the range of U-bar^(x4)."""
    from gen import redundant_gauge
    from oracle import gauge
    p = make_problem(3, 8, 22, 1204, gauge="haar")
    Wo, Wv = redundant_gauge(3, 8, 4, 11, 1205, 4.0)
    a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-11, gauge=(Wo, Wv))
    b1, b2, ib = solvers.solve_pnk(*_args(p), tol=1e-11)
    c1, c2 = gauge.forward(Wo, Wv, b1, b2)
    assert ia.converged and ib.converged
    assert a2.shape == (4, 4, 11, 11)
    assert np.abs(a1 - c1).max() < 1e-9 and np.abs(a2 - c2).max() < 1e-9
    assert abs(ia.e_corr - ib.e_corr) < 1e-10
    Po, Pv = gauge.projector(Wo), gauge.projector(Wv)
    assert np.abs(np.einsum("MA,NB,LC,SD,ABCD->MNLS", Po, Po, Pv, Pv, a2) - a2).max() < 1e-10
