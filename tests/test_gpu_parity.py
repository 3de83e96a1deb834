"""GPU parity: the HIP path through the C boundary against the CPU oracle.

Tolerances (FP64): both sides evaluate the same polynomial in float64 with
different summation orders, so elementwise differences are a few ulps of the
largest intermediate; we allow 1e-10 relative to the largest residual
component. Mixed-precision products are checked against bounds derived from
the unit roundoff of the compute type (FP32: 2^-24, BF16: 2^-8) times the
depth of the longest contraction.
"""

import numpy as np
import pytest

from gen import make_config, make_general, make_problem, random_amplitudes
from oracle import ccsd, solvers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_2608_06669_amd as pk
    pk.load()
    assert torch.cuda.is_available(), "a GPU is required"
    return pk


@pytest.fixture(scope="module")
def handle(lib):
    h = lib.Handle(0)
    yield h
    h.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    return t.detach().cpu().numpy()


def _args(p):
    return p.f_oo, p.f_ov, p.f_vv, p.L


# ------------------------------------------------------------ GEMM -----
# shapes cover the matrix-core tiles with ragged edges, one-row / one-column
# products, the short-contraction kernel (K <= 32 with a side <= 32, long
# side along N or along M) and tall ragged products as wide and long as the
# ladder at o=20 (210 and 129 rows)
@pytest.mark.parametrize("M,N,K", [(16, 16, 4), (33, 70, 19), (130, 257, 100), (400, 129, 300), (7, 1, 300),
                                   (5, 3000, 20), (3000, 7, 11), (32, 33, 32), (1, 1, 1),
                                   (210, 2100, 2100), (129, 2048, 2053)])
@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
def test_gemm_fp64_matches_float64_reference(lib, M, N, K, ta, tb):
    g = torch.Generator(device="cpu").manual_seed(M * 1000 + N + K)
    A = torch.randn(K, M, generator=g, dtype=torch.float64) if ta else torch.randn(M, K, generator=g, dtype=torch.float64)
    B = torch.randn(N, K, generator=g, dtype=torch.float64) if tb else torch.randn(K, N, generator=g, dtype=torch.float64)
    C0 = torch.randn(M, N, generator=g, dtype=torch.float64)
    ref = 0.7 * ((A.T if ta else A) @ (B.T if tb else B)) - 0.3 * C0
    Ad, Bd, Cd = A.cuda(), B.cuda(), C0.cuda()
    a_str = (1, M) if ta else (K, 1)
    b_str = (1, K) if tb else (N, 1)
    lib.diag_gemm(Ad, Bd, Cd, a_str, b_str, (N, 1), M, N, K, alpha=0.7, beta=-0.3)
    torch.cuda.synchronize()
    err = (Cd.cpu() - ref).abs().max().item()
    assert err <= 1e-12 * max(1.0, K ** 0.5) * ref.abs().max().item()


@pytest.mark.parametrize("prec,tol", [("fp32", 3e-5), ("bf16", 2e-2)])
def test_gemm_low_precision_bound(lib, prec, tol):
    g = torch.Generator(device="cpu").manual_seed(5)
    M, N, K = 200, 300, 512
    A = torch.randn(M, K, generator=g, dtype=torch.float64)
    B = torch.randn(K, N, generator=g, dtype=torch.float64)
    ref = A @ B
    Cd = torch.zeros(M, N, dtype=torch.float64, device="cuda")
    lib.diag_gemm(A.cuda(), B.cuda(), Cd, (K, 1), (N, 1), (N, 1), M, N, K, prec=prec)
    torch.cuda.synchronize()
    # error relative to the scale sqrt(K) of a product of unit normals; the
    # bound is K times the unit roundoff of the compute type (FP32 2^-24:
    # rounding of the products plus float accumulation; BF16 2^-8: input
    # rounding dominates)
    err = (Cd.cpu() - ref).abs().max().item() / K ** 0.5
    assert err < tol


# -------------------------------------------------------- residual -----
def _check_residual(handle, lib, p, t1, t2, rel=1e-10):
    P = lib.DeviceProblem.from_problem(p)
    r1, r2, e = handle.residual(P, dev(t1), dev(t2), energy=True)
    o1, o2 = ccsd.residual(*_args(p), t1, t2)
    oe = ccsd.energy(*_args(p), t1, t2)
    scale = max(np.abs(o1).max(), np.abs(o2).max())
    assert np.abs(host(r1) - o1).max() <= rel * scale
    assert np.abs(host(r2) - o2).max() <= rel * scale
    assert abs(e - oe) <= 1e-12 * max(1.0, abs(oe))


@pytest.mark.parametrize("o,v,naux,seed", [(1, 3, 5, 1), (3, 7, 12, 2), (5, 33, 40, 3), (2, 70, 30, 4)])
def test_residual_parity_general_gauge_with_fov(handle, lib, o, v, naux, seed):
    """Dense non-diagonal f with f_ov != 0, random t1, t2: every term."""
    p = make_general(o, v, naux, seed)
    t1, t2 = random_amplitudes(o, v, seed + 50, scale=0.05)
    _check_residual(handle, lib, p, t1, t2)


def test_residual_parity_c1(handle, lib):
    p = make_config("c1_canonical")
    t1, t2 = random_amplitudes(4, 16, 7, scale=0.02)
    _check_residual(handle, lib, p, t1, t2)


def test_residual_parity_c2_haar(handle, lib):
    p = make_config("c2_haar")
    t1, t2 = random_amplitudes(10, 90, 8, scale=0.01)
    _check_residual(handle, lib, p, t1, t2)


def test_residual_at_zero_is_mp2_source(handle, lib):
    p = make_problem(3, 9, 20, 9, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    z1, z2 = P.zeros_t()
    r1, r2 = handle.residual(P, z1, z2)
    o1, o2 = ccsd.residual(*_args(p), np.zeros((3, 9)), np.zeros((3, 3, 9, 9)))
    assert np.abs(host(r2) - o2).max() <= 1e-13 * np.abs(o2).max()
    assert np.abs(host(r1)).max() <= 1e-13


def test_problem_cache_sees_in_place_changes(handle, lib):
    p = make_general(3, 6, 8, 10)
    t1, t2 = random_amplitudes(3, 6, 11)
    P = lib.DeviceProblem.from_problem(p)
    a1, a2 = handle.residual(P, dev(t1), dev(t2))
    P.L.mul_(1.5)  # same pointers, new contents
    b1, b2 = handle.residual(P, dev(t1), dev(t2))
    q1, q2 = ccsd.residual(p.f_oo, p.f_ov, p.f_vv, 1.5 * p.L, t1, t2)
    assert np.abs(host(b2) - q2).max() <= 1e-10 * np.abs(q2).max()
    assert np.abs(host(a2) - host(b2)).max() > 1e-6


# ------------------------------------------------------------- J v -----
@pytest.mark.parametrize("o,v,naux,seed", [(3, 7, 12, 21), (4, 16, 48, 22), (2, 40, 30, 23)])
def test_jvp_fp64_parity(handle, lib, o, v, naux, seed):
    p = make_general(o, v, naux, seed)
    t1, t2 = random_amplitudes(o, v, seed + 1, scale=0.05)
    v1, v2 = random_amplitudes(o, v, seed + 2, scale=1.0)
    P = lib.DeviceProblem.from_problem(p)
    y1, y2 = handle.jvp(P, dev(t1), dev(t2), dev(v1), dev(v2), prec="fp64")
    j1, j2 = ccsd.jvp_complex_step(*_args(p), t1, t2, v1, v2)
    scale = max(np.abs(j1).max(), np.abs(j2).max())
    assert np.abs(host(y1) - j1).max() <= 1e-10 * scale
    assert np.abs(host(y2) - j2).max() <= 1e-10 * scale


@pytest.mark.parametrize("prec,rel", [("fp32", 5e-5), ("bf16", 3e-2)])
def test_jvp_mixed_precision_bound(handle, lib, prec, rel):
    p = make_problem(6, 40, 60, 31, gauge="haar")
    t1, t2 = random_amplitudes(6, 40, 32, scale=0.02)
    v1, v2 = random_amplitudes(6, 40, 33, scale=1.0)
    P = lib.DeviceProblem.from_problem(p)
    y1, y2 = handle.jvp(P, dev(t1), dev(t2), dev(v1), dev(v2), prec=prec)
    j1, j2 = ccsd.jvp_complex_step(*_args(p), t1, t2, v1, v2)
    num = np.sqrt(np.sum((host(y1) - j1) ** 2) + np.sum((host(y2) - j2) ** 2))
    den = np.sqrt(np.sum(j1 ** 2) + np.sum(j2 ** 2))
    assert num / den < rel


# ------------------------------------------------------------- A_F -----
def test_fock_apply_and_inverse(handle, lib):
    p = make_general(3, 8, 6, 41, fov_scale=0.1)
    x1, x2 = random_amplitudes(3, 8, 42, scale=1.0)
    P = lib.DeviceProblem.from_problem(p)
    y1, y2 = handle.fock_apply(P, dev(x1), dev(x2))
    a1, a2 = solvers.fock_apply(p.f_oo, p.f_ov, p.f_vv, x1, x2)
    assert np.abs(host(y1) - a1).max() <= 1e-13 * np.abs(a1).max()
    assert np.abs(host(y2) - a2).max() <= 1e-13 * np.abs(a2).max()
    s1, s2, iters, ok = handle.precond_solve(P, dev(x1), dev(x2), rtol=1e-13, maxit=300)
    e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, x1, x2)
    assert ok and iters > 0
    assert np.abs(host(s1) - e1).max() <= 1e-10 * np.abs(e1).max()
    assert np.abs(host(s2) - e2).max() <= 1e-10 * np.abs(e2).max()


def test_precond_solve_symmetric_fock_operator(handle, lib):
    """f_ov = 0: A_F is symmetric and the device runs the Lanczos form of
    GMRES; the result equals the eigendecomposition inverse."""
    p = make_problem(5, 23, 30, 43, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    # several calls in a row: the iterations replay a recorded HIP graph
    for seed in (44, 45, 46):
        x1, x2 = random_amplitudes(5, 23, seed, scale=1.0)
        s1, s2, iters, ok = handle.precond_solve(P, dev(x1), dev(x2), rtol=1e-12, maxit=300)
        e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, x1, x2)
        assert ok and 0 < iters < 300
        assert np.abs(host(s1) - e1).max() <= 1e-10 * np.abs(e1).max()
        assert np.abs(host(s2) - e2).max() <= 1e-10 * np.abs(e2).max()


@pytest.mark.parametrize("o,v,seed", [(5, 23, 47), (1, 9, 48), (10, 90, 49), (7, 40, 50), (12, 60, 51), (5, 64, 52),
                                      (6, 96, 53), (4, 91, 54), (16, 40, 57), (24, 20, 58), (25, 30, 59),
                                      (6, 17, 60), (8, 36, 61), (10, 100, 62)])
def test_precond_solve_pair_symmetric_packed_layout(handle, lib, o, v, seed):
    """cc_precond_solve_pairsym: the Lanczos vectors hold pairs i <= j only.
    The occupied part runs in the register-blocked form (64 positions per
    workgroup over 8 x 8 blocks, ragged at v=23, 9, 91, 90 and 20; 4 x 4
    blocks of the o x o output, ragged at o=5, 1, 10, 7 and 6) up to o=24,
    whose staging just fits a workgroup's LDS: 4 waves per workgroup at o <=
    8, 8 waves at o=10, 12 and 16, 16 at o=24, with a set's output blocks
    split over two workgroups at o=16/v=40 and o=24/v=20. Where the grid
    ends at most 4 elements into an odd-numbered last block (v=20, 17, 36
    and 100), each set pairing a block with the last one holds that block's
    columns by the 4 edge rows and the transpose (one set in place of two
    half-empty ones; at v=17 the edge strip is ragged too). At o=25 it falls
    back to the tile form (tile edge 2).
    The virtual contraction of the fused step runs in panels of 32 at v=23,
    in one panel of 96 at v=90 and 91 and of 64 at v=60 (o=12: 32-wide
    blocks), and exactly fills its one panel at v=64 and v=96; v=40 takes
    48-wide blocks and the three-launch step. Several calls in a row replay
    the recorded graphs; each result equals the eigendecomposition inverse,
    and agrees with the full-layout solve."""
    p = make_problem(o, v, 3 * (o + v), seed, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    for k in range(3):
        x1, x2 = random_amplitudes(o, v, seed + 100 + k, scale=1.0)
        s1, s2, iters, ok = handle.precond_solve(P, dev(x1), dev(x2), rtol=1e-12, maxit=300, pair_symmetric=True)
        e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, x1, x2)
        assert ok and 0 < iters < 300
        assert np.abs(host(s1) - e1).max() <= 1e-10 * np.abs(e1).max()
        assert np.abs(host(s2) - e2).max() <= 1e-10 * np.abs(e2).max()
        # unpacked by mirroring: x_ji = x_ij^T exactly for i != j; the
        # diagonal blocks hold (a, b) and (b, a) as separate elements
        g2 = host(s2)
        gt = np.transpose(g2, (1, 0, 3, 2))
        off = ~np.eye(o, dtype=bool)
        assert np.array_equal(g2[off], gt[off])
        assert np.abs(g2 - gt).max() <= 1e-12 * np.abs(g2).max()
    f1, f2, _, ok = handle.precond_solve(P, dev(x1), dev(x2), rtol=1e-12, maxit=300)
    assert ok
    assert np.abs(host(f2) - host(s2)).max() <= 1e-10 * np.abs(e2).max()


def test_precond_solve_pair_symmetric_solves_the_symmetric_part(handle, lib):
    """A right-hand side with an antisymmetric pair part: the packed solve
    returns A_F^-1 of its pair-symmetric part (b2[i][j] + b2[j][i]^T) / 2."""
    o, v = 4, 15
    p = make_problem(o, v, 30, 51, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    rng = np.random.default_rng(52)
    b1 = rng.standard_normal((o, v))
    b2 = rng.standard_normal((o, o, v, v))
    s1, s2, _, ok = handle.precond_solve(P, dev(b1), dev(b2), rtol=1e-12, maxit=300, pair_symmetric=True)
    sym2 = 0.5 * (b2 + np.transpose(b2, (1, 0, 3, 2)))
    e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, b1, sym2)
    assert ok
    assert np.abs(host(s1) - e1).max() <= 1e-10 * np.abs(e1).max()
    assert np.abs(host(s2) - e2).max() <= 1e-10 * np.abs(e2).max()


def test_precond_solve_zero_right_hand_side(handle, lib):
    """b = 0 gives x = 0 in both layouts, reported as converged."""
    o, v = 3, 10
    p = make_problem(o, v, 20, 53, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    z1, z2 = np.zeros((o, v)), np.zeros((o, o, v, v))
    for sym in (False, True):
        s1, s2, _, ok = handle.precond_solve(P, dev(z1), dev(z2), rtol=1e-12, maxit=60, pair_symmetric=sym)
        assert ok
        assert not np.any(host(s1)) and not np.any(host(s2))


def test_fock_operator_large_doubles_block(handle, lib):
    """o = 14, v = 130 (26 MB doubles block): the occupied terms leave the
    fused kernel's epilogue for two streaming passes, and the inner solve
    uses the unfused Lanczos step."""
    p = make_problem(14, 130, 20, 55, gauge="haar")
    x1, x2 = random_amplitudes(14, 130, 56, scale=1.0)
    P = lib.DeviceProblem.from_problem(p)
    y1, y2 = handle.fock_apply(P, dev(x1), dev(x2))
    a1, a2 = solvers.fock_apply(p.f_oo, p.f_ov, p.f_vv, x1, x2)
    assert np.abs(host(y1) - a1).max() <= 1e-13 * np.abs(a1).max()
    assert np.abs(host(y2) - a2).max() <= 1e-13 * np.abs(a2).max()
    s1, s2, iters, ok = handle.precond_solve(P, dev(x1), dev(x2), rtol=1e-12, maxit=300)
    e1, e2 = solvers.fock_solve_exact(p.f_oo, p.f_ov, p.f_vv, x1, x2)
    assert ok and 0 < iters < 300
    assert np.abs(host(s1) - e1).max() <= 1e-10 * np.abs(e1).max()
    assert np.abs(host(s2) - e2).max() <= 1e-10 * np.abs(e2).max()


def test_repeated_products_replay_graphs_exactly(handle, lib):
    """The third and later residual / J v calls with the same buffers replay
    recorded HIP graphs; every replay matches the first (eager) evaluation
    bit for bit, with eager work and synchronisations in between."""
    p = make_problem(4, 20, 30, 47, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2 = (dev(a) for a in random_amplitudes(4, 20, 48, scale=0.05))
    v1, v2 = (dev(a) for a in random_amplitudes(4, 20, 49, scale=1.0))
    r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
    ref = None
    for k in range(5):
        handle.residual(P, t1, t2, r1, r2)
        handle.residual(P, t1, t2, r1, r2)
        y1, y2 = handle.jvp(P, t1, t2, v1, v2, prec="fp64")
        torch.cuda.synchronize()
        cur = (host(r1), host(r2), host(y1), host(y2))
        if ref is None:
            ref = cur
        for a, b in zip(cur, ref):
            assert np.array_equal(a, b), k
        _ = (v1 * 2.0).sum().item()  # unrelated eager work between replays


# --------------------------------------------------------- solvers -----
def test_pnk_c1_matches_oracle(handle, lib):
    p = make_config("c1_canonical")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2, info = handle.solve_pnk(P, tol_inf=1e-11)
    a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-11)
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["e_corr"] - ia.e_corr) < 1e-9
    assert np.abs(host(t2) - a2).max() < 1e-9
    # the same Newton/Krylov path as the oracle
    assert info["n_jvp"] == ia.n_jvp and info["newton_iters"] == ia.newton_iters


def test_fp_diis_c1_matches_oracle(handle, lib):
    p = make_config("c1_canonical")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2, info = handle.solve_fp_diis(P, tol_inf=1e-10)
    a1, a2, ia = solvers.solve_fp_diis(*_args(p), tol=1e-10)
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["e_corr"] - ia.e_corr) < 1e-9
    # Far from DIIS's noise floor the two take the same path (near it the
    # Pulay system is nearly singular and rounding picks different steps).
    _, _, info6 = handle.solve_fp_diis(P, tol_inf=1e-6)
    _, _, ia6 = solvers.solve_fp_diis(*_args(p), tol=1e-6)
    assert info6["n_residual"] == ia6.n_residual


def test_fp_diis_in_a_rotated_gauge_matches_the_oracle(handle, lib):
    """FP+DIIS where plain FP diverges (Haar-rotated C1): DIIS carries the
    iteration down to 1e-9, past the point where the Pulay matrix (squared
    error norms) is 1e-14 of its unit border, in the oracle's number of
    steps (its Pulay system is solved in the least-squares sense)."""
    p = make_problem(4, 16, 48, 1001, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2, info = handle.solve_fp_diis(P, tol_inf=1e-9, max_iter=300)
    a1, a2, ia = solvers.solve_fp_diis(*_args(p), tol=1e-9, max_iter=300)
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["newton_iters"] - ia.newton_iters) <= 2
    assert abs(info["e_corr"] - ia.e_corr) < 1e-8
    assert np.abs(host(t2) - a2).max() < 1e-7


@pytest.mark.parametrize("ccd", [False, True])
def test_protocols_match_the_oracle(handle, lib, ccd):
    """The method table on the device: PNK, NK (no preconditioner) and INK
    (A_F dt = -r) in a rotated gauge, at the CCSD and the CCD level, against
    the oracle's solvers: same root, same energy, same number of steps."""
    p = make_problem(3, 7, 14, 97, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    cases = {
        "pnk": ({}, dict()),
        "nk": ({"max_newton": 200}, dict(precond=False, max_newton=200)),
    }
    for name, (gopt, oopt) in cases.items():
        t1, t2, info = handle.solve_pnk(P, tol_inf=1e-10, protocol=name, ccd=int(ccd), **gopt)
        a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-10, ccd=ccd, **oopt)
        assert info["status"] == "CC_OK" and ia.converged, name
        assert abs(info["e_corr"] - ia.e_corr) < 1e-9, name
        assert np.abs(host(t2) - a2).max() < 1e-8 and np.abs(host(t1) - a1).max() < 1e-8, name
        assert info["newton_iters"] == ia.newton_iters, name
        if ccd:
            assert not np.any(host(t1)), name
    t1, t2, info = handle.solve_pnk(P, tol_inf=1e-10, protocol="ink", ccd=int(ccd), max_newton=200)
    a1, a2, ia = solvers.solve_ink(*_args(p), tol=1e-10, ccd=ccd)
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["e_corr"] - ia.e_corr) < 1e-9
    assert np.abs(host(t2) - a2).max() < 1e-8
    assert info["newton_iters"] == ia.newton_iters and info["n_residual"] == ia.n_residual
    assert info["n_jvp"] == 0


def test_sfp_diis_ccd_matches_the_oracle(handle, lib):
    """SFP+DIIS (level shift 0.2) at the CCD level, far from DIIS's noise
    floor: the same path as the oracle, and t1 stays zero."""
    p = make_problem(3, 7, 14, 97, gauge="canonical")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2, info = handle.solve_fp_diis(P, tol_inf=1e-7, level_shift=0.2, ccd=1)
    a1, a2, ia = solvers.solve_fp_diis(*_args(p), tol=1e-7, level_shift=0.2, ccd=True)
    assert info["status"] == "CC_OK" and ia.converged
    assert not np.any(host(t1))
    assert abs(info["e_corr"] - ia.e_corr) < 1e-8
    assert info["n_residual"] == ia.n_residual


@pytest.mark.parametrize("o,v,naux", [(4, 18, 40), (5, 40, 40)])
def test_timed_solve_matches_untimed(handle, lib, o, v, naux):
    """Timing instrumentation (events around the timed A_F launch of each
    step inside the replayed inner-solve graph, for one inner solve in
    eight) changes nothing in the solve: v = 18 plans 32-wide blocks (the two-launch step, the fused
    launch timed), v = 40 48-wide ones (three launches, the occupied launch
    timed)."""
    p = make_problem(o, v, naux, 53, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    _, _, ref = handle.solve_pnk(P, tol_inf=1e-10)
    handle.timing(True)
    try:
        _, _, got = handle.solve_pnk(P, tol_inf=1e-10)
        n_af, _ = handle.timing_read(3)
    finally:
        handle.timing(False)
    assert ref["status"] == got["status"] == "CC_OK"
    assert got["e_corr"] == ref["e_corr"]
    for k in ("newton_iters", "n_residual", "n_jvp", "n_afmv"):
        assert got[k] == ref[k], k
    assert n_af > 0

def test_pnk_c2_root_is_an_oracle_root(handle, lib):
    """FP64 PNK on the Haar-rotated workload (o=10, v=90, naux=300) to its
    stated stopping test, max |R| < 1e-8. The synthetic Hamiltonian is
    strongly correlated (E_corr near -92 Eh); with pair-symmetric
    preconditioned vectors Newton needs about 20 steps (the cap of 200 only
    guards the test). The GPU's amplitudes must be a root of the oracle's
    residual at ten times the stopping level and give the oracle's energy
    to 1e-9 Eh."""
    p = make_config("c2_haar")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2, info = handle.solve_pnk(P, tol_inf=1e-8, max_newton=200)
    assert info["status"] == "CC_OK", (info, handle.history()[-5:])
    h1, h2 = host(t1), host(t2)
    o1, o2 = ccsd.residual(*_args(p), h1, h2)
    # a root of the oracle's residual at ten times the stopping level: the
    # two residual evaluations differ by rounding, amplified on this
    # strongly correlated workload
    assert max(np.abs(o1).max(), np.abs(o2).max()) < 1e-7
    assert abs(ccsd.energy(*_args(p), h1, h2) - info["e_corr"]) < 1e-9


def test_pnk_mixed_precision_energy(handle, lib):
    p = make_problem(6, 30, 60, 51, gauge="haar")
    P = lib.DeviceProblem.from_problem(p)
    _, _, ref = handle.solve_pnk(P, tol_inf=1e-10)
    for prec in ("fp32", "bf16"):
        t1, t2, info = handle.solve_pnk(P, tol_inf=1e-8, jvp_prec=prec)
        assert info["status"] == "CC_OK", prec
        assert abs(info["e_corr"] - ref["e_corr"]) < 1e-6, prec


@pytest.mark.parametrize("o,v,m,shift", [(2, 3, 27, 0.0), (3, 8, 30, 0.5)])
def test_fp_spectral_radius_matches_the_oracle(handle, lib, o, v, m, shift):
    """cc_fp_spectral_radius against the oracle's Arnoldi from the same
    pair-symmetric start, at the PNK root of a rotated problem: over the
    whole pair-symmetric space (o=2, v=3: 27 dimensions) the radius is
    exact; with 30 steps on o=3, v=8 the leading Ritz values agree."""
    p = make_problem(o, v, 3 * (o + v), 70 + o, gauge="haar")
    a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-11)
    assert ia.converged
    q1, q2 = random_amplitudes(o, v, 80 + o, scale=1.0)
    rho_o, ritz_o = solvers.fp_jacobian_spectral_radius(*_args(p), a1, a2, shift=shift, m=m,
                                                          q0=solvers.pack(q1, q2))
    P = lib.DeviceProblem.from_problem(p)
    rho, ritz = handle.fp_spectral_radius(P, dev(a1), dev(a2), dev(q1), dev(q2), shift=shift, m=m)
    assert abs(rho - rho_o) < 1e-8 * max(1.0, rho_o)
    top_o = np.sort(np.abs(ritz_o))[-3:]
    top = np.sort(np.abs(ritz))[-3:]
    assert np.allclose(top, top_o, rtol=1e-6, atol=1e-10)


@pytest.mark.parametrize("o,v,naux", [(4, 16, 48), (6, 37, 50)])
def test_contraction_flop_count(handle, lib, o, v, naux):
    """cc_diag_contraction_flops (the roofline's algorithmic count) covers
    the symmetry-adapted ladder and the ring products exactly once, stays
    below the nominal count of the unreduced equations plus the T1 part of
    the ladder (2 o^3 v^3), and counts the same tangent products in every
    J v precision."""
    p = make_general(o, v, naux, 700 + v)
    P = lib.DeviceProblem.from_problem(p)
    fr, fj = handle.contraction_flops(P, "fp64")
    _, fj16 = handle.contraction_flops(P, "bf16")
    _, fj32 = handle.contraction_flops(P, "fp32")
    assert fj == fj16 == fj32
    p2, p2m = v * (v + 1) // 2, v * (v - 1) // 2
    ladder = 2 * (o * (o + 1) // 2) * p2 * p2 + 2 * (o * (o - 1) // 2) * p2m * p2m
    ring = 6 * 2 * (o * v) ** 3
    nominal = (2 * o * o * v ** 4 + 12 * o ** 3 * v ** 3 + 4 * o ** 4 * v * v + 8 * naux * o * o * v * v
               + 4 * o * o * v ** 3 + 4 * o ** 3 * v * v)
    assert ladder + ring < fr < nominal + 2 * o ** 3 * v ** 3
    # the tangent of every product with a varying operand: at least the
    # residual's amplitude-dependent products once
    assert fj > ladder + ring
