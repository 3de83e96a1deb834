"""GPU parity in non-orthogonal gauges: the gauge entry points of the C
boundary against the oracle's random-gauge equations (oracle.gauge).

Tolerances (FP64): the transforms are four short contractions (depth o or
v) with entries of size cond(W); both sides sum in float64 in different
orders, so we allow 1e-12 relative to the largest output. Residuals and J v
add the orbital-basis residual's 1e-10 relative bound, amplified at most by
cond(W)^4 / cond(W)^0 between the back and the forward transform; with
cond(W) = 4 we allow 1e-9 relative. Solves compare what is unique: the root
(to the stopping tolerance, amplified by the same factor) and the energy.
"""

import numpy as np
import pytest

from gen import make_config, make_general, make_problem, nonorthogonal_gauge, random_amplitudes
from oracle import gauge, solvers

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


def _rel(a, b):
    return np.abs(a - b).max() / max(1.0, np.abs(b).max())


# o, v span one and several matrix-core tiles with ragged edges
SHAPES = [(1, 1, 3), (3, 7, 14), (5, 37, 40), (6, 70, 50)]


@pytest.mark.parametrize("o,v,naux", SHAPES)
def test_gauge_transform_matches_the_oracle(handle, lib, o, v, naux):
    p = make_general(o, v, naux, 300 + v)
    Wo, Wv = nonorthogonal_gauge(o, v, 400 + v, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    x1, x2 = random_amplitudes(o, v, 500 + v, scale=0.3)
    y1, y2 = handle.gauge_transform(P, G, dev(x1), dev(x2), to_gauge=True)
    e1, e2 = gauge.forward(Wo, Wv, x1, x2)
    assert _rel(host(y1), e1) < 1e-12 and _rel(host(y2), e2) < 1e-12
    z1, z2 = handle.gauge_transform(P, G, dev(x1), dev(x2), to_gauge=False)
    b1, b2 = gauge.backward(Wo, Wv, x1, x2)
    assert _rel(host(z1), b1) < 1e-11 and _rel(host(z2), b2) < 1e-11


@pytest.mark.parametrize("o,v,naux", SHAPES)
def test_gauge_residual_and_energy_match_the_oracle(handle, lib, o, v, naux):
    """CCSD with f_ov != 0 and random gauge amplitudes."""
    p = make_general(o, v, naux, 310 + v)
    Wo, Wv = nonorthogonal_gauge(o, v, 410 + v, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    th1, th2 = random_amplitudes(o, v, 510 + v, scale=0.05)
    r1, r2, e = handle.residual_gauge(P, G, dev(th1), dev(th2), energy=True)
    q1, q2 = gauge.residual(*_args(p), Wo, Wv, th1, th2)
    assert _rel(host(r1), q1) < 1e-9 and _rel(host(r2), q2) < 1e-9
    assert abs(e - gauge.energy(*_args(p), Wo, Wv, th1, th2)) < 1e-10 * max(1.0, abs(e))


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-9), ("fp32", 2e-4), ("bf16", 5e-2)])
def test_gauge_jvp_matches_the_oracle(handle, lib, prec, tol):
    o, v, naux = 4, 23, 30
    p = make_general(o, v, naux, 320)
    Wo, Wv = nonorthogonal_gauge(o, v, 420, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    th1, th2 = random_amplitudes(o, v, 520, scale=0.05)
    v1, v2 = random_amplitudes(o, v, 521, scale=1.0)
    y1, y2 = handle.jvp_gauge(P, G, dev(th1), dev(th2), dev(v1), dev(v2), prec=prec)
    j1, j2 = gauge.jvp_complex_step(*_args(p), Wo, Wv, th1, th2, v1, v2)
    scale = max(np.abs(j1).max(), np.abs(j2).max())
    assert np.abs(host(y1) - j1).max() < tol * scale and np.abs(host(y2) - j2).max() < tol * scale


def test_gauge_pnk_matches_the_oracle(handle, lib):
    """PNK on gauge amplitudes: the oracle's iteration (GMRES on the gauge's
    non-symmetric A_F) and the device's (the orbital-basis inner solve
    between the transforms) take the same Newton steps to the same root."""
    p = make_problem(4, 16, 48, 1001, gauge="haar")
    Wo, Wv = nonorthogonal_gauge(4, 16, 2002, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    th1, th2, info = handle.solve_pnk_gauge(P, G, tol_inf=1e-10)
    a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-10, gauge=(Wo, Wv))
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["e_corr"] - ia.e_corr) < 1e-9
    assert np.abs(host(th2) - a2).max() < 1e-8 and np.abs(host(th1) - a1).max() < 1e-8
    assert info["newton_iters"] == ia.newton_iters
    # the same root as the orbital-basis solve, transformed
    b1, b2, ib = solvers.solve_pnk(*_args(p), tol=1e-11)
    c1, c2 = gauge.forward(Wo, Wv, b1, b2)
    assert np.abs(host(th2) - c2).max() < 1e-8
    q1, q2 = gauge.residual(*_args(p), Wo, Wv, host(th1), host(th2))
    assert max(np.abs(q1).max(), np.abs(q2).max()) < 10 * 1e-10


def test_gauge_fp_diis_matches_the_oracle(handle, lib):
    """FP+DIIS with the gauge's diagonal denominators: same root as the
    oracle; plain FP (no DIIS) ends without converging on both sides."""
    p = make_problem(4, 16, 48, 1001, gauge="haar")
    Wo, Wv = nonorthogonal_gauge(4, 16, 2002, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    th1, th2, info = handle.solve_fp_diis_gauge(P, G, tol_inf=1e-9, max_iter=300)
    a1, a2, ia = solvers.solve_fp_diis(*_args(p), tol=1e-9, max_iter=300, gauge=(Wo, Wv))
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["e_corr"] - ia.e_corr) < 1e-8
    assert np.abs(host(th2) - a2).max() < 1e-7
    assert abs(info["newton_iters"] - ia.newton_iters) <= 3
    _, _, info0 = handle.solve_fp_diis_gauge(P, G, tol_inf=1e-9, max_iter=60, diis_size=0)
    _, _, ia0 = solvers.solve_fp_diis(*_args(p), tol=1e-9, max_iter=60, diis_size=0, gauge=(Wo, Wv))
    assert info0["status"] != "CC_OK" and not ia0.converged


@pytest.mark.parametrize("ccd", [False, True])
def test_gauge_protocols_match_the_oracle(handle, lib, ccd):
    """The method table in a cond-4 gauge, at the CCSD and the CCD level: PNK,
    NK and INK on the device against the oracle's same protocols in the same
    gauge (same steps, root and energy)."""
    p = make_problem(3, 7, 14, 97, gauge="haar")
    Wo, Wv = nonorthogonal_gauge(3, 7, 2006, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    cases = {"pnk": ({}, dict()), "nk": ({"max_newton": 200}, dict(precond=False, max_newton=200))}
    for name, (gopt, oopt) in cases.items():
        th1, th2, info = handle.solve_pnk_gauge(P, G, tol_inf=1e-10, protocol=name, ccd=int(ccd), **gopt)
        a1, a2, ia = solvers.solve_pnk(*_args(p), tol=1e-10, ccd=ccd, gauge=(Wo, Wv), **oopt)
        assert info["status"] == "CC_OK" and ia.converged, name
        assert abs(info["e_corr"] - ia.e_corr) < 1e-9, name
        assert np.abs(host(th2) - a2).max() < 1e-8 and np.abs(host(th1) - a1).max() < 1e-8, name
        assert info["newton_iters"] == ia.newton_iters, name
        if ccd:
            assert not np.any(host(th1)), name
    th1, th2, info = handle.solve_pnk_gauge(P, G, tol_inf=1e-10, protocol="ink", ccd=int(ccd), max_newton=200)
    a1, a2, ia = solvers.solve_ink(*_args(p), tol=1e-10, ccd=ccd, gauge=(Wo, Wv))
    assert info["status"] == "CC_OK" and ia.converged
    assert abs(info["e_corr"] - ia.e_corr) < 1e-9
    assert np.abs(host(th2) - a2).max() < 1e-8
    assert info["newton_iters"] == ia.newton_iters and info["n_jvp"] == 0


def test_orthogonal_gauge_solve_equals_the_rotated_problem(handle, lib):
    """With orthogonal W the gauge solve is the orbital solve of the
    Hamiltonian rotated by W^T."""
    p = make_problem(3, 9, 20, 1103, gauge="canonical")
    Wo, Wv = nonorthogonal_gauge(3, 9, 2003, 1.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    th1, th2, info = handle.solve_pnk_gauge(P, G, tol_inf=1e-10)
    o, v = 3, 9
    U = np.zeros((o + v, o + v))
    U[:o, :o], U[o:, o:] = Wo.T, Wv.T
    f = U @ p.fock() @ U.T
    Lr = np.einsum("pr,Prs,qs->Ppq", U, p.L, U)
    Pr = lib.DeviceProblem(f[:o, :o], f[:o, o:], f[o:, o:], Lr)
    t1, t2, info_r = handle.solve_pnk(Pr, tol_inf=1e-10)
    assert info["status"] == info_r["status"] == "CC_OK"
    assert np.abs(host(th2) - host(t2)).max() < 1e-8 and abs(info["e_corr"] - info_r["e_corr"]) < 1e-10


def test_singular_gauge_is_rejected(handle, lib):
    p = make_problem(3, 7, 14, 1104)
    Wo, Wv = nonorthogonal_gauge(3, 7, 2004, 4.0)
    Wv[:, 2] = 0.0
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    t1, t2 = P.zeros_t()
    with pytest.raises(lib.CCError, match="singular"):
        handle.residual_gauge(P, G, t1, t2)


def test_gauge_covariance_at_the_full_c2_size(handle, lib):
    """At o = 10, v = 90, naux = 300 (the Haar workload) and cond(W) = 4:
    the gauge residual at U-bar^(x4) t is U-bar^(x4) r(t) and the energy is
    unchanged (a property at any size; the oracle's transform of sampled
    elements checks the forward map)."""
    p = make_config("c2_haar")
    o, v = p.nocc, p.nvir
    Wo, Wv = nonorthogonal_gauge(o, v, 2002, 4.0)
    P, G = lib.DeviceProblem.from_problem(p), lib.DeviceGauge(Wo, Wv)
    t1, t2 = random_amplitudes(o, v, 530, scale=0.01)
    r1, r2, e = handle.residual(P, dev(t1), dev(t2), energy=True)
    th1, th2 = handle.gauge_transform(P, G, dev(t1), dev(t2), to_gauge=True)
    q1, q2, eg = handle.residual_gauge(P, G, th1, th2, energy=True)
    s1, s2 = handle.gauge_transform(P, G, r1, r2, to_gauge=True)
    assert _rel(host(q2), host(s2)) < 1e-9 and _rel(host(q1), host(s1)) < 1e-9
    assert abs(e - eg) < 1e-10 * max(1.0, abs(e))
    # sampled elements of the forward map against the oracle's formula
    h2 = host(th2)
    rng = np.random.default_rng(7)
    for _ in range(20):
        m, n, lam, sig = rng.integers(0, o), rng.integers(0, o), rng.integers(0, v), rng.integers(0, v)
        ref = np.einsum("i,j,a,b,ijab->", Wo[:, m], Wo[:, n], Wv[:, lam], Wv[:, sig], t2)
        assert abs(h2[m, n, lam, sig] - ref) < 1e-12 * max(1.0, np.abs(h2).max())
