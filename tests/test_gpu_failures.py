"""Failure paths of the C boundary, each forced from the host (no kernel is
made to fault or hang):

- a non-finite Fock element gives CC_ERR_NAN (PNK and FP+DIIS) after a
  bounded amount of work;
- an iteration cap gives CC_NOT_CONVERGED with the last iterate returned;
- the stagnation stop ends a non-converging solve early, by its rule;
- a workspace limit below the problem's needs gives CC_ERR_OOM before any
  allocation;
- invalid options and sizes give CC_ERR_ARG.
"""

import numpy as np
import pytest

from gen import make_config, make_problem

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


def test_nan_in_the_fock_matrix_gives_err_nan(handle, lib):
    p = make_problem(3, 12, 30, 901, gauge="haar")
    p.f_vv[2, 5] = np.nan
    p.f_vv[5, 2] = np.nan
    P = lib.DeviceProblem.from_problem(p)
    _, _, info = handle.solve_pnk(P, tol_inf=1e-8, max_newton=5, inner_maxit=50)
    assert info["status"] == "CC_ERR_NAN", info
    assert not info["converged"] and not np.isfinite(info["res_2"])
    _, _, info = handle.solve_fp_diis(P, tol_inf=1e-8, max_iter=5)
    assert info["status"] == "CC_ERR_NAN", info
    # the handle stays usable
    q = make_problem(3, 12, 30, 902, gauge="haar")
    _, _, ok = handle.solve_pnk(lib.DeviceProblem.from_problem(q), tol_inf=1e-9)
    assert ok["status"] == "CC_OK"


def test_iteration_cap_returns_the_last_iterate(handle, lib):
    """max_newton = 1: CC_NOT_CONVERGED, and the amplitudes returned are the
    iterate whose residual the info reports."""
    p = make_config("c1_canonical")
    P = lib.DeviceProblem.from_problem(p)
    t1, t2, info = handle.solve_pnk(P, tol_inf=1e-12, max_newton=1)
    assert info["status"] == "CC_NOT_CONVERGED" and info["newton_iters"] == 1
    r1, r2 = handle.residual(P, t1, t2)
    rinf = max(float(r1.abs().max()), float(r2.abs().max()))
    assert rinf == pytest.approx(info["res_inf"], rel=1e-12)
    assert rinf > 1e-12
    t1, t2, info = handle.solve_fp_diis(P, tol_inf=1e-12, max_iter=2)
    assert info["status"] == "CC_NOT_CONVERGED" and info["newton_iters"] == 2
    r1, r2 = handle.residual(P, t1, t2)
    assert max(float(r1.abs().max()), float(r2.abs().max())) == pytest.approx(info["res_inf"], rel=1e-12)


def _stall_stop(hist_inf, window, factor):
    """Step at which the stagnation rule stops: the first k with k - k_ref
    >= window, where k_ref is the last step whose ||r||_inf fell below factor
    times the previous reference (step 0 is the first reference)."""
    ref, kref = hist_inf[0], 0
    for k in range(1, len(hist_inf)):
        if hist_inf[k] < factor * ref:
            ref, kref = hist_inf[k], k
        elif k - kref >= window:
            return k
    return None


def test_stagnation_stop_ends_a_stalling_solve_by_its_rule(handle, lib):
    """The near-degenerate o=16/v=144 workload does not converge: ||r||_inf
    drops to about 0.1 within a few Newton steps and stays there. With
    stall_window 4 and factor 0.5 the solve ends as CC_NOT_CONVERGED with
    info.stalled set, at the first step where the rule applied to its own
    residual history says so, far before the cap of 200."""
    p = make_config("c3_neardeg")
    P = lib.DeviceProblem.from_problem(p)
    _, _, info = handle.solve_pnk(P, tol_inf=1e-8, max_newton=200, stall_window=4, stall_factor=0.5)
    hist = handle.history()
    print("||r||_inf:", " ".join(f"{x:.2e}" for x in hist[:, 1]))
    assert info["status"] == "CC_NOT_CONVERGED" and info["stalled"] == 1, info
    k = _stall_stop(list(hist[:, 1]), 4, 0.5)
    assert k is not None and k == len(hist) - 1 == info["newton_iters"], (k, len(hist), info["newton_iters"])
    assert info["newton_iters"] < 40
    # the stop is off by default: the same solve continues past that step
    # along the same path
    _, _, longer = handle.solve_pnk(P, tol_inf=1e-8, max_newton=info["newton_iters"] + 3)
    assert longer["stalled"] == 0 and longer["newton_iters"] == info["newton_iters"] + 3
    assert np.array_equal(handle.history()[: len(hist)], hist)


def test_workspace_limit_gives_err_oom(lib):
    h = lib.Handle(0, workspace_limit=1 << 20)
    try:
        P = lib.DeviceProblem.from_problem(make_config("c1_canonical"))
        with pytest.raises(lib.CCError) as err:
            h.solve_pnk(P, tol_inf=1e-8)
        assert err.value.status == -2  # CC_ERR_OOM
        need = lib.workspace_bytes(4, 16, 48)
        assert need > 1 << 20
    finally:
        h.close()
    h = lib.Handle(0, workspace_limit=lib.workspace_bytes(4, 16, 48) + (8 << 20))
    try:
        _, _, info = h.solve_pnk(lib.DeviceProblem.from_problem(make_config("c1_canonical")), tol_inf=1e-8)
        assert info["status"] == "CC_OK"
    finally:
        h.close()


@pytest.mark.parametrize("opts", [dict(m_max=0), dict(m_max=500), dict(inner_rtol=0.0), dict(eta_max=1.5),
                                  dict(stall_window=-1), dict(stall_window=3, stall_factor=1.5),
                                  dict(jvp_prec="bf16", use_fd_jvp=1)])
def test_invalid_options_give_err_arg(handle, lib, opts):
    P = lib.DeviceProblem.from_problem(make_problem(2, 5, 8, 903))
    with pytest.raises(lib.CCError) as err:
        handle.solve_pnk(P, **opts)
    assert err.value.status == -1  # CC_ERR_ARG
