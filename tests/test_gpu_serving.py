"""GPU serving loop (cc_server_*): continuous batching of PNK solves.

Checks, on a small mixed stream (FP64 and BF16 J v, canonical and rotated
gauges, uneven sizes):
- every result equals the same request solved alone on a handle (the
  kernels are deterministic, so equality is exact), and the FP64 ones agree
  with the oracle;
- admission never exceeds the memory budget, and requests do overlap;
- submit <= admit <= finish times are recorded for every request.
"""

import numpy as np
import pytest

from gen import make_problem
from oracle import solvers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    import paper_2608_06669_amd as pk
    pk.load()
    assert torch.cuda.is_available(), "a GPU is required"
    return pk


# (nocc, nvir, gauge, J v precision)
STREAM = [(3, 15, "canonical", "fp64"), (4, 20, "haar", "bf16"), (5, 25, "haar", "fp64"),
          (3, 18, "haar", "bf16"), (4, 24, "canonical", "fp32"), (5, 20, "canonical", "bf16"),
          (4, 16, "haar", "fp64"), (3, 21, "canonical", "fp32")]
TOL = 1e-9


def _problems():
    return [make_problem(o, v, 3 * (o + v), 7000 + k, gauge=g) for k, (o, v, g, _) in enumerate(STREAM)]


def _footprint(lib, o, v, naux, prec):
    lowp = {"fp64": 0, "fp32": 1, "bf16": 2}[prec]
    problem = 8 * (o * o + o * v + v * v + naux * (o + v) ** 2)
    return lib.workspace_bytes(o, v, naux, lowp, 20, 30, 0) + problem + (1 << 20)


def test_serving_matches_solo_solves_and_respects_the_budget(lib):
    probs = _problems()
    h = lib.Handle(0)
    solo = []
    for p, (_, _, _, prec) in zip(probs, STREAM):
        t1, t2, info = h.solve_pnk(lib.DeviceProblem.from_problem(p), tol_inf=TOL, jvp_prec=prec)
        assert info["status"] == "CC_OK"
        solo.append((t1.cpu().numpy(), t2.cpu().numpy(), info))
    h.close()

    foot = [_footprint(lib, p.nocc, p.nvir, p.naux, prec) for p, (_, _, _, prec) in zip(probs, STREAM)]
    budget = int(2.5 * max(foot))  # two or three requests fit at a time
    srv = lib.Server(0, mem_budget=budget, max_slots=4)
    try:
        ids = [srv.submit(p, tol_inf=TOL, jvp_prec=prec) for p, (_, _, _, prec) in zip(probs, STREAM)]
        srv.drain()
        res = [srv.poll(i) for i in ids]
        stats = srv.stats()
        times = [srv.times(i) for i in ids]
    finally:
        srv.close()

    assert stats["finished"] == len(STREAM) and stats["rejected"] == 0
    assert stats["peak_bytes"] <= budget
    assert 2 <= stats["peak_running"] <= 4, stats
    for (t_sub, t_adm, t_fin) in times:
        assert 0.0 <= t_sub <= t_adm <= t_fin
    for r, (s1, s2, sinfo) in zip(res, solo):
        assert r["status"] == "CC_OK"
        assert r["e_corr"] == sinfo["e_corr"]
        assert r["n_jvp"] == sinfo["n_jvp"] and r["newton_iters"] == sinfo["newton_iters"]
        assert np.array_equal(r["t1"], s1) and np.array_equal(r["t2"], s2)


def test_serving_results_match_the_oracle(lib):
    """FP64 requests against the oracle's PNK energy (1e-9 Eh); mixed
    precision requests within 1e-6 Eh of it."""
    probs = _problems()
    srv = lib.Server(0, max_slots=3)
    try:
        ids = [srv.submit(p, tol_inf=1e-10, jvp_prec=prec) for p, (_, _, _, prec) in zip(probs, STREAM)]
        srv.drain()
        res = [srv.poll(i, want_amplitudes=False) for i in ids]
    finally:
        srv.close()
    for k in (0, 1, 4):  # one of each precision
        p = probs[k]
        _, _, ref = solvers.solve_pnk(p.f_oo, p.f_ov, p.f_vv, p.L, tol=1e-11)
        tol = 1e-9 if STREAM[k][3] == "fp64" else 1e-6
        assert res[k]["status"] == "CC_OK"
        assert abs(res[k]["e_corr"] - ref.e_corr) < tol, (k, res[k]["e_corr"], ref.e_corr)
