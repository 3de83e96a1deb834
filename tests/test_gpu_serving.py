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


def test_serving_reuses_cached_handles_with_identical_results(lib):
    """Requests of one shape and precision take over the handle a finished
    one left (integral workspace, recorded graphs): the results are still
    bit for bit those of solo solves, and the cache's memory stays inside
    the budget."""
    shapes = [(4, 20, "haar", "fp64"), (4, 20, "canonical", "fp64"), (4, 20, "haar", "bf16"),
              (4, 20, "haar", "fp64"), (4, 20, "haar", "bf16"), (5, 25, "haar", "fp64")]
    probs = [make_problem(o, v, 3 * (o + v), 7100 + k, gauge=g) for k, (o, v, g, _) in enumerate(shapes)]
    h = lib.Handle(0)
    solo = []
    for p, (_, _, _, prec) in zip(probs, shapes):
        t1, t2, info = h.solve_pnk(lib.DeviceProblem.from_problem(p), tol_inf=TOL, jvp_prec=prec)
        solo.append((t1.cpu().numpy(), t2.cpu().numpy(), info))
    h.close()
    foot = max(_footprint(lib, p.nocc, p.nvir, p.naux, prec) for p, (_, _, _, prec) in zip(probs, shapes))
    srv = lib.Server(0, mem_budget=3 * foot, max_slots=1)  # one slot: each request follows the previous one
    try:
        res = []
        for p, (_, _, _, prec) in zip(probs, shapes):
            rid = srv.submit(p, tol_inf=TOL, jvp_prec=prec)
            srv.drain()
            res.append(srv.poll(rid))
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["handle_reuses"] >= 3, stats
    assert stats["peak_bytes"] <= 3 * foot
    assert stats["cached_bytes"] <= stats["bytes_in_use"] <= 3 * foot
    for r, (s1, s2, sinfo) in zip(res, solo):
        assert r["status"] == "CC_OK"
        assert r["e_corr"] == sinfo["e_corr"]
        assert np.array_equal(r["t1"], s1) and np.array_equal(r["t2"], s2)


def test_serving_host_memory_is_released(lib):
    """Once a request has finished only its results are held on the host
    (its input copies are dropped), and once collected nothing is held; a
    collected request cannot be polled again but its times remain."""
    probs = _problems()[:4]
    srv = lib.Server(0, max_slots=2)
    try:
        ids = [srv.submit(p, tol_inf=1e-8) for p in probs]
        srv.drain()
        st = srv.stats()
        results = sum(8 * (p.nocc * p.nvir + (p.nocc * p.nvir) ** 2) for p in probs)
        assert st["requests_held"] == len(probs)
        assert st["host_bytes_held"] == results, (st["host_bytes_held"], results)
        for i in ids:
            assert srv.poll(i, want_amplitudes=False)["status"] == "CC_OK"
        st = srv.stats()
        assert st["requests_held"] == 0 and st["host_bytes_held"] == 0
        with pytest.raises(lib.CCError):
            srv.poll(ids[0])
        t_sub, t_adm, t_fin = srv.times(ids[0])
        assert 0.0 <= t_sub <= t_adm <= t_fin
    finally:
        srv.close()


def test_server_rejects_a_request_larger_than_the_budget(lib):
    """A request whose footprint exceeds the whole budget can never run: it
    is refused at submission with CC_ERR_REJECTED (nothing is queued)."""
    p = make_problem(4, 20, 72, 7200, gauge="haar")
    srv = lib.Server(0, mem_budget=1 << 20, max_slots=2)
    try:
        with pytest.raises(lib.CCError) as err:
            srv.submit(p)
        assert err.value.status == -5  # CC_ERR_REJECTED
        st = srv.stats()
        assert st["rejected"] == 1 and st["queued"] == 0 and st["finished"] == 0
    finally:
        srv.close()


def test_serving_c5_sized_requests_match_solo_solves_and_fp64(lib):
    """Requests of the serving stream's larger shapes (o = 8..12, v = 5..9
    times o, naux = 3(o + v), canonical and rotated gauges), FP64 and
    mixed precision (BF16 J v with the Krylov-loop inner solves to 1e-6, as
    the stream runs them), three in flight: every result is bit for bit the
    same request solved alone on a handle, and each mixed-precision energy
    is within 1e-6 Eh of the FP64 one."""
    shapes = [(8, 40, "haar"), (10, 70, "canonical"), (12, 60, "haar"), (9, 54, "canonical")]
    probs = [make_problem(o, v, 3 * (o + v), 7300 + k, gauge=g) for k, (o, v, g) in enumerate(shapes)]
    kinds = [dict(jvp_prec="fp64"), dict(jvp_prec="bf16", inner_rtol_jv=1e-6)]
    h = lib.Handle(0)
    solo = {}
    for k, p in enumerate(probs):
        for j, kw in enumerate(kinds):
            t1, t2, info = h.solve_pnk(lib.DeviceProblem.from_problem(p), tol_inf=1e-8, max_newton=200, **kw)
            assert info["status"] == "CC_OK", (k, kw, info)
            solo[(k, j)] = (t1.cpu().numpy(), t2.cpu().numpy(), info)
    h.close()
    srv = lib.Server(0, max_slots=3)
    try:
        ids = {(k, j): srv.submit(p, tol_inf=1e-8, max_newton=200, **kw)
               for k, p in enumerate(probs) for j, kw in enumerate(kinds)}
        srv.drain()
        res = {key: srv.poll(rid) for key, rid in ids.items()}
        stats = srv.stats()
    finally:
        srv.close()
    assert stats["peak_running"] >= 2
    for key, r in res.items():
        s1, s2, sinfo = solo[key]
        assert r["status"] == "CC_OK", key
        assert r["e_corr"] == sinfo["e_corr"], key
        assert np.array_equal(r["t1"], s1) and np.array_equal(r["t2"], s2), key
    for k in range(len(probs)):
        assert abs(res[(k, 1)]["e_corr"] - res[(k, 0)]["e_corr"]) <= 1e-6, k
