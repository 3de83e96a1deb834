"""The seeded input generators (CPU): shapes, symmetries and distributions
of the synthetic workloads, which both the oracle and the GPU path read."""

import numpy as np

from gen import CONFIGS, make_config, make_general, make_problem, random_amplitudes
from gen.problems import haar_orthogonal, poisson_arrivals, serving_request_shapes, symmetric_df_factors


def test_df_factors_are_symmetric_with_the_stated_spread():
    rng = np.random.default_rng(3)
    L = symmetric_df_factors(rng, 40, 30, 0.05)
    assert np.array_equal(L, np.transpose(L, (0, 2, 1)))
    iu = np.triu_indices(30)
    up = L[:, iu[0], iu[1]]
    assert abs(up.std() - 0.05) < 0.002 and abs(up.mean()) < 0.002


def test_haar_matrices_are_orthogonal_and_seeded():
    U = haar_orthogonal(np.random.default_rng(1), 17)
    assert np.abs(U @ U.T - np.eye(17)).max() < 1e-13
    assert np.array_equal(U, haar_orthogonal(np.random.default_rng(1), 17))


def test_rotated_gauge_keeps_the_spectrum_and_the_integrals():
    a = make_problem(4, 11, 20, 9, gauge="canonical")
    b = make_problem(4, 11, 20, 9, gauge="haar")
    assert np.allclose(np.linalg.eigvalsh(b.f_oo), np.diag(a.f_oo))
    assert np.allclose(np.linalg.eigvalsh(b.f_vv), np.diag(a.f_vv))
    assert np.abs(b.f_oo - np.diag(np.diag(b.f_oo))).max() > 1e-3  # dense off-diagonal
    assert np.array_equal(b.f_ov, np.zeros((4, 11)))
    # (pq|rs) summed over all orbitals is invariant under the block rotation
    ga = np.einsum("Ppp,Pqq->", a.L[:, :4, :4], a.L[:, :4, :4])
    gb = np.einsum("Ppp,Pqq->", b.L[:, :4, :4], b.L[:, :4, :4])
    assert abs(ga - gb) < 1e-12 * max(1.0, abs(ga))


def test_configs_have_the_stated_shapes_and_tolerances():
    shapes = {"c1_canonical": (4, 16, 48, 1e-10), "c2_haar": (10, 90, 300, 1e-8),
              "c3_neardeg": (16, 144, 480, 1e-8), "c4_mixed": (20, 180, 600, 1e-8)}
    for name, (o, v, naux, tol) in shapes.items():
        c = CONFIGS[name]
        assert (c["nocc"], c["nvir"], c["naux"], c["tol"]) == (o, v, naux, tol)
    p = make_config("c1_canonical")
    assert p.f_oo.shape == (4, 4) and p.L.shape == (48, 20, 20)
    assert np.all(np.diag(p.f_oo) >= -1.5) and np.all(np.diag(p.f_oo) <= -0.5)
    assert np.all(np.diag(p.f_vv) >= 0.3) and np.all(np.diag(p.f_vv) <= 2.5)


def test_general_problem_has_occupied_virtual_coupling():
    p = make_general(3, 7, 10, 4)
    assert np.abs(p.f_ov).max() > 0
    assert np.array_equal(p.f_oo, p.f_oo.T) and np.array_equal(p.f_vv, p.f_vv.T)


def test_random_amplitudes_are_pair_symmetric():
    t1, t2 = random_amplitudes(3, 5, 2)
    assert t1.shape == (3, 5) and t2.shape == (3, 3, 5, 5)
    assert np.array_equal(t2, np.transpose(t2, (1, 0, 3, 2)))


def test_serving_stream_shapes_and_arrivals():
    shapes = serving_request_shapes(200)
    for s in shapes:
        o, v = s["nocc"], s["nvir"]
        assert 4 <= o <= 16 and v % o == 0 and 5 <= v // o <= 9
        assert s["naux"] == 3 * (o + v)
        assert s["gauge"] == ("canonical" if s["rid"] % 2 == 0 else "haar")
    assert len({s["nocc"] for s in shapes}) == 13
    t = poisson_arrivals(2000, 4.0)
    assert np.all(np.diff(t) > 0)
    assert abs(t[-1] / 2000 - 0.25) < 0.02  # mean gap 1 / rate
