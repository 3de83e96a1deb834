"""CPU checks of the C boundary: the library loads and exports every entry
point the public header declares (no compute calls without a GPU)."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnkcc.h")
LIB = os.path.join(ROOT, "paper_2608_06669_amd", "libpnkcc.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(cc_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_solver_entry_points():
    names = declared_functions()
    for n in ["cc_residual", "cc_jvp", "cc_precond_solve", "cc_solve_pnk", "cc_solve_fp_diis",
              "cc_server_create", "cc_server_submit", "cc_server_poll"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_signatures_cover_the_header():
    from paper_2608_06669_amd import _lib
    assert set(declared_functions()) == set(_lib.SIGNATURES)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_workspace_size_query_and_option_defaults():
    from paper_2608_06669_amd import _lib
    lib = _lib.load()
    small = lib.cc_workspace_bytes(4, 16, 48, 0, 20, 30, 0)
    assert small > 0
    # the (ac|bd) tensor alone is nvir^4 doubles
    assert lib.cc_workspace_bytes(20, 180, 600, 0, 20, 30, 0) > 8 * 180 ** 4
    assert lib.cc_workspace_bytes(20, 180, 600, 2, 20, 30, 0) > lib.cc_workspace_bytes(20, 180, 600, 0, 20, 30, 0)
    assert lib.cc_workspace_bytes(0, 16, 48, 0, 20, 30, 0) == 0
    o = _lib.cc_pnk_opts()
    lib.cc_pnk_opts_default(ctypes.byref(o))
    assert (o.tol_inf, o.m_max, o.gamma, o.alpha, o.inner_restart) == (1e-8, 20, 0.9, 1.5, 30)
    f = _lib.cc_fp_opts()
    lib.cc_fp_opts_default(ctypes.byref(f))
    assert (f.diis_size, f.diis_start, f.level_shift) == (8, 2, 0.0)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_null_arguments_are_rejected_without_a_device():
    from paper_2608_06669_amd import _lib
    lib = _lib.load()
    assert lib.cc_residual(None, None, None, None, None, None, None, None) == _lib.CC_ERR_ARG
    assert lib.cc_create(None, 0, 0) == _lib.CC_ERR_ARG
    assert lib.cc_server_submit(None, None, None, None) == _lib.CC_ERR_ARG
    assert lib.cc_diag_gemm(0, 1, 1, None, 0, 0, None, 0, 0, None, 0, 0, 1.0, 0.0, 0, None) == _lib.CC_ERR_ARG


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_host_hessenberg_eigenvalues_match_numpy():
    """The host QR iteration behind cc_fp_spectral_radius (runs without a
    GPU) against numpy's eigenvalues: random Hessenberg matrices with real
    and complex spectra, a rotation with a purely imaginary pair, a zero
    matrix, a 1 x 1 case and a Jordan-like block."""
    import numpy as np

    import paper_2608_06669_amd as pk
    rng = np.random.default_rng(7)
    cases = [np.triu(rng.standard_normal((m, m)), -1) for m in (2, 3, 5, 12, 30, 60)]
    cases.append(np.array([[0.0, 1.0], [-1.0, 0.0]]))
    cases.append(np.zeros((4, 4)))
    cases.append(np.array([[2.5]]))
    cases.append(np.diag(np.full(5, 0.3)) + np.diag(np.ones(4), 1) + np.diag(np.full(4, 1e-3), -1))
    for H in cases:
        got = pk.hessenberg_eigenvalues(H)
        ref = np.linalg.eigvals(H)
        scale = max(1.0, np.abs(H).max())
        # match each reference eigenvalue to its nearest computed one
        for lam in ref:
            assert np.min(np.abs(got - lam)) < 1e-9 * scale * H.shape[0], (H.shape, lam)
        assert abs(np.max(np.abs(got)) - np.max(np.abs(ref))) < 1e-9 * scale * H.shape[0]


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_occupied_kernel_position_sets_cover_every_pair_once():
    """The occupied A_F kernel's position sets (cc_diag_occ_sets, host
    code): every (a, b) with a, b < v lies in exactly one lane of one set,
    each lane's partner lane holds (b, a), and the set count is nb^2 (nb =
    ceil(v / 8) blocks per side) less one per block paired with a last
    block that the grid leaves at most 4 elements into (nb odd): 507 sets
    at v = 180, 144 at v = 90."""
    import numpy as np

    import paper_2608_06669_amd as pk
    for v in list(range(1, 41)) + [57, 90, 91, 96, 100, 144, 172, 180, 181, 185]:
        a, b, lt = pk.occ_sets(v)
        nb = -(-v // 8)
        edge = nb % 2 == 1 and v - 8 * (nb - 1) <= 4
        assert a.shape[0] == nb * nb - (nb - 1 if edge else 0), v
        rows = np.arange(a.shape[0])[:, None]
        assert np.array_equal(a[rows, lt], b) and np.array_equal(b[rows, lt], a), v
        valid = (a < v) & (b < v)
        cover = np.zeros((v, v), dtype=np.int64)
        np.add.at(cover, (a[valid], b[valid]), 1)
        assert (cover == 1).all(), v
    assert pk.occ_sets(180)[0].shape[0] == 507 and pk.occ_sets(90)[0].shape[0] == 144
