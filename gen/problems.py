"""Seeded synthetic closed-shell Hamiltonians in density-fitted form.

This module only draws inputs. It holds none of the coupled-cluster
arithmetic: it returns Fock blocks f_oo, f_ov, f_vv and density-fitting
factors L[P][p][q] (symmetric in p, q) such that the two-electron integrals
are (pq|rs) = sum_P L[P][p][q] L[P][r][s]. Both the CPU oracle and the GPU
path read the same arrays, so neither side needs its own random numbers.

Orbital gauges. A gauge change is an orthogonal transformation of the
orbitals within the occupied and within the virtual space, f -> U f U^T,
L^P -> U L^P U^T (the Fock transformation of the random-gauge appendix).
The Haar-random orthogonal matrices come from the QR factorisation of a
Gaussian matrix with the signs of R's diagonal folded into Q (Mezzadri,
Notices AMS 54 (2007) 592).

Draw order for one problem: occupied orbital energies, virtual orbital
energies, the DF factors, then the occupied and the virtual rotation.
"""

from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """One closed-shell problem. All arrays are float64, C-contiguous."""

    f_oo: np.ndarray  # [o][o]
    f_ov: np.ndarray  # [o][v]
    f_vv: np.ndarray  # [v][v]
    L: np.ndarray  # [naux][n][n], L[P] symmetric
    meta: dict = field(default_factory=dict)

    @property
    def nocc(self) -> int:
        return self.f_oo.shape[0]

    @property
    def nvir(self) -> int:
        return self.f_vv.shape[0]

    @property
    def naux(self) -> int:
        return self.L.shape[0]

    def fock(self) -> np.ndarray:
        """Full n x n Fock matrix assembled from the three blocks."""
        o, v = self.nocc, self.nvir
        f = np.zeros((o + v, o + v))
        f[:o, :o] = self.f_oo
        f[:o, o:] = self.f_ov
        f[o:, :o] = self.f_ov.T
        f[o:, o:] = self.f_vv
        return f


def haar_orthogonal(rng: np.random.Generator, m: int) -> np.ndarray:
    """Haar-distributed m x m orthogonal matrix (QR with sign fix)."""
    if m == 0:
        return np.zeros((0, 0))
    z = rng.standard_normal((m, m))
    q, r = np.linalg.qr(z)
    d = np.sign(np.diag(r))
    d[d == 0] = 1.0
    return q * d[None, :]


def symmetric_df_factors(rng: np.random.Generator, naux: int, n: int,
                         sigma: float) -> np.ndarray:
    """naux symmetric n x n matrices: upper triangle (with the diagonal)
    i.i.d. N(0, sigma^2), mirrored into the lower triangle."""
    L = np.zeros((naux, n, n))
    iu = np.triu_indices(n)
    L[:, iu[0], iu[1]] = sigma * rng.standard_normal((naux, iu[0].size))
    L = L + np.transpose(L, (0, 2, 1))
    idx = np.arange(n)
    L[:, idx, idx] *= 0.5
    return np.ascontiguousarray(L)


def _rotate(f_oo, f_vv, L, U_o, U_v):
    o = f_oo.shape[0]
    n = L.shape[1]
    U = np.zeros((n, n))
    U[:o, :o] = U_o
    U[o:, o:] = U_v
    f_oo = U_o @ f_oo @ U_o.T
    f_vv = U_v @ f_vv @ U_v.T
    L = np.einsum("pr,Prs,qs->Ppq", U, L, U, optimize=True)
    # restore exact symmetry lost to rounding
    f_oo = 0.5 * (f_oo + f_oo.T)
    f_vv = 0.5 * (f_vv + f_vv.T)
    L = 0.5 * (L + np.transpose(L, (0, 2, 1)))
    return f_oo, f_vv, np.ascontiguousarray(L)


def make_problem(nocc: int, nvir: int, naux: int, seed: int, *,
                 sigma: float = 0.05, gauge: str = "canonical",
                 occ_range=(-1.5, -0.5), vir_range=(0.3, 2.5)) -> Problem:
    """Diagonal-Fock problem, optionally Haar-rotated within the occupied
    and within the virtual block (gauge='haar')."""
    rng = np.random.default_rng(seed)
    eps_o = np.sort(rng.uniform(occ_range[0], occ_range[1], nocc))
    eps_v = np.sort(rng.uniform(vir_range[0], vir_range[1], nvir))
    n = nocc + nvir
    L = symmetric_df_factors(rng, naux, n, sigma)
    f_oo = np.diag(eps_o)
    f_vv = np.diag(eps_v)
    if gauge == "haar":
        U_o = haar_orthogonal(rng, nocc)
        U_v = haar_orthogonal(rng, nvir)
        f_oo, f_vv, L = _rotate(f_oo, f_vv, L, U_o, U_v)
    elif gauge != "canonical":
        raise ValueError(f"unknown gauge {gauge!r}")
    return Problem(np.ascontiguousarray(f_oo), np.zeros((nocc, nvir)),
                   np.ascontiguousarray(f_vv), L,
                   dict(nocc=nocc, nvir=nvir, naux=naux, seed=seed,
                        sigma=sigma, gauge=gauge))


def make_near_degenerate(nocc: int, nvir: int, naux: int, seed: int, *,
                         sigma: float = 0.08, gap: float = 0.05,
                         window: float = 0.1) -> Problem:
    """HOMO-LUMO gap `gap` around a Fermi level at 0; HOMO-1 and LUMO+1
    drawn within `window` of it; the rest as in make_problem. The gauge is
    rotated only within {HOMO-1, HOMO} and within {LUMO, LUMO+1}."""
    rng = np.random.default_rng(seed)
    eps_o = np.sort(rng.uniform(-1.5, -0.5, nocc))
    eps_v = np.sort(rng.uniform(0.3, 2.5, nvir))
    half = 0.5 * gap
    if nocc >= 2:
        eps_o[-2] = rng.uniform(-window, -half)
    eps_o[-1] = -half
    eps_v[0] = half
    if nvir >= 2:
        eps_v[1] = rng.uniform(half, window)
    eps_o = np.sort(eps_o)
    eps_v = np.sort(eps_v)
    n = nocc + nvir
    L = symmetric_df_factors(rng, naux, n, sigma)
    U_o = np.eye(nocc)
    U_v = np.eye(nvir)
    if nocc >= 2:
        U_o[-2:, -2:] = haar_orthogonal(rng, 2)
    if nvir >= 2:
        U_v[:2, :2] = haar_orthogonal(rng, 2)
    f_oo, f_vv, L = _rotate(np.diag(eps_o), np.diag(eps_v), L, U_o, U_v)
    return Problem(np.ascontiguousarray(f_oo), np.zeros((nocc, nvir)),
                   np.ascontiguousarray(f_vv), L,
                   dict(nocc=nocc, nvir=nvir, naux=naux, seed=seed,
                        sigma=sigma, gauge="frontier", gap=gap))


def make_general(nocc: int, nvir: int, naux: int, seed: int, *,
                 sigma: float = 0.1, fov_scale: float = 0.05) -> Problem:
    """Small test problem with a dense symmetric Fock matrix that has a
    nonzero occupied-virtual block (a non-Brillouin reference)."""
    rng = np.random.default_rng(seed)
    o, v = nocc, nvir
    n = o + v
    eps = np.concatenate([np.sort(rng.uniform(-1.5, -0.5, o)),
                          np.sort(rng.uniform(0.3, 2.5, v))])
    f = np.diag(eps)
    g = 0.05 * rng.standard_normal((n, n))
    g = 0.5 * (g + g.T)
    f = f + g
    f[:o, o:] = fov_scale * rng.standard_normal((o, v))
    f[o:, :o] = f[:o, o:].T
    L = symmetric_df_factors(rng, naux, n, sigma)
    return Problem(np.ascontiguousarray(f[:o, :o]), np.ascontiguousarray(f[:o, o:]),
                   np.ascontiguousarray(f[o:, o:]), L,
                   dict(nocc=o, nvir=v, naux=naux, seed=seed, sigma=sigma,
                        gauge="general"))


def nonorthogonal_gauge(nocc: int, nvir: int, seed: int, cond: float = 4.0):
    """Invertible, non-orthogonal gauge matrices W_o [o][o] and W_v [v][v]:
    Q1 diag(s) Q2 with Haar Q1, Q2 and singular values s = cond^u, u
    uniform on [-1/2, 1/2] with the two ends always drawn, so each block's
    condition number is `cond` (1 gives an orthogonal gauge). Column mu of
    W holds the expansion of gauge function mu in the orthonormal orbitals
    of its block; the gauge functions overlap as S = W^T W."""
    rng = np.random.default_rng(seed)
    out = []
    for m in (nocc, nvir):
        u = rng.uniform(-0.5, 0.5, m)
        if m >= 2:
            u[0], u[1] = -0.5, 0.5
        s = cond ** u
        q1 = haar_orthogonal(rng, m)
        q2 = haar_orthogonal(rng, m)
        out.append(np.ascontiguousarray((q1 * s[None, :]) @ q2))
    return out[0], out[1]


def redundant_gauge(nocc: int, nvir: int, m_occ: int, m_vir: int, seed: int, cond: float = 4.0):
    """Redundant gauge matrices W_o [o][m_occ] and W_v [v][m_vir] (m >= the
    block size): m gauge functions spanning each block, as projected atomic
    orbitals span the virtual space. W = Q1 [diag(s) 0] Q2 with Haar Q1
    (n x n) and Q2 (m x m) and nonzero singular values s = cond^u, u uniform
    on [-1/2, 1/2] with both ends drawn: full row rank, the nonzero part with
    condition number `cond`; the overlap S = W^T W has rank n."""
    rng = np.random.default_rng(seed)
    out = []
    for n, m in ((nocc, m_occ), (nvir, m_vir)):
        if m < n:
            raise ValueError("a gauge needs at least as many functions as the block has orbitals")
        u = rng.uniform(-0.5, 0.5, n)
        if n >= 2:
            u[0], u[1] = -0.5, 0.5
        s = cond ** u
        q1 = haar_orthogonal(rng, n)
        q2 = haar_orthogonal(rng, m)
        out.append(np.ascontiguousarray((q1 * s[None, :]) @ q2[:n, :]))
    return out[0], out[1]


def random_amplitudes(nocc: int, nvir: int, seed: int, scale: float = 0.05):
    """Random t1 [o][v] and pair-symmetric t2 [o][o][v][v] (t_ij^ab = t_ji^ba)."""
    rng = np.random.default_rng(seed)
    t1 = scale * rng.standard_normal((nocc, nvir))
    t2 = scale * rng.standard_normal((nocc, nocc, nvir, nvir))
    t2 = 0.5 * (t2 + np.transpose(t2, (1, 0, 3, 2)))
    return t1, np.ascontiguousarray(t2)


# The five workloads the solver is measured on, by name.
CONFIGS = {
    # canonical gauge, FP64, FP and PNK to ||R||_inf < 1e-10
    "c1_canonical": dict(kind="plain", nocc=4, nvir=16, naux=48, seed=1001,
                         sigma=0.05, gauge="canonical", tol=1e-10),
    # Haar-rotated occupied/virtual blocks, PNK vs FP+DIIS(8) to 1e-8
    "c2_haar": dict(kind="plain", nocc=10, nvir=90, naux=300, seed=1002,
                    sigma=0.05, gauge="haar", tol=1e-8),
    # near-degenerate frontier levels, sigma 0.08
    "c3_neardeg": dict(kind="neardeg", nocc=16, nvir=144, naux=480, seed=1003,
                       sigma=0.08, tol=1e-8),
    # mixed-precision PNK, Haar gauge
    "c4_mixed": dict(kind="plain", nocc=20, nvir=180, naux=600, seed=1004,
                     sigma=0.05, gauge="haar", tol=1e-8),
}

# Non-orthogonal gauge workload: the C2 Hamiltonian (Haar-rotated orbitals)
# solved for the amplitudes in a gauge of condition number `cond` per block.
GAUGE_WORKLOAD = dict(config="c2_haar", gauge_seed=2002, cond=4.0)


def make_config(name: str) -> Problem:
    c = dict(CONFIGS[name])
    kind = c.pop("kind")
    tol = c.pop("tol")
    if kind == "plain":
        p = make_problem(c["nocc"], c["nvir"], c["naux"], c["seed"],
                         sigma=c["sigma"], gauge=c["gauge"])
    else:
        p = make_near_degenerate(c["nocc"], c["nvir"], c["naux"], c["seed"],
                                 sigma=c["sigma"])
    p.meta["tol"] = tol
    p.meta["config"] = name
    return p


def serving_request_shapes(n_requests: int, base_seed: int = 5000):
    """Shapes of the serving stream: nocc ~ U{4..16}, nvir = nocc * U{5..9},
    naux = 3 (nocc + nvir), alternating canonical / Haar gauges."""
    out = []
    for rid in range(n_requests):
        rng = np.random.default_rng(base_seed + rid)
        o = int(rng.integers(4, 17))
        v = o * int(rng.integers(5, 10))
        out.append(dict(rid=rid, nocc=o, nvir=v, naux=3 * (o + v),
                        seed=base_seed + rid,
                        gauge="canonical" if rid % 2 == 0 else "haar"))
    return out


def make_serving_request(shape: dict) -> Problem:
    p = make_problem(shape["nocc"], shape["nvir"], shape["naux"],
                     shape["seed"] + 100000, sigma=0.05, gauge=shape["gauge"])
    p.meta["rid"] = shape["rid"]
    return p


def poisson_arrivals(n_requests: int, rate: float, seed: int = 4242) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n_requests))
