"""Benchmark: PNK CCSD solves/s on one MI355X.

One step = one complete mixed-precision PNK solve of the o=20/v=180/naux=600
Haar-rotated workload to ||r||_inf < 1e-8: integral preparation (the
symmetry-adapted (ac|bd) tensor from the DF factors), MP2 start, FP64
residuals, J v products in BF16 on the matrix cores with float
accumulation, inner A_F solves, FP64 Arnoldi, Givens and updates, and the
FP64 energy. Every step solves a fresh device copy of the problem, so
nothing derived from the integrals is reused across steps. Inputs are
resident in HBM when the timed region starts.

Prints one JSON line: solves/s, p50/p99 latency of the solves, the energy
difference against an FP64 solve of the same problem (untimed, when the
run's time allows it) and the oracle's residual and energy at the
mixed-precision root. `roofline` is for the residual evaluation (its
matrix-core contractions, FP64): algorithmic flops per residual over its
duration measured with HIP events on its stream during the timed region.
`roofline_inner` is the same for the occupied A_F launch of the inner solve
(HBM bound). Other workloads: --workload c2_haar | c3_neardeg | c4_single |
serving | inner | protocols | levelshift | gauge | residual.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix
BF16_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix
HBM_PEAK_GBS = 8000.0
WORKLOAD = "c2_haar"      # the FP64 solve line (--workload c2_haar)
HEADLINE = "c4_mixed"     # the default line
# Time allowed for the whole default run (20 timed solves, 5 warm-up and the
# host baseline); the untimed FP64 reference
# solve is skipped when it would not fit.
RUN_BUDGET_S = 540.0
# HBM bytes per launch of the fused first kernel of the inner Lanczos step
# (packed pair layout) on this workload, from the rocprofv3 FETCH_SIZE /
# WRITE_SIZE passes in profiles/fock_vir_lz_kernel_c2_haar_counters.md
# (each scaled by the same counter for a copy kernel of known size). None
# when the kernel has changed since the counters were taken.
VIR_LZ_TRAFFIC_BYTES = 33288550
# HBM bytes of one residual evaluation and of one occupied A_F launch on the
# default workload, from the rocprofv3 FETCH_SIZE / WRITE_SIZE passes (each
# scaled by the same counter for a copy of known size) in
# profiles/residual_jvp_c2_c4_mfma_and_hbm_counters.md and
# profiles/fock_occ_set_kernel_c2_c4_counters.md; None when a kernel has
# changed since the counters were taken.
RESIDUAL_TRAFFIC_BYTES = 39757973068
OCC_PACKED_TRAFFIC_BYTES = 276513390


def nominal_residual_flops(o, v, naux):
    """Nominal FP64 flops of one residual evaluation (fixed formula)."""
    return (2 * o * o * v ** 4 + 12 * o ** 3 * v ** 3 + 4 * o ** 4 * v * v + 8 * naux * o * o * v * v
            + 4 * o * o * v ** 3 + 4 * o ** 3 * v * v)


def fock_vir_lz_bytes(o, v):
    """Algorithmic HBM bytes of one launch of the fused first kernel of the
    inner Lanczos step on the packed pairs i <= j (n_l = o v + o (o + 1) / 2
    v^2 FP64 elements per vector): p_{k-1}, v_{k-1}, w_{k-2}, w_{k-3} and
    the iterate read and v_k, w_{k-1} and the iterate written once (8 vector
    passes), the virtual part f_vv v_k + v_k f_vv of the doubles written,
    f_vv read."""
    npair = o * (o + 1) // 2
    nl = o * v + npair * v * v
    return 8 * (8 * nl + npair * v * v + v * v)


def fock_vir_lz_flops(o, v):
    """Its flops: two v-deep products per packed doubles block (4 v^3) and
    about 8 per element for the update."""
    npair = o * (o + 1) // 2
    return 4 * npair * v ** 3 + 8 * (o * v + npair * v * v)


def cpu_baseline(problem, counts, t1_gpu, t2_gpu, e_gpu):
    """Oracle timed on the host on a bounded sample (one residual, one
    complex-step J v and one A_F GMRES solve of the same workload), scaled
    to solves/s with the GPU solve's operation counts. Also evaluates the
    oracle's residual and energy at the GPU's converged amplitudes."""
    from gen import random_amplitudes
    from oracle import ccsd, solvers
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    p = problem
    o, v = p.nocc, p.nvir
    t1, t2 = random_amplitudes(o, v, 11, scale=0.01)
    x1, x2 = random_amplitudes(o, v, 12, scale=1.0)
    t0 = time.perf_counter()
    ccsd.residual(p.f_oo, p.f_ov, p.f_vv, p.L, t1, t2)
    t_res = time.perf_counter() - t0
    t0 = time.perf_counter()
    ccsd.jvp_complex_step(p.f_oo, p.f_ov, p.f_vv, p.L, t1, t2, x1, x2)
    t_jvp = time.perf_counter() - t0
    t0 = time.perf_counter()
    _, _, res = solvers.fock_solve_gmres(p.f_oo, p.f_ov, p.f_vv, x1, x2, rtol=1e-12)
    t_af = (time.perf_counter() - t0) / max(res.iters, 1)
    per_solve = counts["n_residual"] * t_res + counts["n_jvp"] * t_jvp + counts["n_afmv"] * t_af
    r1, r2 = ccsd.residual(p.f_oo, p.f_ov, p.f_vv, p.L, t1_gpu, t2_gpu)
    e_or = ccsd.energy(p.f_oo, p.f_ov, p.f_vv, p.L, t1_gpu, t2_gpu)
    import numpy as np
    out = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
           "sample": (f"oracle (numpy FP64) on {o}/{v}/{p.naux}: 1 residual {t_res:.2f}s, 1 complex-step J v "
                      f"{t_jvp:.2f}s, 1 A_F GMRES solve of {res.iters} products {t_af * res.iters:.2f}s; scaled by "
                      f"the GPU solve's {counts['n_residual']} residuals, {counts['n_jvp']} J v and "
                      f"{counts['n_afmv']} A_F products -> {per_solve:.0f} s per solve")}
    check = {"oracle_res_inf_at_gpu_root": float(max(np.abs(r1).max(), np.abs(r2).max())),
             "abs_dE_oracle_energy_at_gpu_root": float(abs(e_or - e_gpu))}
    return out, check


def bench_c2(args):
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config

    pk.load()
    p = make_config(WORKLOAD)
    o, v, naux = p.nocc, p.nvir, p.naux
    tol = p.meta["tol"]
    h = pk.Handle(0)
    nsteps = args.warmup + args.steps
    probs = [pk.DeviceProblem.from_problem(p) for _ in range(nsteps)]
    torch.cuda.synchronize()

    def step(P):
        return h.solve_pnk(P, tol_inf=tol, max_newton=200)

    for i in range(args.warmup):
        step(probs[i])
    torch.cuda.synchronize()
    h.timing(True)
    lat, infos = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.warmup, nsteps):
        s0 = time.perf_counter()
        t1, t2, info = step(probs[i])
        lat.append(time.perf_counter() - s0)  # solve_pnk returns after its final sync
        infos.append(info)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n_res, ms_res = h.timing_read(1)
    n_jvp, ms_jvp = h.timing_read(2)
    n_afm, ms_afm = h.timing_read(3)
    n_pre, ms_pre = h.timing_read(4)
    h.timing(False)

    ok = all(i["status"] == "CC_OK" for i in infos)
    e = infos[-1]["e_corr"]
    ms_step = 1000.0 * elapsed / args.steps
    lat_ms = sorted(1000.0 * x for x in lat)

    def pct(q):
        k = min(len(lat_ms) - 1, max(0, int(round(q / 100.0 * (len(lat_ms) - 1)))))
        return lat_ms[k]

    F_R = nominal_residual_flops(o, v, naux)
    res_ms = ms_res / max(n_res, 1)
    af_ms = ms_afm / n_afm if n_afm else None
    af_bytes = fock_vir_lz_bytes(o, v)
    roof = None
    if af_ms:
        gbs = af_bytes / (af_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbs / HBM_PEAK_GBS, "traffic": VIR_LZ_TRAFFIC_BYTES,
                "kernel": "fock_vir_lz_kernel (inner Lanczos step on the packed pairs: the previous step's "
                          "update fused with the A_F virtual contractions)",
                "launches_timed": n_afm, "avg_us": af_ms * 1e3, "bytes_per_launch": af_bytes,
                "flops_per_launch": fock_vir_lz_flops(o, v)}
    out = {
        "metric": "PNK CCSD solves/s + p50/p99 latency at |dE|<1e-6 Eh; residual TFLOP/s vs FP64",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{WORKLOAD}: RCCSD Haar-rotated gauge, nocc={o} nvir={v} naux={naux}, "
                               f"FP64 PNK (m_max 20, A_F^-1 by inner Lanczos/GMRES rtol 1e-12) to "
                               f"||r||_inf<{tol:g}",
                   "nocc": o, "nvir": v, "naux": naux, "tol_inf": tol},
        "latency_ms": {"p50": pct(50), "p99": pct(99)},
        "converged": ok,
        "e_corr": e,
        "counts_per_solve": {k: infos[-1][k] for k in ("newton_iters", "n_residual", "n_jvp", "n_afmv")},
        "residual_tflops_fp64": F_R / (res_ms * 1e-3) / 1e12 if n_res else None,
        "residual_ms": res_ms if n_res else None,
        "jvp_ms": ms_jvp / n_jvp if n_jvp else None,
        "precond_solve_ms": ms_pre / n_pre if n_pre else None,
        "time_share": {"residual": ms_res / (1000 * elapsed), "jvp": ms_jvp / (1000 * elapsed),
                       "precond_solve": ms_pre / (1000 * elapsed),
                       # the average of the sampled launches times every launch that ran
                       # (one per inner step plus the normalising one per inner solve)
                       "A_F_fused_virtual_kernel": (af_ms or 0.0) * (sum(i["n_afmv"] for i in infos) + n_pre)
                       / (1000 * elapsed)},
        "roofline": roof,
    }
    if not args.no_cpu_baseline:
        cb, check = cpu_baseline(p, infos[-1], t1.cpu().numpy(), t2.cpu().numpy(), e)
        out["cpu_baseline"] = cb
        out.update(check)
    print(json.dumps(out), flush=True)
    h.close()


def krylov_inner_rtol(prec):
    """Tolerance of the inner A_F solves applied to J q in the Krylov loop:
    an order of magnitude below the relative error of the J v product it
    preconditions (BF16: near 1e-3; FP32: near 1e-6, so 1e-6 there too);
    FP64 solves every inner system to the Newton right-hand side's 1e-12
    (0: the same tolerance). On the o=20 v=180 line the Newton count stays at
    34 from 1e-3 to 1e-12; the A_F products per solve fall from 17888
    (1e-12) to 9713 (1e-6) and 6811 (1e-4)."""
    return {"bf16": 1e-4, "fp32": 1e-6}.get(prec, 0.0)


def occ_packed_bytes(o, v):
    """Algorithmic HBM bytes of one occupied A_F launch of the packed inner
    step (three-launch form): v_k, the virtual part of p and v_{k-1} read,
    p written, n_l = o v + o (o + 1) / 2 v^2 elements each."""
    nl = o * v + o * (o + 1) // 2 * v * v
    return 8 * 4 * nl


def cpu_baseline_sample(problem, counts, t1_gpu, t2_gpu, e_gpu):
    """The oracle on the host, on a bounded sample of the same workload: one
    residual evaluation (at the device's root, which also checks it) and a
    few A_F products of its GMRES. A complex-step J v costs at least one
    residual (it evaluates the residual once in complex arithmetic), so each
    is counted as one residual: the rate is an upper bound of the oracle's."""
    import numpy as np

    from oracle import ccsd, solvers
    try:
        from threadpoolctl import threadpool_info
        threads = max((i.get("num_threads", 1) for i in threadpool_info()), default=1)
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    p = problem
    o, v = p.nocc, p.nvir
    t0 = time.perf_counter()
    r1, r2 = ccsd.residual(p.f_oo, p.f_ov, p.f_vv, p.L, t1_gpu, t2_gpu)
    t_res = time.perf_counter() - t0
    e_or = float(ccsd.energy(p.f_oo, p.f_ov, p.f_vv, p.L, t1_gpu, t2_gpu))
    t0 = time.perf_counter()
    _, _, res = solvers.fock_solve_gmres(p.f_oo, p.f_ov, p.f_vv, r1, r2, rtol=1e-12, maxit=4)
    t_af = (time.perf_counter() - t0) / max(res.iters, 1)
    per_solve = (counts["n_residual"] + counts["n_jvp"]) * t_res + counts["n_afmv"] * t_af
    out = {"value": 1.0 / per_solve, "unit": "solves/s", "cores": int(threads), "kind": "oracle",
           "sample": (f"oracle (numpy FP64) on {o}/{v}/{p.naux}: 1 residual {t_res:.1f} s, {res.iters} A_F "
                      f"products {t_af * res.iters:.2f} s; scaled by the device solve's {counts['n_residual']} "
                      f"residuals, {counts['n_jvp']} J v (each counted as one residual, a lower bound of the "
                      f"complex-step product) and {counts['n_afmv']} A_F products -> {per_solve:.0f} s per solve "
                      f"(an upper bound of the oracle's rate)")}
    check = {"oracle_res_inf_at_root": float(max(np.abs(r1).max(), np.abs(r2).max())),
             "abs_dE_oracle_energy_at_root": float(abs(e_or - e_gpu))}
    return out, check


def bench_headline(args):
    """The default line: mixed-precision PNK solves of c4_mixed."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config

    t_begin = time.perf_counter()
    pk.load()
    p = make_config(HEADLINE)
    o, v, naux = p.nocc, p.nvir, p.naux
    tol = p.meta["tol"]
    prec = args.prec or "bf16"
    rtol_jv = args.inner_rtol_jv if args.inner_rtol_jv is not None else krylov_inner_rtol(prec)
    h = pk.Handle(0)
    nsteps = args.warmup + args.steps
    probs = [pk.DeviceProblem.from_problem(p) for _ in range(nsteps)]
    torch.cuda.synchronize()

    def step(P, jprec):
        return h.solve_pnk(P, tol_inf=tol, max_newton=200, jvp_prec=jprec, inner_rtol=args.inner_rtol,
                           inner_rtol_jv=rtol_jv if jprec == prec else 0.0)

    for i in range(args.warmup):
        step(probs[i], prec)
        print(f"warm-up solve {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    h.timing(True)
    lat, infos = [], []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.warmup, nsteps):
        s0 = time.perf_counter()
        t1, t2, info = step(probs[i], prec)
        lat.append(time.perf_counter() - s0)  # solve_pnk returns after its final sync
        infos.append(info)
        print(f"solve {i + 1 - args.warmup}/{args.steps}: {lat[-1]:.2f} s, {info['status']}", file=sys.stderr,
              flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    n_res, ms_res = h.timing_read(1)
    n_jvp, ms_jvp = h.timing_read(2)
    n_afm, ms_afm = h.timing_read(3)
    n_pre, ms_pre = h.timing_read(4)
    h.timing(False)
    ok = all(x["status"] == "CC_OK" for x in infos)
    e = infos[-1]["e_corr"]
    lat_ms = sorted(1000.0 * x for x in lat)

    def pct(q):
        k = min(len(lat_ms) - 1, max(0, int(round(q / 100.0 * (len(lat_ms) - 1)))))
        return lat_ms[k]

    # FP64 reference solve of the same problem (untimed), when it fits the
    # run's window: about 1.7 mixed-precision solves, plus the oracle leg
    ref = None
    spent = time.perf_counter() - t_begin
    est = 1.9 * (elapsed / max(args.steps, 1)) + 60.0
    if prec != "fp64" and spent + est < RUN_BUDGET_S:
        s0 = time.perf_counter()
        _, _, ri = step(probs[0], "fp64")
        ref = {"status": ri["status"], "e_corr": ri["e_corr"], "newton_iters": ri["newton_iters"],
               "seconds": time.perf_counter() - s0}
        print(f"FP64 reference solve: {ref['seconds']:.1f} s", file=sys.stderr, flush=True)

    F_R = nominal_residual_flops(o, v, naux)
    # algorithmic flops: 2 M N K of every contraction as the library runs it
    # (symmetry-adapted ladder; tiles' padding not counted), from the library
    F_alg, F_jv = h.contraction_flops(probs[0], prec)
    res_ms = ms_res / max(n_res, 1)
    roof = None
    if n_res:
        tf = F_alg / (res_ms * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tf / FP64_PEAK_TFLOPS, "traffic": RESIDUAL_TRAFFIC_BYTES,
                "kernel": "FP64 residual evaluation (recorded graph of matrix-core products: ladder in the "
                          "symmetric/antisymmetric pair basis, ring, hole-hole, Fock and dressing terms)",
                "launches_timed": n_res, "avg_ms": res_ms, "flops_per_launch": F_alg}
    roof_jvp = None
    if n_jvp and prec == "bf16":
        jv_ms = ms_jvp / n_jvp
        tj = F_jv / (jv_ms * 1e-3) / 1e12
        roof_jvp = {"bound": "mfma", "achieved": tj, "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                    "frac": tj / BF16_PEAK_TFLOPS, "traffic": None,
                    "kernel": "BF16 J v product (recorded graph: the tangent contractions in BF16 with float "
                              "accumulation, their FP64 operands rounded once per product)",
                    "launches_timed": n_jvp, "avg_ms": jv_ms, "flops_per_launch": F_jv}
    roof_inner = None
    if n_afm:
        af_ms = ms_afm / n_afm
        b = occ_packed_bytes(o, v)
        gbs = b / (af_ms * 1e-3) / 1e9
        roof_inner = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                      "frac": gbs / HBM_PEAK_GBS, "traffic": OCC_PACKED_TRAFFIC_BYTES,
                      "kernel": "fock_occ_set_kernel (occupied A_F contractions of the inner Lanczos step on "
                                "the packed pairs, register-blocked over transpose-closed position sets)",
                      "launches_timed": n_afm, "avg_us": af_ms * 1e3,
                      "bytes_per_launch": b}
    out = {
        "metric": "PNK CCSD solves/s + p50/p99 latency at |dE|<1e-6 Eh; residual TFLOP/s vs FP64",
        "value": args.steps / elapsed,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1000.0 * elapsed / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+bf16" if prec == "bf16" else ("f64+f32" if prec == "fp32" else "f64"),
        "data": "synthetic",
        "config": {"workload": f"{HEADLINE}: RCCSD Haar-rotated gauge, nocc={o} nvir={v} naux={naux}, "
                               f"mixed-precision PNK (J v in {prec.upper()} on the matrix cores with float "
                               f"accumulation; residual, energy, Arnoldi, least squares and update in FP64; "
                               f"m_max 20, A_F^-1 by inner Lanczos/GMRES to rtol {args.inner_rtol:g} for "
                               f"the Newton right-hand side and {rtol_jv or args.inner_rtol:g} for A_F^-1 J q in "
                               f"the Krylov loop) to ||r||_inf<{tol:g}, one solve per step",
                   "nocc": o, "nvir": v, "naux": naux, "tol_inf": tol, "jvp_prec": prec,
                   "inner_rtol": args.inner_rtol, "inner_rtol_jv": rtol_jv,
                   "latency": "per-solve latency of back-to-back solves (the serving stream is "
                              "--workload serving)"},
        "latency_ms": {"p50": pct(50), "p99": pct(99)},
        "converged": ok,
        "e_corr": e,
        "fp64_reference": ref,
        "abs_dE_vs_fp64_root": abs(e - ref["e_corr"]) if ref else None,
        "counts_per_solve": {k: infos[-1][k] for k in ("newton_iters", "n_residual", "n_jvp", "n_afmv")},
        "residual_tflops_fp64_nominal": F_R / (res_ms * 1e-3) / 1e12 if n_res else None,
        "residual_tflops_fp64_algorithmic": F_alg / (res_ms * 1e-3) / 1e12 if n_res else None,
        "flops_per_residual": {"nominal": F_R, "algorithmic": F_alg},
        "flops_per_jvp_algorithmic": F_jv,
        "residual_ms": res_ms if n_res else None,
        "jvp_ms": ms_jvp / n_jvp if n_jvp else None,
        "precond_solve_ms": ms_pre / n_pre if n_pre else None,
        "time_share": {"residual": ms_res / (1000 * elapsed), "jvp": ms_jvp / (1000 * elapsed),
                       "precond_solve": ms_pre / (1000 * elapsed)},
        "roofline": roof,
        "roofline_inner": roof_inner,
        "roofline_jvp": roof_jvp,
    }
    if not args.no_cpu_baseline:
        cb, check = cpu_baseline_sample(p, infos[-1], t1.cpu().numpy(), t2.cpu().numpy(), e)
        out["cpu_baseline"] = cb
        out.update(check)
    out["run_seconds"] = time.perf_counter() - t_begin
    print(json.dumps(out), flush=True)
    h.close()


def bench_large(args):
    """One PNK solve of a larger workload (near-degenerate o=16/v=144 or the
    mixed-precision o=20/v=180), J v in the requested precision; prints one
    JSON line with the time to solution and the operation counts."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config

    pk.load()
    p = make_config("c4_mixed" if args.workload == "c4_single" else args.workload)
    o, v, naux = p.nocc, p.nvir, p.naux
    tol = p.meta["tol"]
    args.prec = args.prec or "fp64"
    h = pk.Handle(0)
    P = pk.DeviceProblem.from_problem(p)
    torch.cuda.synchronize()
    h.timing(True)
    t0 = time.perf_counter()
    t1, t2, info = h.solve_pnk(P, tol_inf=tol, max_newton=args.max_newton, jvp_prec=args.prec,
                               inner_rtol=args.inner_rtol, inner_rtol_jv=args.inner_rtol_jv or 0.0)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n_res, ms_res = h.timing_read(1)
    n_jvp, ms_jvp = h.timing_read(2)
    n_pre, ms_pre = h.timing_read(4)
    h.timing(False)
    hist = h.history()
    F_R = nominal_residual_flops(o, v, naux)
    out = {"workload": args.workload, "nocc": o, "nvir": v, "naux": naux, "tol_inf": tol, "jvp_prec": args.prec,
           "inner_rtol": args.inner_rtol,
           "status": info["status"], "seconds": dt, "e_corr": info["e_corr"], "res_inf": info["res_inf"],
           "counts": {k: info[k] for k in ("newton_iters", "n_residual", "n_jvp", "n_afmv")},
           "residual_ms": ms_res / max(n_res, 1), "residual_tflops_fp64_nominal": F_R / (ms_res / max(n_res, 1) * 1e-3) / 1e12,
           "jvp_ms": ms_jvp / max(n_jvp, 1), "precond_solve_ms": ms_pre / max(n_pre, 1),
           "res_inf_history": [float(x) for x in hist[:, 1][:: max(1, len(hist) // 40)]]}
    print(json.dumps(out), flush=True)
    h.close()


def bench_serving(args):
    """Serving stream: seeded requests with nocc ~ U{4..16}, nvir = nocc *
    U{5..9}, naux = 3 (nocc + nvir), alternating canonical and rotated
    gauges. The closed-loop rate mu (all requests queued at once) is measured
    first, then an open-loop Poisson stream at 0.7 mu; both for FP64 J v and
    for the mixed-precision (BF16 J v) path. Prints one JSON line."""
    import numpy as np

    import paper_2608_06669_amd as pk
    from gen import make_serving_request, poisson_arrivals, serving_request_shapes

    pk.load()
    reqs = [make_serving_request(s) for s in serving_request_shapes(args.requests)]
    res = {}

    def opts(prec):
        o = dict(tol_inf=1e-8, max_newton=args.max_newton, jvp_prec=prec, stall_window=args.stall_window,
                 stall_factor=0.5)
        if prec != "fp64":
            o["inner_rtol_jv"] = krylov_inner_rtol(prec)  # as on the default line's mixed path
        return o

    def run(prec, arrivals=None):
        srv = pk.Server(0, max_slots=args.slots)
        try:
            t0 = time.perf_counter()
            ids = []
            for k, r in enumerate(reqs):
                if arrivals is not None:
                    wait = arrivals[k] - (time.perf_counter() - t0)
                    if wait > 0:
                        time.sleep(wait)
                ids.append(srv.submit(r, **opts(prec)))
            # collect as they finish (progress on stderr)
            out = [None] * len(ids)
            left = set(range(len(ids)))
            while left:
                for k in list(left):
                    res_k = srv.poll(ids[k], want_amplitudes=False)
                    if res_k is not None:
                        out[k] = res_k
                        left.discard(k)
                        done = len(ids) - len(left)
                        if done % 8 == 0 or not left:
                            print(f"{prec} {'open' if arrivals is not None else 'closed'} loop: {done}/{len(ids)} "
                                  f"done, {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
                if left:
                    time.sleep(0.005)
            wall = time.perf_counter() - t0
            times = [srv.times(i) for i in ids]
            stats = srv.stats()
        finally:
            srv.close()
        lat = sorted(1000.0 * (f - s) for (s, _, f) in times)
        return dict(wall=wall, solves_per_s=len(reqs) / wall, p50_ms=float(np.percentile(lat, 50)),
                    p99_ms=float(np.percentile(lat, 99)), peak_running=stats["peak_running"],
                    peak_bytes=stats["peak_bytes"], budget=stats["budget"], handle_reuses=stats["handle_reuses"],
                    converged=sum(1 for x in out if x["status"] == "CC_OK"),
                    stalled=sum(1 for x in out if x["stalled"]),
                    energies=[x["e_corr"] for x in out], ok=[x["status"] == "CC_OK" for x in out])

    closed = {prec: run(prec) for prec in ("fp64", "bf16")}
    mu = closed["fp64"]["solves_per_s"]
    lam = 0.7 * mu
    arr = poisson_arrivals(len(reqs), lam)
    opened = {prec: run(prec, arr) for prec in ("fp64", "bf16")}
    both = [k for k in range(len(reqs)) if closed["fp64"]["ok"][k] and closed["bf16"]["ok"][k]]
    de = max((abs(closed["fp64"]["energies"][k] - closed["bf16"]["energies"][k]) for k in both), default=None)
    for d in (closed, opened):
        for x in d.values():
            x.pop("energies")
            x.pop("ok")
    sizes = [(r.nocc, r.nvir) for r in reqs]
    out = {"workload": f"serving stream, {len(reqs)} requests (C5 sample), PNK to ||r||_inf<1e-8, {args.slots} "
                       f"slots, stagnation stop after {args.stall_window} Newton steps without halving "
                       f"||r||_inf; BF16 path with the Krylov-loop inner solves to {krylov_inner_rtol('bf16'):g}",
           "request_sizes": sizes, "closed_loop": closed, "poisson_rate_per_s": lam, "open_loop": opened,
           "max_abs_dE_bf16_vs_fp64_converged": de, "n_converged_in_both": len(both)}
    print(json.dumps(out), flush=True)


def bench_inner(args):
    """Inner A_F solves alone (--config, default the C2 shapes): `steps` solves of A_F x = b
    with a seeded pair-symmetric b; used for kernel counters. Each solve
    ends with one copy of the N-vector (a copy kernel of known size)."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config, random_amplitudes

    pk.load()
    cfg = args.config or WORKLOAD
    p = make_config(cfg)
    o, v = p.nocc, p.nvir
    h = pk.Handle(0)
    P = pk.DeviceProblem.from_problem(p)
    b1, b2 = (torch.as_tensor(a, device="cuda") for a in random_amplitudes(o, v, 77, scale=1.0))
    out = {"workload": f"inner A_F solves, {cfg} (o={o} v={v})", "solves": args.steps,
           "n_vector": o * v + o * o * v * v}
    # full layout (cc_precond_solve), then the packed pair layout the PNK
    # solver uses (cc_precond_solve_pairsym); --layout picks one of them
    layouts = [("full", False), ("pairsym", True)]
    if args.layout != "both":
        layouts = [x for x in layouts if x[0] == args.layout]
    for name, sym in layouts:
        h.precond_solve(P, b1, b2, pair_symmetric=sym)  # warm-up: preparation and graph recording
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = 0
        for _ in range(args.steps):
            _, _, it, _ = h.precond_solve(P, b1, b2, pair_symmetric=sym)
            iters += it
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out[name] = {"products": iters, "us_per_product": 1e6 * dt / max(iters, 1),
                     "ms_per_solve": 1e3 * dt / args.steps}
    print(json.dumps(out), flush=True)
    h.close()


def bench_protocols(args):
    """The method table on the device: PNK, NK, INK, FP and SFP+DIIS on C1
    (canonical) and C2 (Haar-rotated), at the CCSD and the CCD level. Prints
    one JSON line with, per run, the residual evaluations (residuals plus
    Jacobian products, the paper's cost measure), A_F products, steps, time,
    energy and whether ||r||_inf < tol was reached."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config

    pk.load()
    h = pk.Handle(0)
    out = {"workload": "protocols (method table) on c1_canonical and c2_haar, CCSD and CCD", "runs": []}
    runs = [("PNK", "pnk", {}), ("NK", "pnk", {"protocol": "nk"}), ("INK", "pnk", {"protocol": "ink"}),
            ("FP", "fp", {"diis_size": 0}), ("SFP+DIIS", "fp", {"level_shift": 0.2})]
    for cfg in ("c1_canonical", "c2_haar"):
        p = make_config(cfg)
        tol = p.meta["tol"]
        P = pk.DeviceProblem.from_problem(p)
        for level in ("ccsd", "ccd"):
            for name, kind, opts in runs:
                o = dict(opts, tol_inf=tol, ccd=int(level == "ccd"))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if kind == "pnk":
                    _, _, info = h.solve_pnk(P, max_newton=args.max_newton, **o)
                else:
                    _, _, info = h.solve_fp_diis(P, max_iter=max(args.max_newton, 200), **o)
                dt = time.perf_counter() - t0
                out["runs"].append({"config": cfg, "level": level, "protocol": name,
                                    "converged": info["status"] == "CC_OK",
                                    "residual_evaluations": info["n_residual"] + info["n_jvp"],
                                    "n_residual": info["n_residual"], "n_jvp": info["n_jvp"],
                                    "n_afmv": info["n_afmv"], "steps": info["newton_iters"],
                                    "seconds": dt, "e_corr": info["e_corr"], "res_inf": info["res_inf"]})
                print(f"{cfg} {level} {name}: {out['runs'][-1]}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    h.close()


def bench_levelshift(args):
    """The regularization study: at the PNK root of C1 (canonical) and C2
    (Haar-rotated), the spectral radius of the (S)FP map's Jacobian for a
    range of level shifts (30 Arnoldi steps from a seeded pair-symmetric
    start), and what SFP does from the MP2 start at each shift (without
    DIIS and with DIIS(8)). One JSON line."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config, random_amplitudes

    pk.load()
    h = pk.Handle(0)
    shifts = [0.0, 0.1, 0.25, 0.5, 1.0, 2.0]
    out = {"workload": "level-shift study at the PNK root (c1_canonical, c2_haar)", "m": 30, "shifts": shifts,
           "configs": []}
    for cfg in ("c1_canonical", "c2_haar"):
        p = make_config(cfg)
        tol = p.meta["tol"]
        P = pk.DeviceProblem.from_problem(p)
        t1, t2, info = h.solve_pnk(P, tol_inf=tol, max_newton=args.max_newton)
        q1, q2 = (torch.as_tensor(a, device="cuda") for a in random_amplitudes(p.nocc, p.nvir, 4242, scale=1.0))
        rec = {"config": cfg, "pnk_converged": info["status"] == "CC_OK", "e_corr": info["e_corr"], "rho": [],
               "sfp": [], "sfp_diis": []}
        for s in shifts:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rho, _ = h.fp_spectral_radius(P, t1, t2, q1, q2, shift=s, m=30)
            rec["rho"].append({"shift": s, "rho": rho, "seconds": time.perf_counter() - t0})
            for key, nd in (("sfp", 0), ("sfp_diis", 8)):
                _, _, fi = h.solve_fp_diis(P, tol_inf=tol, level_shift=s, diis_size=nd, max_iter=200)
                rec[key].append({"shift": s, "converged": fi["status"] == "CC_OK", "n_residual": fi["n_residual"],
                                 "res_inf": fi["res_inf"]})
            print(f"{cfg} shift {s}: rho {rho:.4f} sfp {rec['sfp'][-1]} sfp+diis {rec['sfp_diis'][-1]}",
                  file=sys.stderr, flush=True)
        out["configs"].append(rec)
    print(json.dumps(out), flush=True)
    h.close()


def bench_gauge(args):
    """Solves in non-orthogonal gauges (gauge functions chi = phi W per
    orbital block, cond(W) = kappa): on C1 (canonical orbitals, where FP
    converges) PNK, FP and FP+DIIS(8) in gauges of growing kappa, all from
    the MP2 start; on C2 (Haar-rotated) PNK in the kappa = 4 gauge beside the
    orbital-basis PNK solve (same root, transformed). One JSON line."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import GAUGE_WORKLOAD, make_config, nonorthogonal_gauge

    pk.load()
    h = pk.Handle(0)
    out = {"workload": "non-orthogonal gauges: c1_canonical at cond(W) 1..16, c2_haar at cond(W) 4", "runs": []}

    def rec(cfg, kappa, name, info, dt):
        r = {"config": cfg, "cond_W": kappa, "solver": name, "converged": info["status"] == "CC_OK",
             "residual_evaluations": info["n_residual"] + info["n_jvp"], "n_jvp": info["n_jvp"],
             "n_afmv": info["n_afmv"], "steps": info["newton_iters"], "seconds": dt, "e_corr": info["e_corr"],
             "res_inf": info["res_inf"]}
        out["runs"].append(r)
        print(f"{cfg} cond {kappa} {name}: {r}", file=sys.stderr, flush=True)

    def timed(fn, *a, **kw):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = fn(*a, **kw)
        torch.cuda.synchronize()
        return res, time.perf_counter() - t0

    p = make_config("c1_canonical")
    tol = p.meta["tol"]
    P = pk.DeviceProblem.from_problem(p)
    for kappa in (1.0, 2.0, 4.0, 8.0, 16.0):
        G = pk.DeviceGauge(*nonorthogonal_gauge(p.nocc, p.nvir, GAUGE_WORKLOAD["gauge_seed"], kappa))
        (_, _, info), dt = timed(h.solve_pnk_gauge, P, G, tol_inf=tol, max_newton=args.max_newton)
        rec("c1_canonical", kappa, "PNK", info, dt)
        (_, _, info), dt = timed(h.solve_fp_diis_gauge, P, G, tol_inf=tol, diis_size=0, max_iter=500)
        rec("c1_canonical", kappa, "FP", info, dt)
        (_, _, info), dt = timed(h.solve_fp_diis_gauge, P, G, tol_inf=tol, max_iter=500)
        rec("c1_canonical", kappa, "FP+DIIS", info, dt)
    cfg = GAUGE_WORKLOAD["config"]
    p = make_config(cfg)
    tol = p.meta["tol"]
    P = pk.DeviceProblem.from_problem(p)
    kappa = GAUGE_WORKLOAD["cond"]
    G = pk.DeviceGauge(*nonorthogonal_gauge(p.nocc, p.nvir, GAUGE_WORKLOAD["gauge_seed"], kappa))
    h.solve_pnk(P, tol_inf=tol, max_newton=args.max_newton)  # warm-up: graphs and integrals
    (_, _, info), dt = timed(h.solve_pnk, P, tol_inf=tol, max_newton=args.max_newton)
    rec(cfg, 1.0, "PNK (orbital basis)", info, dt)
    h.solve_pnk_gauge(P, G, tol_inf=tol, max_newton=args.max_newton)
    (_, _, info), dt = timed(h.solve_pnk_gauge, P, G, tol_inf=tol, max_newton=args.max_newton)
    rec(cfg, kappa, "PNK", info, dt)
    (_, _, info), dt = timed(h.solve_fp_diis_gauge, P, G, tol_inf=tol, max_iter=200)
    rec(cfg, kappa, "FP+DIIS", info, dt)
    print(json.dumps(out), flush=True)
    h.close()


def bench_residual(args):
    """Residual and J v (FP64, FP32, BF16) evaluations alone (recorded graphs
    replayed) on c2_haar and c4_mixed at seeded amplitudes, --steps of each
    (a J v call also evaluates the residual at its point; the J v times
    subtract the residual's), plus one
    1024^3 FP64 product through cc_diag_gemm (2^31 flops). A torch
    elementwise kernel runs before every evaluation and after the last, so
    that a counter run (rocprofv3 --pmc) can attribute the dispatches
    between two such markers to one evaluation; the 1024^3 product
    calibrates the matrix-core operation counters. One JSON line."""
    import torch

    import paper_2608_06669_amd as pk
    from gen import make_config, random_amplitudes

    pk.load()
    h = pk.Handle(0)
    mark = torch.zeros(1, dtype=torch.float64, device="cuda")
    out = {"workload": "residual and J v alone (c2_haar, c4_mixed)", "steps": args.steps, "configs": []}
    A = torch.randn(1024, 1024, dtype=torch.float64, device="cuda")
    B = torch.randn(1024, 1024, dtype=torch.float64, device="cuda")
    C = torch.zeros(1024, 1024, dtype=torch.float64, device="cuda")
    mark.add_(1.0)
    pk.diag_gemm(A, B, C, (1024, 1), (1024, 1), (1024, 1), 1024, 1024, 1024)
    mark.add_(1.0)
    # a plain copy of 2^25 doubles (256 MiB read, 256 MiB written): the
    # scale for the FETCH_SIZE / WRITE_SIZE counters
    src = torch.randn(1 << 25, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    mark.add_(1.0)
    torch.cuda.synchronize()
    for cfg in ("c2_haar", "c4_mixed"):
        p = make_config(cfg)
        o, v, naux = p.nocc, p.nvir, p.naux
        P = pk.DeviceProblem.from_problem(p)
        t1, t2 = (torch.as_tensor(a, device="cuda") for a in random_amplitudes(o, v, 77, scale=0.01))
        q1, q2 = (torch.as_tensor(a, device="cuda") for a in random_amplitudes(o, v, 78, scale=1.0))
        r1, r2 = torch.empty_like(t1), torch.empty_like(t2)
        for _ in range(3):  # integrals, then the recorded graph
            h.residual(P, t1, t2, r1, r2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mark.add_(1.0)
            h.residual(P, t1, t2, r1, r2)
        mark.add_(1.0)
        torch.cuda.synchronize()
        res_ms = 1000.0 * (time.perf_counter() - t0) / max(args.steps, 1)
        y = (torch.empty_like(q1), torch.empty_like(q2))
        for _ in range(3):
            h.jvp(P, t1, t2, q1, q2, out=y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mark.add_(1.0)
            h.jvp(P, t1, t2, q1, q2, out=y)  # a residual (the linearisation point) and J v
        mark.add_(1.0)
        torch.cuda.synchronize()
        rj_ms = 1000.0 * (time.perf_counter() - t0) / max(args.steps, 1)
        F_R = nominal_residual_flops(o, v, naux)
        rec = {"config": cfg, "nocc": o, "nvir": v, "naux": naux, "residual_ms": res_ms,
               "residual_tflops_nominal": F_R / (res_ms * 1e-3) / 1e12, "nominal_residual_flops": F_R,
               "residual_plus_jvp_ms": rj_ms, "jvp_ms": rj_ms - res_ms}
        # the low-precision products of the Krylov loop, each after a
        # marker: a residual (FP64) then J v in that precision
        for prec in ("fp32", "bf16"):
            for _ in range(3):
                h.jvp(P, t1, t2, q1, q2, prec=prec, out=y)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                mark.add_(1.0)
                h.jvp(P, t1, t2, q1, q2, prec=prec, out=y)
            mark.add_(1.0)
            torch.cuda.synchronize()
            rec[f"jvp_{prec}_ms"] = 1000.0 * (time.perf_counter() - t0) / max(args.steps, 1) - res_ms
        # 2 M N K of every contraction as run (an eager evaluation after the
        # last marker of this configuration)
        fr, fj = h.contraction_flops(P, "fp64")
        rec["flops_algorithmic"] = {"residual": fr, "jvp": fj}
        rec["residual_tflops_algorithmic"] = fr / (res_ms * 1e-3) / 1e12
        rec["jvp_fp64_tflops_algorithmic"] = fj / (rec["jvp_ms"] * 1e-3) / 1e12
        rec["jvp_bf16_tflops_algorithmic"] = fj / (rec["jvp_bf16_ms"] * 1e-3) / 1e12
        out["configs"].append(rec)
        print(f"{cfg}: {rec}", file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)
    h.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default=HEADLINE,
                    choices=[HEADLINE, WORKLOAD, "c3_neardeg", "c4_single", "serving", "inner", "protocols",
                             "levelshift", "gauge", "residual"],
                    help="default: the bench line; the others print their own measurement line")
    ap.add_argument("--prec", default=None, choices=["fp64", "fp32", "bf16"],
                    help="J v precision (default line: bf16; c3_neardeg / c4_single: fp64)")
    ap.add_argument("--max-newton", type=int, default=200)
    ap.add_argument("--inner-rtol", type=float, default=1e-12, help="A_F^-1 inner solve tolerance (c3/c4)")
    ap.add_argument("--inner-rtol-jv", type=float, default=None,
                    help="tolerance of the inner solves of A_F^-1 J q in the Krylov loop (0: --inner-rtol)")
    ap.add_argument("--layout", default="both", choices=["both", "full", "pairsym"],
                    help="inner: which inner-solve layout to time")
    ap.add_argument("--config", default=None, choices=["c2_haar", "c4_mixed"],
                    help="inner: the workload whose shapes the inner solves take (default c2_haar)")
    ap.add_argument("--requests", type=int, default=40)
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--stall-window", type=int, default=10, help="serving: stagnation stop window (0: off)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU (asked for {args.gpus}): one solve is not sharded across GPUs here; "
              "see the design notes for how it would shard", file=sys.stderr)
        sys.exit(2)
    if args.workload == HEADLINE:
        bench_headline(args)
    elif args.workload == WORKLOAD:
        bench_c2(args)
    elif args.workload == "serving":
        bench_serving(args)
    elif args.workload == "inner":
        bench_inner(args)
    elif args.workload == "protocols":
        bench_protocols(args)
    elif args.workload == "levelshift":
        bench_levelshift(args)
    elif args.workload == "gauge":
        bench_gauge(args)
    elif args.workload == "residual":
        bench_residual(args)
    else:
        bench_large(args)


if __name__ == "__main__":
    main()
