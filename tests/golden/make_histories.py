"""Write tests/golden/oracle_histories.json: residual-norm histories of the
CPU oracle's solvers on two workloads where the solver does not converge,
so that a device solve can be compared with it step by step.

* neardeg_o4_v36: the near-degenerate recipe (HOMO-LUMO gap 0.05 Eh, two
  occupied and two virtual levels within 0.1 Eh of the Fermi level, DF
  entries N(0, 0.08^2), the frontier pairs rotated) at o=4, v=36,
  naux=3(o+v), seed 1003: PNK (Algorithm 1 with the Eisenstat-Walker
  forcing term, m_max 20) to ||r||_inf < 1e-8, at most 40 Newton steps.
* neardeg_o6_v54: the same recipe at o=6, v=54, naux=180, seed 1003, PNK
  to 1e-8 with at most 20 Newton steps (it stalls near 3e-2).
* c2_haar_fp_diis: FP+DIIS(8) on the Haar-rotated o=10/v=90/naux=300
  workload from the MP2 start, at most 10 iterations (the iteration stops
  once ||r||_2 exceeds 1e6).

History entries are (residual evaluations so far, ||r||_2, ||r||_inf) after
each outer residual. Calls only oracle/ (and the input generator). Run from
the repository root:
    python tests/golden/make_histories.py [name ...]
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import make_config  # noqa: E402
from gen.problems import make_near_degenerate  # noqa: E402
from oracle import solvers  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_histories.json")


def record(info, t0, **extra):
    return dict(converged=bool(info.converged), newton_iters=info.newton_iters, n_residual=info.n_residual,
                n_jvp=info.n_jvp, e_corr=info.e_corr, res_inf=info.res_inf, res_2=info.res_2,
                history=[[int(a), float(b), float(c)] for a, b, c in info.history], seconds=time.time() - t0, **extra)


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    if "neardeg_o4_v36" in names:
        t0 = time.time()
        p = make_near_degenerate(4, 36, 120, 1003, sigma=0.08)
        _, _, info = solvers.solve_pnk(p.f_oo, p.f_ov, p.f_vv, p.L, tol=1e-8, max_newton=40)
        data["neardeg_o4_v36"] = record(info, t0, recipe="make_near_degenerate(4, 36, 120, 1003, sigma=0.08)",
                                        solver="oracle PNK tol 1e-8 max_newton 40 m_max 20")
        print("neardeg o4", data["neardeg_o4_v36"]["newton_iters"], data["neardeg_o4_v36"]["res_inf"], flush=True)
    if "neardeg_o6_v54" in names:
        t0 = time.time()
        p = make_near_degenerate(6, 54, 180, 1003, sigma=0.08)
        _, _, info = solvers.solve_pnk(p.f_oo, p.f_ov, p.f_vv, p.L, tol=1e-8, max_newton=20)
        data["neardeg_o6_v54"] = record(info, t0, recipe="make_near_degenerate(6, 54, 180, 1003, sigma=0.08)",
                                        solver="oracle PNK tol 1e-8 max_newton 20 m_max 20")
        print("neardeg o6", data["neardeg_o6_v54"]["newton_iters"], data["neardeg_o6_v54"]["res_inf"],
              [f"{h[2]:.3e}" for h in data["neardeg_o6_v54"]["history"]], flush=True)
    if "c2_haar_fp_diis" in names:
        t0 = time.time()
        p = make_config("c2_haar")
        _, _, info = solvers.solve_fp_diis(p.f_oo, p.f_ov, p.f_vv, p.L, tol=1e-8, max_iter=10)
        data["c2_haar_fp_diis"] = record(info, t0, recipe="make_config('c2_haar')",
                                         solver="oracle FP+DIIS(8) from MP2, max_iter 10, divergence at "
                                                "||r||_2 > 1e6")
        print("c2 fp+diis", data["c2_haar_fp_diis"]["history"], flush=True)
    with open(OUT, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["neardeg_o4_v36", "neardeg_o6_v54", "c2_haar_fp_diis"])
