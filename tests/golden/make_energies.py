"""Write tests/golden/oracle_energies.json: CPU-oracle CCSD correlation
energies of the named synthetic workloads, converged to ||r||_inf < 1e-11.

Calls only oracle/ (and the input generator). Run from the repository root:
    python tests/golden/make_energies.py [config ...]
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import make_config  # noqa: E402
from oracle import solvers  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_energies.json")


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        p = make_config(name)
        t0 = time.time()
        _, _, info = solvers.solve_pnk(p.f_oo, p.f_ov, p.f_vv, p.L, tol=1e-11)
        data[name] = dict(e_corr=info.e_corr, converged=bool(info.converged), res_inf=info.res_inf,
                          tol=1e-11, solver="oracle PNK (complex-step J v, GMRES A_F^-1)",
                          n_residual=info.n_residual, n_jvp=info.n_jvp, seconds=time.time() - t0)
        print(name, data[name], flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1_canonical", "c2_haar"])
