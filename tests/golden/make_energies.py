"""Write tests/golden/oracle_energies.json: CPU-oracle CCSD solutions of the
named synthetic workloads, converged to ||r||_inf < 1e-11.

For each workload it stores the correlation energy, the solve's counts and
a seeded sample of the converged amplitudes (indices drawn by
numpy default_rng(77); t1 and t2 values at those indices), so that a device
solve can be compared element by element without storing the whole vector.

Calls only oracle/ (and the input generator). Run from the repository root:
    python tests/golden/make_energies.py [config ...]
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import make_config  # noqa: E402
from oracle import solvers  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_energies.json")
N_SAMPLE_T1 = 64
N_SAMPLE_T2 = 512


def amplitude_sample(t1, t2, seed=77):
    rng = np.random.default_rng(seed)
    i1 = np.sort(rng.choice(t1.size, size=min(N_SAMPLE_T1, t1.size), replace=False))
    i2 = np.sort(rng.choice(t2.size, size=min(N_SAMPLE_T2, t2.size), replace=False))
    return dict(t1_index=[int(i) for i in i1], t1=[float(x) for x in t1.ravel()[i1]],
                t2_index=[int(i) for i in i2], t2=[float(x) for x in t2.ravel()[i2]],
                t1_max_abs=float(np.abs(t1).max()), t2_max_abs=float(np.abs(t2).max()),
                t2_norm=float(np.linalg.norm(t2)))


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        p = make_config(name)
        t0 = time.time()
        t1, t2, info = solvers.solve_pnk(p.f_oo, p.f_ov, p.f_vv, p.L, tol=1e-11, max_newton=200)
        data[name] = dict(e_corr=info.e_corr, converged=bool(info.converged), res_inf=info.res_inf,
                          tol=1e-11, solver="oracle PNK (complex-step J v, GMRES A_F^-1)",
                          newton_iters=info.newton_iters, n_residual=info.n_residual, n_jvp=info.n_jvp,
                          seconds=time.time() - t0, sample=amplitude_sample(t1, t2))
        print(name, {k: v for k, v in data[name].items() if k != "sample"}, flush=True)
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c1_canonical", "c2_haar"])
