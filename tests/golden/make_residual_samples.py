"""Write tests/golden/oracle_residual_samples.json: the CPU oracle's CCSD
residual, energy and Jacobian-vector product at seeded amplitudes of the
full-size workloads, stored as a seeded sample of elements plus whole-vector
norms.

The residual is equation CC_ampl (oracle.ccsd.residual), the energy equation
CC_energy, and J v the complex-step derivative of the residual (exact to
rounding). At these sizes the oracle takes minutes (the complex-step product
forms the complex (ac|bd) block, nvir^4 elements), so the values are written
once here and the device tests compare against them.

Amplitudes: gen.random_amplitudes(o, v, seed_t, scale 0.01) for t and
(seed_v, scale 1.0) for the direction. Element indices: numpy
default_rng(1234) without replacement, in the flattened t1 / t2 layouts.

Calls only oracle/ (and the input generator). Run from the repository root:
    python tests/golden/make_residual_samples.py [config ...]
"""

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from gen import make_config, random_amplitudes  # noqa: E402
from oracle import ccsd  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "oracle_residual_samples.json")
SEEDS = {"c3_neardeg": (301, 302), "c4_mixed": (401, 402)}
N1, N2 = 128, 768


def sample(x, idx):
    return [float(a) for a in np.ravel(x)[idx]]


def summary(x1, x2, i1, i2):
    return dict(s1=sample(x1, i1), s2=sample(x2, i2), max1=float(np.abs(x1).max()), max2=float(np.abs(x2).max()),
                norm1=float(np.linalg.norm(x1)), norm2=float(np.linalg.norm(x2)))


def main(names):
    data = json.load(open(OUT)) if os.path.exists(OUT) else {}
    for name in names:
        p = make_config(name)
        o, v = p.nocc, p.nvir
        seed_t, seed_v = SEEDS[name]
        t1, t2 = random_amplitudes(o, v, seed_t, scale=0.01)
        v1, v2 = random_amplitudes(o, v, seed_v, scale=1.0)
        rng = np.random.default_rng(1234)
        i1 = np.sort(rng.choice(o * v, size=N1, replace=False))
        i2 = np.sort(rng.choice(o * o * v * v, size=N2, replace=False))
        t0 = time.time()
        r1, r2 = ccsd.residual(p.f_oo, p.f_ov, p.f_vv, p.L, t1, t2)
        e = float(ccsd.energy(p.f_oo, p.f_ov, p.f_vv, p.L, t1, t2))
        t_res = time.time() - t0
        t0 = time.time()
        j1, j2 = ccsd.jvp_complex_step(p.f_oo, p.f_ov, p.f_vv, p.L, t1, t2, v1, v2)
        t_jvp = time.time() - t0
        data[name] = dict(amplitudes=dict(seed_t=seed_t, scale_t=0.01, seed_v=seed_v, scale_v=1.0),
                          index1=[int(i) for i in i1], index2=[int(i) for i in i2], e_corr=e,
                          residual=summary(r1, r2, i1, i2), jvp=summary(j1, j2, i1, i2),
                          seconds=dict(residual=t_res, jvp_complex_step=t_jvp))
        print(name, "E", e, "residual", round(t_res, 1), "s, J v", round(t_jvp, 1), "s", flush=True)
        del r1, r2, j1, j2
        with open(OUT, "w") as fh:
            json.dump(data, fh, indent=0, sort_keys=True)


if __name__ == "__main__":
    main(sys.argv[1:] or ["c3_neardeg", "c4_mixed"])
