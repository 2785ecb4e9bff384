"""Write stored oracle results for workloads too large to run inside a test.

Calls only the oracle (FP64, CPU).  Usage:
    python tests/golden/make_golden.py cfg1_batch16 [cfg2 ...]
Writes tests/golden/<name>_oracle.json with, per shift, the gains sigma_B
(Algorithm 1 step 5) and sigma_AV (steps 6-8) for the workload's k, q, seed
and Phi-weighted test matrix (eq. 10).
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import operator as op, resolvent, sketch  # noqa: E402


def run(name: str):
    w = W.CONFIGS[name]
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    phi = sketch.gradient_weight(U, hx, hy).ravel()
    Om = sketch.test_matrix(w.n, w.k, phi, seed=w.seed)
    out = {"workload": name, "n": w.n, "k": w.k, "q": w.q, "seed": w.seed,
           "omegas": list(w.omegas), "sigma_B": [], "sigma_AV": [], "seconds": []}
    for om in w.omegas:
        t = time.time()
        r = resolvent.randomized_resolvent(L, om, Om, q=w.q)
        out["sigma_B"].append([float(x) for x in r.sigma_B])
        out["sigma_AV"].append([float(x) for x in r.sigma_AV])
        out["seconds"].append(time.time() - t)
        print(name, om, r.sigma_B[:3], f"{time.time() - t:.1f}s", flush=True)
        with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as fh:
            json.dump(out, fh, indent=1)


if __name__ == "__main__":
    for nm in sys.argv[1:]:
        run(nm)
