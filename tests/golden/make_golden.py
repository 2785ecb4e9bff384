"""Write stored oracle results for workloads too large to run inside a test.

Calls only the oracle (FP64, CPU).  Usage:
    python tests/golden/make_golden.py cfg1_batch16 [cfg2 cfg3 ...]
Writes tests/golden/<name>_oracle.json with, per shift, the gains sigma_B
(Algorithm 1 step 5) and sigma_AV (steps 6-8) for the workload's k, q, seed
and Phi-weighted test matrix (eq. 10).  With --grad (the gradient workload)
it also stores, per shift, the triplet residual of the conditioning report
and the gradient of sigma_1 with respect to every node of U (ring included),
nu and omega, the last three in tests/golden/<name>_grad.npz.
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402
from oracle import grad, operator as op, resolvent, sketch  # noqa: E402
from oracle.operator import shifted  # noqa: E402
from oracle.solver import ShiftedSolver  # noqa: E402


def run(name: str, with_grad: bool = False):
    w = W.CONFIGS[name]
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    phi = sketch.gradient_weight(U, hx, hy).ravel()
    Om = sketch.test_matrix(w.n, w.k, phi, seed=w.seed)
    out = {"workload": name, "n": w.n, "k": w.k, "q": w.q, "seed": w.seed,
           "omegas": list(w.omegas), "sigma_B": [], "sigma_AV": [], "seconds": []}
    grads = {"dU": [], "dnu": [], "domega": []}
    if with_grad:
        out["triplet_res"] = []
    for om in w.omegas:
        t = time.time()
        S = ShiftedSolver(shifted(L, om))
        r = resolvent.randomized_resolvent(L, om, Om, q=w.q, solver=S)
        out["sigma_B"].append([float(x) for x in r.sigma_B])
        out["sigma_AV"].append([float(x) for x in r.sigma_AV])
        if with_grad:
            s1, u1, v1 = r.sigma_AV[0], r.U_AV[:, 0], r.V[:, 0]
            res = S.solve_adjoint(u1) - s1 * v1   # the triplet residual (conditioning report)
            out["triplet_res"].append(float(np.linalg.norm(res) / s1))
            dU, dnu, dom = grad.gradient_full(s1, u1, v1, w.nx, w.ny, hx, hy)
            grads["dU"].append(dU)
            grads["dnu"].append(dnu)
            grads["domega"].append(dom)
        out["seconds"].append(time.time() - t)
        print(name, om, r.sigma_B[:3], f"{time.time() - t:.1f}s", flush=True)
        with open(os.path.join(HERE, f"{name}_oracle.json"), "w") as fh:
            json.dump(out, fh, indent=1)
    if with_grad:
        np.savez_compressed(os.path.join(HERE, f"{name}_grad.npz"),
                            dU=np.array(grads["dU"]), dnu=np.array(grads["dnu"]),
                            domega=np.array(grads["domega"]))


if __name__ == "__main__":
    g = "--grad" in sys.argv[1:]
    for nm in [a for a in sys.argv[1:] if not a.startswith("--")]:
        run(nm, with_grad=g)
