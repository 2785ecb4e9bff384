"""Throughput of the randomized-resolvent hot path on one MI355X.

Workload: the 512 x 256 linearised Burgers operator (n = 262144, half-bandwidth
512) swept over 16 shifts omega_i = 2^((i-6)/3) (0.25 .. 8, holding 2.0), sketch
width k = 20, one subspace iteration, Phi-weighted complex Gaussian test matrix,
seed 0.  One step = the whole path for the batch: 16 band factorisations, the
sketch, the forward / adjoint / subspace-iteration solves (with FP64-residual
refinement in the mixed path), every Cholesky QR, the k x k SVDs, V and the
response recovery of eq. (9).  Inputs (U, coefficients, Phi) are resident on the
GPU before timing starts.

Prints one JSON line: value = omega-solves/s of the mixed path; the FP64 path,
the roofline of the factorisation kernel and the oracle's CPU rate ride along.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "ω-solves/sec at n=262k,k=20: mixed+refine vs FP64 at σ1 rel err ≤1e-8"
PEAK = {"mixed": 157.3, "fp64": 78.6}  # dense MFMA TFLOP/s: fp32, fp64
GOLDEN = os.path.join(ROOT, "tests", "golden", "cfg1_batch16_oracle.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="cfg1_batch16")
    ap.add_argument("--tile", type=int, default=64)
    ap.add_argument("--refine-iters", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-shifts", type=int, default=1)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "kernel for scaling hardware byte counters)")
    return ap.parse_args()


def run_path(prob, w, precision, steps, warmup, tile, refine_iters):
    import torch

    import paper_1902_01458_amd as rr
    f = rr.factor(prob, list(w.omegas), precision, k_max=w.k, tile=tile,
                  refine_iters=refine_iters)
    f.check()
    stream = torch.cuda.current_stream()
    Q = f.empty_block(w.k)
    Z = f.empty_block(w.k)
    outs = {}

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        f.refactor()
        if ev is not None:
            ev[1].record(stream)
        f.sketch_solve(w.k, w.seed, w.q, out=Q)
        f.adjoint_solve(Q, out=Z)
        outs.update(f.gains(Q, Z, "av", out=outs))

    for _ in range(warmup):
        step()
    f.check()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    f.check()
    factor_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps, "factor_ms": factor_ms,
           "sigma_B": outs["sigma_B"].cpu().numpy(), "sigma_AV": outs["sigma_AV"].cpu().numpy(),
           "refine": f.refine_count(), "bytes": f.nbytes()}
    f.free()
    del Q, Z, outs
    torch.cuda.empty_cache()
    return res


def accuracy(res, gold):
    if gold is None:
        return None
    sb = np.asarray(gold["sigma_B"])[:, 0]
    return float(np.max(np.abs(res["sigma_B"][:, 0] - sb) / sb))


def cpu_baseline(w, shifts):
    """The oracle (Algorithm 1 in FP64 on the host) on `shifts` of the batch."""
    import threadpoolctl

    from oracle import operator as op, resolvent as ores, sketch as osk
    import workloads as W
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    phi = osk.gradient_weight(U, hx, hy).ravel()
    Om = osk.test_matrix(w.n, w.k, phi, w.seed)
    cores = os.cpu_count() or 1
    sel = [w.omegas[6]] if shifts == 1 else list(w.omegas[:shifts])  # 6 -> omega = 2.0
    with threadpoolctl.threadpool_limits(cores):
        t0 = time.perf_counter()
        for om in sel:
            ores.randomized_resolvent(L, om, Om, q=w.q)
        dt = time.perf_counter() - t0
    return {"value": len(sel) / dt, "unit": "ω-solves/s", "cores": cores, "kind": "oracle",
            "sample": f"{len(sel)} of {len(w.omegas)} shifts (omega={sel[0]:.3g}) of the same "
                      f"workload, SuperLU factor + 5 solves + QR + SVD in FP64, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the batch of shifts is "
              "one GPU's share of a sweep and the multi-GPU split is by shift.", file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_1902_01458_amd as rr
    import workloads as W
    w = W.CONFIGS[args.workload]
    torch.cuda.init()
    if args.copy_calibration_mib:
        src = torch.ones(args.copy_calibration_mib << 17, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    prob = rr.BurgersProblem.from_workload(w)
    torch.cuda.synchronize()
    gold = json.load(open(GOLDEN)) if (os.path.exists(GOLDEN) and args.workload == "cfg1_batch16") \
        else None
    b = 2 * w.ny
    flops = 8.0 * w.n * b * b * len(w.omegas)  # algorithmic band-LU flops per launch
    mixed = run_path(prob, w, "mixed", args.steps, args.warmup, args.tile, args.refine_iters)
    print(f"# mixed: {mixed['ms_per_step']:.1f} ms/step, factor {mixed['factor_ms']:.1f} ms, "
          f"refine {mixed['refine']}", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_path(prob, w, "fp64", args.steps, args.warmup, args.tile, 0)
        print(f"# fp64: {fp64['ms_per_step']:.1f} ms/step, factor {fp64['factor_ms']:.1f} ms",
              file=sys.stderr, flush=True)
    n_om = len(w.omegas)
    value = n_om / (mixed["ms_per_step"] * 1e-3)
    ach = flops / (mixed["factor_ms"] * 1e-3) / 1e12
    line = {
        "metric": METRIC, "value": value, "unit": "ω-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 factor/solves + f64 residual, Gram, SVD", "data": "synthetic",
        "config": {"workload": f"{args.workload}: 2-D linearised Burgers {w.nx}x{w.ny}, n={w.n}, "
                               f"half-bandwidth {b}, {n_om} shifts 0.25..8, k={w.k}, q={w.q}, "
                               "Phi-weighted Gaussian sketch, seed 0",
                   "tile": args.tile},
        "gains_per_s": value * w.k,
        "sigma1_rel_err_vs_oracle": accuracy(mixed, gold),
        "refine_corrections": mixed["refine"],
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK["mixed"], "unit": "TFLOP/s",
                     "frac": ach / PEAK["mixed"], "traffic": None,
                     "kernel": "k_factor<float,64> (band LU, 16 shifts per launch)",
                     "factor_ms": mixed["factor_ms"]},
    }
    if fp64 is not None:
        a64 = flops / (fp64["factor_ms"] * 1e-3) / 1e12
        line["fp64"] = {"value": n_om / (fp64["ms_per_step"] * 1e-3),
                        "ms_per_step": fp64["ms_per_step"], "factor_ms": fp64["factor_ms"],
                        "sigma1_rel_err_vs_oracle": accuracy(fp64, gold),
                        "factor_tflops": a64, "factor_frac": a64 / PEAK["fp64"]}
        line["mixed_over_fp64"] = line["fp64"]["ms_per_step"] / mixed["ms_per_step"]
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_shifts)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
