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
    ap.add_argument("--tile", type=int, default=64,
                    help="band tile when --no-autotune is given")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--graph-reps", type=int, default=2)
    ap.add_argument("--refine-iters", type=int, default=0)
    ap.add_argument("--refine-tol", type=float, default=1e-8,
                    help="mixed path: refinement tolerance of the projection and recovery solves "
                         "(1e-8: the metric's own bound on the sigma_1 error; the library "
                         "default 1e-10 costs one more correction per solve)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-shifts", type=int, default=1)
    ap.add_argument("--no-cpu-1-thread", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the single-shift, 64-shift and 1024 x 512 rates")
    ap.add_argument("--no-cfg4", action="store_true")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (a known-size "
                         "kernel for scaling hardware byte counters)")
    return ap.parse_args()


def run_path(prob, w, precision, steps, warmup, tile, refine_iters, autotune, graph_reps,
             refine_tol=0.0):
    import torch

    import paper_1902_01458_amd as rr
    tune = {"tile": tile, "grid": 0, "superblock": 0, "ms": None}
    if autotune:
        tune = rr.autotune(prob, list(w.omegas), w.k, precision)
    f = rr.factor(prob, list(w.omegas), precision, k_max=w.k, tile=tune["tile"],
                  grid=tune["grid"], superblock=tune["superblock"], refine_iters=refine_iters,
                  refine_tol=refine_tol)
    f.check()
    stream = torch.cuda.current_stream()
    Q = f.empty_block(w.k)
    Z = f.empty_block(w.k)
    outs = {}
    names = ("factor", "sketch", "adjoint", "gains")

    def step(ev=None):
        # ev: 5 events bracketing the four calls, recorded on the launch stream
        if ev is not None:
            ev[0].record(stream)
        f.refactor()
        if ev is not None:
            ev[1].record(stream)
        f.sketch_solve(w.k, w.seed, w.q, out=Q)
        if ev is not None:
            ev[2].record(stream)
        f.adjoint_solve(Q, out=Z)
        if ev is not None:
            ev[3].record(stream)
        outs.update(f.gains(Q, Z, "av", out=outs))
        if ev is not None:
            ev[4].record(stream)

    for _ in range(warmup):
        step()
    f.check()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(5)] for _ in range(steps)]
    # per step: the factor kernel alone and the step's last main solve launch
    # (the forward solve of the eq. 9 recovery), recorded by the library
    kev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    for e in kev:
        for x in e:
            x.record(stream)  # creates the events before the library records them
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(steps):
        f.set_timing_events(factor=(kev[i][0], kev[i][1]), solve=(kev[i][2], kev[i][3]))
        step(evs[i])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    f.set_timing_events()
    f.check()
    per = {nm: float(np.mean([e[c].elapsed_time(e[c + 1]) for e in evs]))
           for c, nm in enumerate(names)}
    kern = {"factor": float(np.mean([e[0].elapsed_time(e[1]) for e in kev])),
            "solve": float(np.mean([e[2].elapsed_time(e[3]) for e in kev]))}
    # the optional steps 10-11 (not part of the timed step), on the last outputs
    sv = f.resvd(outs["U"], outs["V"], scale=outs["sigma_AV"])
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    f.resvd(outs["U"], outs["V"], scale=outs["sigma_AV"], out=sv)
    e1.record(stream)
    f.check()
    resvd_ms = e0.elapsed_time(e1)
    res = {"ms_per_step": (t1 - t0) * 1e3 / steps, "factor_ms": kern["factor"],
           "solve_ms": kern["solve"], "calls_ms": per,
           "sigma_B": outs["sigma_B"].cpu().numpy(), "sigma_AV": outs["sigma_AV"].cpu().numpy(),
           "refine": f.refine_count(), "bytes": f.nbytes(), "tune": tune,
           "optional_svd_ms": resvd_ms}
    if graph_reps > 0:
        # the same pass captured once and replayed (outside the timed region)
        g = rr.capture(f, w.k, w.seed, w.q, "av", refactor=True)
        g.launch()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(graph_reps):
            g.launch()
        torch.cuda.synchronize()
        res["graph_ms_per_step"] = (time.perf_counter() - t0) * 1e3 / graph_reps
        f.check()
        res["graph_sigma_equal"] = bool(np.array_equal(g.sigma_B.cpu().numpy(), res["sigma_B"]))
        g.free()
    f.free()
    del Q, Z, outs
    torch.cuda.empty_cache()
    return res


def timed_pass(f, k, seed, q, reps):
    """Mean event-timed ms of `reps` passes of Algorithm 1 (refactorisation,
    sketch and subspace iteration, adjoint solve, gains with the eq. 9
    recovery) on the handle, after one warm-up pass."""
    import torch
    stream = torch.cuda.current_stream()
    Q = f.empty_block(k)
    Z = f.empty_block(k)
    outs = {}

    def one():
        f.refactor()
        f.sketch_solve(k, seed, q, out=Q)
        f.adjoint_solve(Q, out=Z)
        outs.update(f.gains(Q, Z, "av", out=outs))

    one()
    f.check()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        one()
    e1.record(stream)
    f.check()
    return e0.elapsed_time(e1) / reps, outs


def extras(args):
    """The other rates the benchmark plan asks for, each a timed pass after a
    warm-up: the single shift omega = 2 of the 512 x 256 configuration, the
    64-shift sweep of config 2 (mixed and FP64) and config 4's 16 shifts in
    chunks that fit the device (mixed; allocation outside the timed passes)."""
    import torch

    import paper_1902_01458_amd as rr
    import workloads as W
    out = {}
    w1 = W.CONFIGS["cfg1"]
    p1 = rr.BurgersProblem.from_workload(w1)
    for prec, tol in (("mixed", args.refine_tol), ("fp64", 0.0)):
        f = rr.factor(p1, [2.0], prec, k_max=w1.k, refine_tol=tol)
        ms, o = timed_pass(f, w1.k, w1.seed, w1.q, 3)
        out.setdefault("single_omega2_ms", {})[prec] = ms
        f.free()
    del p1
    w2 = W.CONFIGS["cfg2"]
    p2 = rr.BurgersProblem.from_workload(w2)
    gold2 = os.path.join(ROOT, "tests", "golden", "cfg2_oracle.json")
    g2 = json.load(open(gold2)) if os.path.exists(gold2) else None
    for prec, tol in (("mixed", args.refine_tol), ("fp64", 0.0)):
        f = rr.factor(p2, list(w2.omegas), prec, k_max=w2.k, refine_tol=tol)
        ms, o = timed_pass(f, w2.k, w2.seed, w2.q, 2)
        err = None
        if g2 is not None:
            sb = np.asarray(g2["sigma_B"])[:, 0]
            err = float(np.max(np.abs(o["sigma_B"][:, 0].cpu().numpy() - sb) / sb))
        out.setdefault("cfg2_64shifts", {})[prec] = {
            "ms_per_pass": ms, "omega_solves_per_s": len(w2.omegas) / (ms * 1e-3),
            "sigma1_rel_err_vs_oracle": err}
        f.free()
        torch.cuda.empty_cache()
    del p2
    if not args.no_cfg4:
        w4 = W.CONFIGS["cfg4"]
        p4 = rr.BurgersProblem.from_workload(w4)
        free, _ = torch.cuda.mem_get_info()
        per = rr.factor_bytes(w4.nx, w4.ny, 1, w4.k, "mixed") + 6 * w4.k * w4.n * 16
        chunk = max(1, min(16, int(0.8 * free // per)))
        total = 0.0
        s1 = []
        for c0 in range(0, 16, chunk):
            oms = list(w4.omegas[c0:c0 + chunk])
            f = rr.factor(p4, oms, "mixed", k_max=w4.k, refine_tol=args.refine_tol)
            ms, o = timed_pass(f, w4.k, w4.seed, w4.q, 1)
            total += ms
            s1 += list(o["sigma_AV"][:, 0].cpu().numpy())
            del o
            f.free()
            torch.cuda.empty_cache()
        out["cfg4_16shifts_mixed"] = {"chunk": chunk, "ms_total": total,
                                      "omega_solves_per_s": 16 / (total * 1e-3),
                                      "sigma1_AV_first": float(s1[0])}
    return out


TRAFFIC = os.path.join(ROOT, "profiles", "pmc_traffic.json")
CSRC = os.path.join(ROOT, "paper_1902_01458_amd", "csrc")


def traffic(kernel):
    """HBM bytes per launch of `kernel` from the calibrated FETCH_SIZE / WRITE_SIZE
    counters recorded in profiles/pmc_traffic.json, or None when none were taken
    or the kernel sources changed since (the file keeps their SHA-256)."""
    import hashlib
    if not os.path.exists(TRAFFIC):
        return None
    rec = json.load(open(TRAFFIC))
    h = hashlib.sha256()
    for fn in sorted(os.listdir(CSRC)):
        h.update(open(os.path.join(CSRC, fn), "rb").read())
    if rec.get("sources_sha256") != h.hexdigest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["read_bytes"] + k["write_bytes"]


def accuracy(res, gold):
    if gold is None:
        return None
    sb = np.asarray(gold["sigma_B"])[:, 0]
    return float(np.max(np.abs(res["sigma_B"][:, 0] - sb) / sb))


def cpu_baseline(w, shifts, threads1=True):
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
    # one shift: omega = 2.0, the single frequency of the 512 x 256 configuration
    i2 = int(np.argmin(np.abs(np.asarray(w.omegas) - 2.0)))
    sel = [w.omegas[i2]] if shifts == 1 else list(w.omegas[:shifts])
    with threadpoolctl.threadpool_limits(cores):
        t0 = time.perf_counter()
        for om in sel:
            ores.randomized_resolvent(L, om, Om, q=w.q)
        dt = time.perf_counter() - t0
    res = {"value": len(sel) / dt, "unit": "ω-solves/s", "cores": cores, "kind": "oracle",
           "sample": f"{len(sel)} of {len(w.omegas)} shifts (omega={sel[0]:.3g}) of the same "
                     f"workload, SuperLU factor + 5 solves + QR + SVD in FP64, {dt:.1f} s"}
    if threads1:
        with threadpoolctl.threadpool_limits(1):
            t0 = time.perf_counter()
            ores.randomized_resolvent(L, sel[0], Om, q=w.q)
            res["value_1_thread"] = 1.0 / (time.perf_counter() - t0)
    model = mem = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal"):
                mem = f"{int(ln.split()[1]) / 2**20:.0f} GiB"
                break
    except OSError:
        pass
    res["cpu_model"], res["host_memory"] = model, mem
    return res


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
    n_om = len(w.omegas)
    flops = 8.0 * w.n * b * b * n_om  # algorithmic band-LU flops per launch (all shifts)
    auto = not args.no_autotune
    mixed = run_path(prob, w, "mixed", args.steps, args.warmup, args.tile, args.refine_iters,
                     auto, args.graph_reps, args.refine_tol)
    print(f"# mixed: {mixed['ms_per_step']:.1f} ms/step {mixed['calls_ms']}, refine "
          f"{mixed['refine']}, tune {mixed['tune']}", file=sys.stderr, flush=True)
    fp64 = None
    if not args.no_fp64:
        fp64 = run_path(prob, w, "fp64", args.steps, args.warmup, args.tile, 0, auto,
                        args.graph_reps)
        print(f"# fp64: {fp64['ms_per_step']:.1f} ms/step {fp64['calls_ms']}, tune "
              f"{fp64['tune']}", file=sys.stderr, flush=True)
    value = n_om / (mixed["ms_per_step"] * 1e-3)
    ach = flops / (mixed["factor_ms"] * 1e-3) / 1e12
    fk = f"k_factor<float,{mixed['tune']['tile']}>"
    # algorithmic bytes of one solve launch: the factor once (n (2b+1) entries
    # per shift, FP32 or FP64), the right-hand sides in and the solutions out
    # (FP64 complex, the caller's blocks)
    def solve_roofline(res, esize, name):
        byt = n_om * (w.n * (2 * b + 1) * esize + 2 * w.k * w.n * 16)
        bw = byt / (res["solve_ms"] * 1e-3) / 1e9
        np_ = 16 * ((w.k + 15) // 16)
        T = res["tune"]["tile"]
        # the superblock solve's short-piece form when the half-band spans at most 8
        # tiles, with its last column block in real form when that holds at most 8
        # of the k columns
        short = (b + T - 1) // T <= 8
        tail = short and w.k - (np_ - 16) <= 8
        kname = (f"k_solve2<{name},{T},16,false>" if (res["tune"].get("superblock") or 0) < 0
                 else f"k_ssolve<{name},{T},{np_},false,{str(short).lower()},{str(tail).lower()}>")
        return {"bound": "hbm", "achieved": bw, "peak": 8000.0, "unit": "GB/s",
                "frac": bw / 8000.0, "bytes_per_launch": byt, "traffic": traffic(kname),
                "kernel": f"{kname} (forward solve of the eq. 9 recovery, all {n_om} shifts x "
                          f"{w.k} columns, one launch)",
                "launch_ms": res["solve_ms"]}
    line = {
        "metric": METRIC, "value": value, "unit": "ω-solves/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": mixed["ms_per_step"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "c64 factor/solves + f64 residual, Gram, SVD", "data": "synthetic",
        "config": {"workload": f"{args.workload}: 2-D linearised Burgers {w.nx}x{w.ny}, n={w.n}, "
                               f"half-bandwidth {b}, {n_om} shifts 0.25..8, k={w.k}, q={w.q}, "
                               "Phi-weighted Gaussian sketch, seed 0",
                   "tile": mixed["tune"]["tile"], "grid": mixed["tune"]["grid"],
                   "superblock": mixed["tune"].get("superblock"),
                   "autotuned": auto, "refine_tol": args.refine_tol, "refine_tol_sketch": 1e-8},
        "gains_per_s": value * w.k,
        "sigma1_rel_err_vs_oracle": accuracy(mixed, gold),
        "refine_corrections": mixed["refine"],
        "calls_ms": mixed["calls_ms"],
        "optional_svd_ms": mixed["optional_svd_ms"],
        "graph_ms_per_step": mixed.get("graph_ms_per_step"),
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK["mixed"], "unit": "TFLOP/s",
                     "frac": ach / PEAK["mixed"], "traffic": traffic(fk),
                     "kernel": f"{fk} (band LU of all {n_om} shifts, one launch)",
                     "launch_ms": mixed["factor_ms"]},
        "roofline_solve_fp32": solve_roofline(mixed, 8, "float"),
    }
    if fp64 is not None:
        a64 = flops / (fp64["factor_ms"] * 1e-3) / 1e12
        line["fp64"] = {"value": n_om / (fp64["ms_per_step"] * 1e-3),
                        "ms_per_step": fp64["ms_per_step"], "calls_ms": fp64["calls_ms"],
                        "optional_svd_ms": fp64["optional_svd_ms"],
                        "graph_ms_per_step": fp64.get("graph_ms_per_step"),
                        "tile": fp64["tune"]["tile"], "grid": fp64["tune"]["grid"],
                        "superblock": fp64["tune"].get("superblock"),
                        "sigma1_rel_err_vs_oracle": accuracy(fp64, gold),
                        "factor_roofline": {"bound": "mfma", "achieved": a64,
                                            "peak": PEAK["fp64"], "unit": "TFLOP/s",
                                            "frac": a64 / PEAK["fp64"],
                                            "launch_ms": fp64["factor_ms"]}}
        line["roofline_solve"] = solve_roofline(fp64, 16, "double")
        line["mixed_over_fp64"] = line["fp64"]["ms_per_step"] / mixed["ms_per_step"]
    if not args.no_extras:
        line["extras"] = extras(args)
        print(f"# extras: {line['extras']}", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w, args.cpu_sample_shifts,
                                            threads1=not args.no_cpu_1_thread)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
