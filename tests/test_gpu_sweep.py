"""Batched frequency sweeps on the GPU: captured graphs, the autotuner and
the config-2 sweep (64 shifts sharing one L) against the FP64 oracle."""
import json
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import gain_errors, mode_angles, oracle_problem, to_np

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def rr():
    import paper_1902_01458_amd as m
    return m


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_graph_replays_equal_eager_pass(prec):
    """A captured pass replays bit for bit what the eager calls compute, on
    the capturing handle, with unrelated eager work and synchronisations
    between the replays, on torch's stream and on a second stream."""
    w = W.small("gr", 40, 32, nu=1e-2, omegas=(0.3, 0.8, 1.5, 2.9, 5.0, 7.7), k=8, q=1)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, list(w.omegas), prec, k_max=w.k, tile=32)
    Q = f.sketch_solve(w.k, w.seed, w.q)
    Z = f.adjoint_solve(Q)
    ref = f.gains(Q, Z, "av")
    f.check()
    ref = {key: to_np(v) for key, v in ref.items() if v is not None}
    g = rr().capture(f, w.k, w.seed, w.q, "av", refactor=True)
    other = torch.cuda.Stream()
    X = torch.randn((len(w.omegas), 3, w.n), dtype=torch.complex128, device="cuda")
    for rep in range(4):
        # unrelated eager work in between, then a replay
        Y = prob.apply(list(w.omegas), X)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(Y)).all()
        if rep % 2 == 0:
            out = g.launch()
            f.check()
        else:
            other.wait_stream(torch.cuda.current_stream())
            out = g.launch(stream=other)
            f.check(stream=other)
        for key in ("sigma_B", "sigma_AV", "V", "U"):
            np.testing.assert_array_equal(to_np(out[key]), ref[key])
    g.free()
    f.free()


def test_autotuner_pick_runs_and_matches_oracle():
    w = W.small("at", 48, 40, nu=1e-2, omegas=(0.6, 2.2), k=10, q=1)
    prob = rr().BurgersProblem.from_workload(w)
    t = rr().autotune(prob, list(w.omegas), w.k, "fp64")
    assert t["tile"] in (32, 64) and t["grid"] > 0 and t["ms"] > 0
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, seed=w.seed, precision="fp64",
                         tile=t["tile"], grid=t["grid"])
    U, coef, L, phi, hx, hy = oracle_problem(w)
    Om = osk.test_matrix(w.n, w.k, phi, seed=w.seed)
    for i, om in enumerate(w.omegas):
        r = ores.randomized_resolvent(L, om, Om, q=w.q)
        assert gain_errors(to_np(out["sigma_AV"][i]), r.sigma_AV).max() <= 1e-10


def test_autotuner_cache_skips_the_trials(tmp_path, monkeypatch):
    """With RR_AUTOTUNE_CACHE set, the first call runs the trials (tile, grid,
    then superblock) and stores its pick in the JSON file; a second call with
    the same key returns the same pick from the file without running any
    trial (orders of magnitude faster), and a different k is a new key."""
    import time
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("RR_AUTOTUNE_CACHE", str(cache))
    w = W.small("atc", 40, 32, nu=1e-2, omegas=(0.6, 2.2), k=8, q=0)
    prob = rr().BurgersProblem.from_workload(w)
    t0 = time.perf_counter()
    first = rr().autotune(prob, list(w.omegas), w.k, "fp64")
    t1 = time.perf_counter()
    second = rr().autotune(prob, list(w.omegas), w.k, "fp64")
    t2 = time.perf_counter()
    assert first == second
    assert first["superblock"] in (-1, 0, 2, 4, 8) and first["tile"] in (32, 64)
    assert (t2 - t1) * 20 < (t1 - t0), (t1 - t0, t2 - t1)
    entries = json.loads(cache.read_text())
    assert len(entries) == 1
    (key, val), = entries.items()
    assert key.endswith("|40x32|w2|k8|fp64") and val["tile"] == first["tile"]
    rr().autotune(prob, list(w.omegas), 6, "fp64")  # another key: trials, a second entry
    assert len(json.loads(cache.read_text())) == 2


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_cfg2_sweep_matches_oracle(prec, tol):
    """Config 2: 256 x 128 grid (n = 65536), 64 log-spaced shifts in [0.1, 10],
    k = 10, all sharing one L; run as chunks of 16 captured passes.  Every
    shift's sigma_B and sigma_AV against the oracle's, stored by
    tests/golden/make_golden.py (cfg2_oracle.json)."""
    w = W.CONFIGS["cfg2"]
    gold = json.load(open(os.path.join(GOLDEN, "cfg2_oracle.json")))
    assert gold["k"] == w.k and gold["q"] == w.q and len(gold["sigma_B"]) == 64
    np.testing.assert_allclose(gold["omegas"], w.omegas, rtol=1e-15)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().sweep(prob, list(w.omegas), w.k, q=w.q, seed=w.seed, precision=prec, chunk=16)
    assert out["chunk"] == 16
    sB = to_np(out["sigma_B"])
    sAV = to_np(out["sigma_AV"])
    assert np.all(np.isfinite(sB)) and np.all(np.diff(sB, axis=1) <= 0)
    eB = np.array([gain_errors(sB[i], gold["sigma_B"][i]).max() for i in range(64)])
    eAV = np.array([gain_errors(sAV[i], gold["sigma_AV"][i]).max() for i in range(64)])
    print(f"\n[{prec}] cfg2 64 shifts: max sigma_B err {eB.max():.2e}, sigma_AV {eAV.max():.2e}")
    assert eB.max() <= tol, int(np.argmax(eB))
    assert eAV.max() <= tol, int(np.argmax(eAV))


def test_torch_caching_allocator_owns_handle_memory():
    """rr_set_allocator: a handle built through PyTorch's caching allocator
    gives the same bits as one built with hipMalloc, its bytes show up in
    torch's accounting, and they go back when the handle is freed."""
    w = W.small("al", 30, 24, nu=1e-2, omegas=(0.5, 2.0), k=6, q=1)
    prob = rr().BurgersProblem.from_workload(w)
    ref = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, tile=32)
    ref_s = to_np(ref["sigma_B"])
    ref["factors"].free()
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    rr().use_torch_allocator(True)
    try:
        f = rr().factor(prob, list(w.omegas), "fp64", k_max=w.k, tile=32)
        assert torch.cuda.memory_allocated() - before >= f.nbytes()
        out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, factors=f)
        np.testing.assert_array_equal(to_np(out["sigma_B"]), ref_s)
        del out
        f.free()
        torch.cuda.synchronize()
        assert torch.cuda.memory_allocated() <= before + 4096
    finally:
        rr().use_torch_allocator(False)
