"""The benchmark's own workload at full size (512 x 256 Burgers, n = 262144,
16 shifts, k = 20, q = 1) in the launch configuration the benchmark times,
against the oracle's gains stored by tests/golden/make_golden.py: every gain
sigma_B (step 5) and sigma_AV (steps 6-8) of every shift."""
import json
import os

import numpy as np
import pytest

import workloads as W
from tests.gpu_util import gain_errors, to_np

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "cfg1_batch16_oracle.json")


def rr():
    import paper_1902_01458_amd as m
    return m


@pytest.mark.parametrize("prec,tol,refine_tol", [("fp64", 1e-10, 0.0), ("mixed", 1e-8, 1e-8)])
def test_full_batch_matches_stored_oracle(prec, tol, refine_tol):
    gold = json.load(open(GOLD))
    w = W.CONFIGS["cfg1_batch16"]
    assert gold["n"] == w.n and gold["k"] == w.k and gold["q"] == w.q
    np.testing.assert_allclose(gold["omegas"], w.omegas, rtol=0)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, seed=w.seed, precision=prec,
                         tile=64, refine_tol=refine_tol)
    sB, sAV = to_np(out["sigma_B"]), to_np(out["sigma_AV"])
    for i in range(len(w.omegas)):
        assert gain_errors(sB[i], gold["sigma_B"][i]).max() <= tol, i
        assert gain_errors(sAV[i], gold["sigma_AV"][i]).max() <= tol, i
    out["factors"].free()
