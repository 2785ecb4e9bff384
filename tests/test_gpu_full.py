"""The benchmark's own workload at full size (512 x 256 Burgers, n = 262144,
16 shifts, k = 20, q = 1) in the launch configuration the benchmark times,
against the oracle's gains stored by tests/golden/make_golden.py: every gain
sigma_B (step 5) and sigma_AV (steps 6-8) of every shift; and properties that
hold at any size: Q and V orthonormal within the Cholesky QR bound
6 (n k + k (k + 1)) u, unit response modes, and sigma_AV_j >= sigma_B_j
(||H v_j|| >= ||Q^H H v_j|| for orthonormal Q)."""
import functools
import json
import os

import numpy as np
import pytest

import workloads as W
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import gain_errors, mode_angles, oracle_problem, to_np

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
    orth_bound = 6 * (w.n * w.k + w.k * (w.k + 1)) * 2.0 ** -53
    eye = np.eye(w.k)
    worst = {"Q": 0.0, "V": 0.0, "U": 0.0}
    for i in range(len(w.omegas)):
        for key in ("Q", "V"):
            X = to_np(out[key][i])  # (k, n): the k columns as rows
            worst[key] = max(worst[key], np.abs(X @ X.conj().T - eye).max())
        U = to_np(out["U"][i])
        worst["U"] = max(worst["U"], np.abs(np.linalg.norm(U, axis=1) - 1).max())
        big = sB[i] >= 1e-3 * sB[i][0]
        assert np.all(sAV[i][big] >= sB[i][big] * (1 - tol)), i
    print(f"\n{prec}: max |Q^H Q - I| {worst['Q']:.1e}, |V^H V - I| {worst['V']:.1e}, "
          f"| ||u_j|| - 1 | {worst['U']:.1e} (bound {orth_bound:.1e})")
    assert worst["Q"] <= orth_bound and worst["V"] <= orth_bound
    assert worst["U"] <= 1e-12
    out["factors"].free()


@functools.lru_cache(maxsize=1)
def oracle_at(omega):
    """The oracle's Algorithm 1 at one shift of the benchmark batch, full size
    (SuperLU factor, five solves, Householder QR, SVD: about 15 s)."""
    w = W.CONFIGS["cfg1_batch16"]
    U, coef, L, phi, hx, hy = oracle_problem(w)
    return ores.randomized_resolvent(L, omega, osk.test_matrix(w.n, w.k, phi, w.seed), q=w.q)


@pytest.mark.parametrize("prec,refine_tol", [("fp64", 0.0), ("mixed", 1e-8)])
def test_full_batch_modes_match_oracle_at_one_shift(prec, refine_tol):
    """Forcing and response modes at full size, sampled at omega = 2 (the one
    shift the oracle recomputes here): sine of the largest principal angle
    below 1e-6 over the gain clusters within the first five modes."""
    w = W.CONFIGS["cfg1_batch16"]
    i = int(np.argmin(np.abs(np.asarray(w.omegas) - 2.0)))
    ref = oracle_at(w.omegas[i])
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, seed=w.seed, precision=prec,
                         tile=64, refine_tol=refine_tol)
    aV = mode_angles(to_np(out["V"][i]).T, ref.V, ref.sigma_B, 5)
    aU = mode_angles(to_np(out["U"][i]).T, ref.U_AV, ref.sigma_B, 5)
    print(f"\n{prec} at omega = {w.omegas[i]}: forcing-mode angle {aV:.1e}, response {aU:.1e}")
    assert aV < 1e-6 and aU < 1e-6
    out["factors"].free()
