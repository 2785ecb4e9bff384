"""Test-matrix variants of Algorithm 1 step 1 on the GPU (Section 2.2.2 and
3.4): the device generator against the oracle's, the pipeline per kind
against the oracle, and the k-convergence study against the dense SVD."""
import numpy as np
import pytest

import workloads as W
from oracle import dense as odense
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import gain_errors, mode_angles, oracle_problem, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


@pytest.mark.parametrize("kind,zeta", [("gaussian", 0), ("rademacher", 0), ("sparse", 0),
                                       ("sparse", 3), ("sparse", 1)])
@pytest.mark.parametrize("weighted", [True, False])
def test_device_test_matrix_matches_oracle(kind, zeta, weighted):
    w = W.CONFIGS["cfg0"]
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w, weighted=weighted)
    th = to_np(rr().sketch(prob, w.k, seed=7, kind=kind, zeta=zeta)).T
    ref = osk.test_matrix(w.n, w.k, phi if weighted else None, seed=7, kind=kind, zeta=zeta)
    if kind == "gaussian":
        assert np.abs(th - ref).max() <= 1e-14 * np.abs(ref).max()
    else:
        np.testing.assert_array_equal(th != 0, ref != 0)  # the same sparsity pattern
        np.testing.assert_allclose(th, ref, rtol=1e-15, atol=0)


def test_orthonormal_kind_is_rejected_by_the_elementwise_hook():
    w = W.small("o", 8, 8)
    prob = rr().BurgersProblem.from_workload(w)
    with pytest.raises(rr().RRError):
        rr().sketch(prob, 4, kind="orthonormal")


@pytest.mark.parametrize("kind", ["rademacher", "sparse", "orthonormal"])
def test_pipeline_per_kind_matches_oracle(kind):
    w = W.small("k", 32, 24, nu=1e-2, omegas=(0.6, 2.2), k=8, q=1)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, seed=w.seed, tile=32,
                         test_matrix=kind, zeta=3)
    Om = osk.test_matrix(w.n, w.k, phi, w.seed, kind=kind, zeta=3)
    for i, om in enumerate(w.omegas):
        ref = ores.randomized_resolvent(L, om, Om, q=w.q)
        assert gain_errors(to_np(out["sigma_B"][i]), ref.sigma_B).max() <= 1e-10
        assert gain_errors(to_np(out["sigma_AV"][i]), ref.sigma_AV).max() <= 1e-10
        assert mode_angles(to_np(out["U"][i]).T, ref.U_AV, ref.sigma_B, 5) < 1e-6
    out["factors"].free()


def test_k_convergence_and_test_matrices_against_dense_svd():
    """The k study of Section 3.2 (Fig. 7) and the test-matrix comparison of
    Section 3.4 at n = 1024 (nu = 1e-3, omega = 1, q = 0): the error of
    sigma_1 (eq. 9) and of the leading response pair against the dense SVD
    for k = 2 .. 32 and each test matrix, Phi-weighted (eq. 10) and, for the
    Gaussian one, plain.  Every kind converges: the error at k = 32 is below
    1 % of the one at k = 4."""
    w = W.small("c", 32, 16, nu=1e-3, omegas=(1.0,), k=32, q=0)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    Ud, sd, Vd = odense.resolvent_svd(L, 1.0)
    m = 2  # the leading pair: sigma_1 / sigma_2 < 1.01, sigma_2 / sigma_3 > 2
    assert sd[0] / sd[1] < 1.01 and sd[1] / sd[2] > 2
    ks = (2, 4, 8, 16, 32)
    rows = []
    for weighted in (True, False):
        prob = rr().BurgersProblem.from_workload(w, weighted=weighted)
        f = rr().factor(prob, [1.0], "fp64", k_max=32, tile=32)
        kinds = ("gaussian", "rademacher", "sparse", "orthonormal") if weighted else ("gaussian",)
        for kind in kinds:
            f.set_test_matrix(kind, 0)
            es, eu = [], []
            for k in ks:
                Q = f.sketch_solve(k, w.seed, 0)
                Z = f.adjoint_solve(Q)
                g = f.gains(Q, Z, "av")
                f.check()
                es.append(abs(sd[0] - float(g["sigma_AV"][0, 0])) / sd[0])
                eu.append(odense.sin_angle(Ud[:, :m], to_np(g["U"][0, :min(m, k)]).T)
                          if k >= m else 1.0)
            assert es[-1] < 1e-2 * es[1], (kind, weighted, es)
            rows.append((kind + (" Phi" if weighted else " plain"), es, eu))
        f.free()
    print("\ntest matrix        " + "  ".join(f"sig k={k:<3d}" for k in ks) + "   "
          + "  ".join(f"U k={k:<3d}" for k in ks))
    for name, es, eu in rows:
        print(f"{name:18s} " + "  ".join(f"{e:9.1e}" for e in es) + "   "
              + "  ".join(f"{e:7.1e}" for e in eu))


@pytest.mark.parametrize("kind", ["sparse", "orthonormal"])
def test_graph_replay_with_test_matrix_kind(kind):
    """The handle's test matrix is part of a captured pass: the replays equal
    the eager calls bit for bit (the orthonormal kind adds a CholQR2 of Theta)."""
    import torch
    w = W.small("gk", 24, 16, nu=1e-2, omegas=(0.5, 2.5), k=6, q=1)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, list(w.omegas), "fp64", k_max=w.k, tile=32, test_matrix=kind, zeta=2)
    Q = f.sketch_solve(w.k, w.seed, w.q)
    Z = f.adjoint_solve(Q)
    ref = {key: to_np(v) for key, v in f.gains(Q, Z, "av").items() if v is not None}
    f.check()
    g = rr().capture(f, w.k, w.seed, w.q, "av", refactor=True)
    for rep in range(3):
        torch.cuda.synchronize()
        out = g.launch()
        f.check()
        for key in ("sigma_B", "sigma_AV", "V", "U"):
            np.testing.assert_array_equal(to_np(out[key]), ref[key])
    g.free()
    f.free()
