"""Wide sketches, 32 < k <= 512 (the k study of Section 3.2, Fig. 7), FP64,
through the C ABI, against the oracle on the 64 x 32 configuration (n = 4096):

  * Algorithm 1 with one subspace iteration at k = 48, 100, 256 and 500
    (every column group of the band solve, the tiled Gram / Cholesky / k x k
    products and the wide Jacobi SVD): sigma_B and sigma_AV within 1e-10 of
    the oracle's pass on the same test matrix, and the leading modes within
    a sine angle of 1e-8;
  * the same through a Krylov handle (BiCGStab, ILU(0)) at k = 64;
  * the accuracy study itself: the leading gain against the dense SVD of the
    resolvent falls with k, and at k = 500 it is exact to 1e-10;
  * mixed precision keeps k <= 32."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense as odense
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import gain_errors, oracle_problem, sin_angle, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


W0 = W.CONFIGS["cfg0"]


@pytest.fixture(scope="module")
def problem():
    U, coef, L, phi, hx, hy = oracle_problem(W0)
    return L, phi


def run_gpu(k, omegas, q=1, **kw):
    prob = rr().BurgersProblem.from_workload(W0)
    out = rr().resolvent(prob, list(omegas), k=k, q=q, seed=W0.seed, precision="fp64", **kw)
    return {key: (to_np(v) if isinstance(v, torch.Tensor) else v) for key, v in out.items()}


@pytest.mark.parametrize("k", [48, 100, 256, 500])
def test_wide_pipeline_matches_oracle(problem, k):
    L, phi = problem
    oms = [1.0, 2.5 + 0.1j] if k <= 100 else [1.0]
    out = run_gpu(k, oms)
    Om = osk.test_matrix(W0.n, k, phi, seed=W0.seed)
    for i, om in enumerate(oms):
        ref = ores.randomized_resolvent(L, om, Om, q=1)
        top = min(k, 10)
        assert gain_errors(out["sigma_B"][i][:top], ref.sigma_B[:top]).max() <= 1e-10
        assert gain_errors(out["sigma_AV"][i][:top], ref.sigma_AV[:top]).max() <= 1e-10
        assert sin_angle(out["V"][i][:1].T, ref.V[:, :1]) <= 1e-8
        assert sin_angle(out["U"][i][:1].T, ref.U_AV[:, :1]) <= 1e-8


def test_wide_krylov_pipeline_matches_oracle(problem):
    L, phi = problem
    k = 64
    out = run_gpu(k, [1.0], solver="bicgstab", precond="ilu0", krylov_tol=1e-13,
                  krylov_maxit=2000)
    Om = osk.test_matrix(W0.n, k, phi, seed=W0.seed)
    ref = ores.randomized_resolvent(L, 1.0, Om, q=1)
    assert gain_errors(out["sigma_B"][0][:10], ref.sigma_B[:10]).max() <= 1e-9


def test_accuracy_against_k(problem):
    """Fig. 7's study on this operator at omega = 1, where sigma_1 / sigma_2 is
    only 1.003: |sigma_1(k) - sigma_1| / sigma_1 against the dense SVD falls
    steadily with k for the plain sketch (q = 0; about k^-0.8 here, the paper
    reports O(k) convergence), every point equal to the oracle's on the same
    test matrix; with one subspace iteration k = 500 is exact to 1e-9."""
    L, phi = problem
    U, s, V = odense.resolvent_svd(L, 1.0)
    ks = [2, 8, 32, 128, 500]
    err = []
    for k in ks:
        out = run_gpu(k, [1.0], q=0)
        ref = ores.randomized_resolvent(L, 1.0, osk.test_matrix(W0.n, k, phi, seed=W0.seed), q=0)
        assert gain_errors(out["sigma_B"][0][:1], ref.sigma_B[:1]).max() <= 1e-10
        err.append(abs(out["sigma_B"][0][0] - s[0]) / s[0])
    print("k-study, q = 0, sigma_1 rel. error:", dict(zip(ks, err)))
    assert all(a > b for a, b in zip(err, err[1:]))
    assert err[0] / err[-1] > 50
    out = run_gpu(500, [1.0], q=1)
    assert abs(out["sigma_B"][0][0] - s[0]) / s[0] <= 1e-9


def test_mixed_precision_keeps_narrow_sketches():
    prob = rr().BurgersProblem.from_workload(W0)
    with pytest.raises(rr().RRError) as e:
        rr().factor(prob, [1.0], "mixed", k_max=40)
    assert e.value.status == 1
