"""Degenerate and limit cases on the GPU: one block row with a full-rank
sketch (k = n, where the randomized SVD is exact), a one-column sketch on two
block rows, and a batch of more shifts than one factor launch takes."""
import numpy as np
import pytest

import workloads as W
from oracle import dense as odense
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import gain_errors, oracle_problem, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_single_block_row_full_rank_sketch_is_exact(prec, tol):
    w = W.small("e", 4, 4, nu=5e-2, omegas=(0.7,), k=32)  # n = 32 = one 32-tile block row
    assert w.n == 32
    U, coef, L, phi, hx, hy = oracle_problem(w)
    Ud, sd, Vd = odense.resolvent_svd(L, 0.7)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, [0.7], k=32, seed=w.seed, precision=prec, tile=32)
    assert gain_errors(to_np(out["sigma_B"])[0], sd).max() <= tol
    assert gain_errors(to_np(out["sigma_AV"])[0], sd).max() <= tol
    out["factors"].free()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_one_column_sketch_on_two_block_rows(prec, tol):
    w = W.small("f", 8, 4, nu=5e-2, omegas=(0.3, 1.9), k=1, q=1)  # n = 64: two block rows
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=1, q=1, seed=w.seed, precision=prec, tile=32)
    Om = osk.test_matrix(w.n, 1, phi, w.seed)
    for i, om in enumerate(w.omegas):
        ref = ores.randomized_resolvent(L, om, Om, q=1)
        assert gain_errors(to_np(out["sigma_B"])[i], ref.sigma_B).max() <= tol
        assert gain_errors(to_np(out["sigma_AV"])[i], ref.sigma_AV).max() <= tol
    out["factors"].free()


def test_more_shifts_than_one_factor_launch():
    """70 shifts: the factorisation runs as two launches (64 + 6)."""
    omegas = tuple(np.linspace(0.1, 7.0, 70))
    w = W.small("g", 12, 10, nu=2e-2, omegas=omegas, k=4)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(omegas), k=4, seed=w.seed, tile=32)
    Om = osk.test_matrix(w.n, 4, phi, w.seed)
    for i in (0, 1, 63, 64, 65, 69):
        ref = ores.randomized_resolvent(L, omegas[i], Om, q=0)
        assert gain_errors(to_np(out["sigma_B"])[i], ref.sigma_B).max() <= 1e-10, i
        assert gain_errors(to_np(out["sigma_AV"])[i], ref.sigma_AV).max() <= 1e-10, i
    out["factors"].free()


def test_jacobi_svd_reports_non_convergence():
    """With the Jacobi SVD capped at one sweep, a k x k factor that is not
    already diagonal still rotates at the cap: rr_check reports
    RR_ERR_NOT_CONVERGED instead of returning unconverged gains silently;
    the default cap on the same handle converges and matches the oracle."""
    w = W.small("j", 12, 8, nu=2e-2, omegas=(0.9,), k=12)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, list(w.omegas), "fp64", k_max=w.k, tile=32)
    Q = f.sketch_solve(w.k, w.seed, 0)
    Z = f.adjoint_solve(Q)
    f.set_jacobi_sweeps(1)
    f.gains(Q, Z, "av")
    with pytest.raises(rr().RRError) as e:
        f.check()
    assert e.value.status == 3 and "Jacobi" in str(e.value)
    f.set_jacobi_sweeps(40)
    out = f.gains(Q, Z, "av")
    f.check()
    U, coef, L, phi, hx, hy = oracle_problem(w)
    ref = ores.randomized_resolvent(L, 0.9, osk.test_matrix(w.n, w.k, phi, w.seed), q=0)
    assert gain_errors(to_np(out["sigma_B"])[0], ref.sigma_B).max() <= 1e-10
    f.free()
