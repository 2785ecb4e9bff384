"""LU-free solves (the paper's closing remark of Section 3.2: BiCGStab or GMRES
with an incomplete-LU or Jacobi preconditioner in place of the direct solves),
through the C ABI, against the oracle.

  * the preconditioners alone (rr_precond_apply) against oracle/precond.py's
    block Jacobi and block ILU(0), forward and adjoint, to 1e-12;
  * on a one-line grid ILU(0) has no fill: K^-1 is M^-1 itself (the oracle's
    LAPACK band solve), a pin that does not go through the oracle's ILU;
  * BiCGStab and restarted GMRES, each with both preconditioners, against the
    oracle's direct solves (residual tolerance 1e-11; forward error bound
    1e-9 relative at these condition numbers, kappa <= 1e2);
  * Algorithm 1 end to end on a Krylov handle against the oracle (1e-9 on
    sigma_j), a graph replay equal to the eager pass, and the error paths
    (not converged, FP64 only)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operator as op
from oracle import precond as opc
from oracle import resolvent as ores
from oracle import sketch as osk
from oracle.solver import ShiftedSolver
from tests.gpu_util import gain_errors, oracle_problem, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


def rand_block(shape, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("precond", ["jacobi", "ilu0"])
@pytest.mark.parametrize("adjoint", [False, True])
def test_preconditioner_matches_oracle(precond, adjoint):
    w = W.small("kp", 12, 10, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.7, 1.9 + 0.1j]
    f = rr().factor(prob, oms, "fp64", k_max=3, solver="bicgstab", precond=precond)
    X = rand_block((2, 3, w.n), 5)
    Xt = torch.tensor(X, device="cuda")
    Y = to_np(f.precond_apply(Xt, adjoint=adjoint))
    Yin = to_np(f.precond_apply(Xt.clone(), adjoint=adjoint, out=None))
    Xt2 = Xt.clone()
    f.precond_apply(Xt2, adjoint=adjoint, out=Xt2)  # in place
    f.check()
    pat = opc.stencil_pattern(w.nx, w.ny)
    for i, om in enumerate(oms):
        M = op.shifted(L, om).toarray()
        K = opc.block_jacobi(M) if precond == "jacobi" else opc.block_ilu0(M, pat)
        ref = opc.apply_inverse(K, X[i].T, adjoint=adjoint).T
        np.testing.assert_allclose(Y[i], ref, rtol=0, atol=1e-12 * np.abs(ref).max())
    np.testing.assert_array_equal(Yin, Y)
    np.testing.assert_array_equal(to_np(Xt2), Y)
    f.free()


@pytest.mark.parametrize("nx,ny", [(1, 37), (29, 1)])
@pytest.mark.parametrize("adjoint", [False, True])
def test_ilu0_is_the_exact_solve_on_a_line(nx, ny, adjoint):
    w = W.small("kl", nx, ny, nu=3e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.3, 2.2]
    f = rr().factor(prob, oms, "fp64", k_max=2, solver="gmres", precond="ilu0")
    X = rand_block((2, 2, w.n), 6)
    Y = to_np(f.precond_apply(torch.tensor(X, device="cuda"), adjoint=adjoint))
    f.check()
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref = (S.solve_adjoint(X[i].T) if adjoint else S.solve(X[i].T)).T
        assert np.linalg.norm(Y[i] - ref) <= 1e-12 * np.linalg.norm(ref)
    f.free()


SOLVERS = [("bicgstab", "jacobi"), ("bicgstab", "ilu0"), ("gmres", "jacobi"), ("gmres", "ilu0")]


@pytest.mark.parametrize("solver,precond", SOLVERS)
def test_krylov_solve_matches_oracle(solver, precond):
    w = W.small("ks", 24, 16, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.5, 2.3 + 0.1j]
    k = 4
    f = rr().factor(prob, oms, "fp64", k_max=k, solver=solver, precond=precond,
                    krylov_tol=1e-11, krylov_maxit=3000)
    B = rand_block((2, k, w.n), 7)
    Bt = torch.tensor(B, device="cuda")
    X = to_np(f.solve(Bt))
    Z = to_np(f.adjoint_solve(Bt))
    f.check()
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref = S.solve(B[i].T).T
        refh = S.solve_adjoint(B[i].T).T
        assert np.linalg.norm(X[i] - ref) <= 1e-9 * np.linalg.norm(ref)
        assert np.linalg.norm(Z[i] - refh) <= 1e-9 * np.linalg.norm(refh)
    f.free()


@pytest.mark.parametrize("solver", ["bicgstab", "gmres"])
def test_krylov_pipeline_matches_oracle(solver):
    w = W.CONFIGS["cfg0"]
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [w.omegas[0], 2.5]
    out = rr().resolvent(prob, oms, k=w.k, q=1, seed=w.seed, precision="fp64", solver=solver,
                         precond="ilu0", krylov_tol=1e-13, krylov_maxit=2000)
    Om = osk.test_matrix(w.n, w.k, phi, seed=w.seed)
    for i, om in enumerate(oms):
        ref = ores.randomized_resolvent(L, om, Om, q=1)
        assert gain_errors(to_np(out["sigma_B"][i]), ref.sigma_B).max() <= 1e-9
        assert gain_errors(to_np(out["sigma_AV"][i]), ref.sigma_AV).max() <= 1e-9


def test_krylov_graph_replay_equals_eager():
    w = W.small("kg", 20, 12, nu=3e-2, k=4)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, [0.8, 1.7], "fp64", k_max=w.k, solver="bicgstab", precond="ilu0",
                    krylov_tol=1e-12, krylov_maxit=60)
    Q = f.sketch_solve(w.k, 3, 1)
    Z = f.adjoint_solve(Q)
    eager = to_np(f.gains(Q, Z, "av")["sigma_AV"])
    f.check()
    g = rr().capture(f, w.k, 3, 1, "av", refactor=True)
    for _ in range(3):
        out = g.launch()
        torch.cuda.synchronize()
        np.testing.assert_array_equal(to_np(out["sigma_AV"]), eager)
        f.check()
    g.free()
    f.free()


def test_krylov_reports_non_convergence_and_fp64_only():
    w = W.small("kn", 20, 12, nu=1e-2)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, [0.4], "fp64", k_max=2, solver="bicgstab", precond="jacobi",
                    krylov_tol=1e-12, krylov_maxit=3)
    f.solve(torch.tensor(rand_block((1, 2, w.n), 8), device="cuda"))
    with pytest.raises(rr().RRError) as e:
        f.check()
    assert e.value.status == 3 and "Krylov" in str(e.value)
    f.free()
    with pytest.raises(rr().RRError) as e:
        rr().factor(prob, [0.4], "mixed", k_max=2, solver="gmres")
    assert e.value.status == 1
