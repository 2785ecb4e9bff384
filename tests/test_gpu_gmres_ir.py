"""GMRES-IR for the mixed-precision solves (Carson & Higham): where plain
refinement with the FP32 LU stalls (kappa(M) eps_32 well above one, here a
shift 1e-7 |lambda| from the rightmost eigenvalue of a Burgers operator),
GMRES-IR still reaches the accuracy of an FP64 direct solve; elsewhere it
agrees with plain refinement and the oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import operator as op
from oracle import resolvent as ores
from oracle import sketch as osk
from oracle.solver import ShiftedSolver
from tests.gpu_util import gain_errors, oracle_problem, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


def rhs(n, k, seed=0):
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((1, k, n)) + 1j * rng.standard_normal((1, k, n))
    return B, torch.as_tensor(B, device="cuda")


@pytest.mark.parametrize("nx,ny", [(32, 16), (24, 48)])
def test_gmres_ir_converges_where_plain_refinement_stalls(nx, ny):
    """At a shift 1e-7 |lambda| from an eigenvalue (kappa(M) u_32 >> 1) plain
    refinement stalls and GMRES-IR with the FP32 factor as preconditioner
    converges.  With T = 32 the 32 x 16 grid's band is one tile wide (every
    update is a tile's last, four real MFMAs); the 24 x 48 grid's is three,
    so its FP32 factor also has early updates, which take Gauss products."""
    w = W.small("i", nx, ny, nu=1e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    lam = np.linalg.eigvals(L.toarray())
    lam0 = lam[np.argmax(lam.real)]
    omega = -1j * (lam0 + 1e-7 * abs(lam0))  # M = (lam0 + delta) I - L, nearly singular
    B, Bt = rhs(w.n, 4)
    ref = ShiftedSolver(op.shifted(L, omega), "gb").solve(B[0].T).T
    prob = rr().BurgersProblem.from_workload(w)
    errs = {}
    for method in ("plain", "gmres"):
        f = rr().factor(prob, [omega], "mixed", k_max=4, tile=32, refine_iters=6, refine_tol=1e-6,
                        refine_method=method, gmres_restart=8)
        X = f.solve(Bt)
        if method == "plain":
            with pytest.raises(rr().RRError) as e:
                f.check()
            assert e.value.status == 3  # RR_ERR_NOT_CONVERGED
        else:
            f.check()
        errs[method] = float(np.linalg.norm(to_np(X)[0] - ref) / np.linalg.norm(ref))
        f.free()
    print(f"\nforward error against the FP64 direct solve: plain {errs['plain']:.1e}, "
          f"GMRES-IR {errs['gmres']:.1e}")
    assert errs["gmres"] < 1e-5
    assert errs["gmres"] < 1e-2 * errs["plain"]


@pytest.mark.parametrize("adjoint", [False, True])
def test_gmres_ir_matches_oracle_on_ordinary_shifts(adjoint):
    w = W.small("j", 24, 16, nu=1e-2, omegas=(0.5, 2.0))
    U, coef, L, phi, hx, hy = oracle_problem(w)
    B, Bt = rhs(w.n, 5, seed=1)
    Bt = Bt.expand(2, 5, w.n).contiguous()
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, list(w.omegas), "mixed", k_max=5, tile=32, refine_method="gmres",
                    gmres_restart=4)
    X = f.adjoint_solve(Bt) if adjoint else f.solve(Bt)
    f.check()
    for i, om in enumerate(w.omegas):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref = (S.solve_adjoint(B[0].T) if adjoint else S.solve(B[0].T)).T
        assert np.linalg.norm(to_np(X)[i] - ref) <= 1e-10 * np.linalg.norm(ref)
    f.free()


def test_gmres_ir_pipeline_matches_oracle():
    w = W.CONFIGS["cfg0"]
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, seed=w.seed, precision="mixed",
                         refine_method="gmres", gmres_restart=6)
    ref = ores.randomized_resolvent(L, w.omegas[0], osk.test_matrix(w.n, w.k, phi, w.seed),
                                    q=w.q)
    assert gain_errors(to_np(out["sigma_B"])[0], ref.sigma_B).max() <= 1e-8
    assert gain_errors(to_np(out["sigma_AV"])[0], ref.sigma_AV).max() <= 1e-8
    out["factors"].free()


def test_gmres_ir_graph_replays_equal_eager_pass():
    """A captured pass with GMRES-IR corrections (fills and kernels only)
    replays bit for bit what the eager calls compute, with unrelated eager
    work and synchronisations between the replays."""
    w = W.small("gg", 32, 24, nu=1e-2, omegas=(0.4, 1.7, 4.0), k=6, q=1)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, list(w.omegas), "mixed", k_max=w.k, tile=32, refine_method="gmres",
                    gmres_restart=4)
    Q = f.sketch_solve(w.k, w.seed, w.q)
    Z = f.adjoint_solve(Q)
    ref = f.gains(Q, Z, "av")
    f.check()
    ref = {key: to_np(v) for key, v in ref.items() if v is not None}
    g = rr().capture(f, w.k, w.seed, w.q, "av", refactor=True)
    X = torch.randn((len(w.omegas), 3, w.n), dtype=torch.complex128, device="cuda")
    for rep in range(3):
        Y = prob.apply(list(w.omegas), X)
        torch.cuda.synchronize()
        assert torch.isfinite(torch.view_as_real(Y)).all()
        out = g.launch()
        f.check()
        for key in ("sigma_B", "sigma_AV", "V", "U"):
            np.testing.assert_array_equal(to_np(out[key]), ref[key])
    g.free()
    f.free()
