"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Sizes span several band tiles and ragged tails (n not a multiple of the tile,
half-bandwidth not a multiple of the tile).  Tolerances:
  FP64 path:  sigma_j relative 1e-10 (gain_errors), mode sine angle < 1e-6
  mixed path: sigma_j relative 1e-8, mode sine angle < 1e-6
  bit-exact:  the Philox words; bitwise repeatability; batch == single shift
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import grad as ograd
from oracle import operator as op
from oracle import resolvent as ores
from oracle import sketch as osk
from oracle.philox import philox4x32_10
from oracle.solver import ShiftedSolver
from tests.gpu_util import gain_errors, mode_angles, oracle_problem, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib_loaded():
    import paper_1902_01458_amd as rr
    rr.lib()  # raises if librr.so is missing: there is no fallback
    assert torch.cuda.is_available()
    yield


def rr():
    import paper_1902_01458_amd as m
    return m


def test_philox_bitwise_matches_oracle():
    cnt = 100_000
    g = to_np(rr().philox_raw(cnt, c1=3, c2=5, key=(0x1234567, 0x89ABCDE)))
    o = philox4x32_10(np.arange(cnt, dtype=np.uint64), 3, 5, 0, 0x1234567, 0x89ABCDE)
    for t in range(4):
        np.testing.assert_array_equal(g[:, t], o[t].astype(np.int64))


def test_coefficients_and_sketch_match_oracle():
    w = W.CONFIGS["cfg0"]
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    np.testing.assert_allclose(to_np(prob.coef).reshape(coef.shape), coef, rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(to_np(prob.phi), phi, rtol=1e-15)
    th = to_np(rr().sketch(prob, w.k, seed=0)).T
    ref = osk.test_matrix(w.n, w.k, phi, seed=0)
    assert np.abs(th - ref).max() <= 1e-14 * np.abs(ref).max()


@pytest.mark.parametrize("adjoint", [False, True])
def test_apply_matches_oracle(adjoint):
    w = W.small("a", 9, 7, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.7, 1.3 + 0.2j]
    rng = np.random.Generator(np.random.PCG64(3))
    X = rng.standard_normal((2, 3, w.n)) + 1j * rng.standard_normal((2, 3, w.n))
    Y = to_np(prob.apply(oms, torch.tensor(X, device="cuda"), adjoint=adjoint))
    for i, om in enumerate(oms):
        M = op.shifted(L, om)
        if adjoint:
            M = M.conj().T
        ref = (M @ X[i].T).T
        np.testing.assert_allclose(Y[i], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


SOLVE_CASES = [  # (nx, ny, tile, k): ragged n and b, several tiles per half-band
    (10, 6, 32, 3),
    (13, 20, 64, 17),
    (24, 40, 32, 5),
    (9, 48, 64, 20),
    (16, 96, 32, 12),   # B = 6 tiles per half-band: early/final task split
    (12, 100, 64, 32),  # B = 4 at the 64 tile, ragged n, k = 32
    (8, 160, 32, 20),   # B = 10 at the 32 tile: superblock steps with more tiles than waves
    (6, 288, 64, 20),   # B = 9 at the 64 tile: the same at the benchmark's tile
]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny,tile,k", SOLVE_CASES)
def test_band_solve_matches_oracle(prec, nx, ny, tile, k):
    w = W.small("s", nx, ny, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.4, 2.5]
    f = rr().factor(prob, oms, prec, k_max=k, tile=tile)
    rng = np.random.Generator(np.random.PCG64(11))
    Bm = rng.standard_normal((2, k, w.n)) + 1j * rng.standard_normal((2, k, w.n))
    Bt = torch.tensor(Bm, device="cuda")
    X = to_np(f.solve(Bt))
    Z = to_np(f.adjoint_solve(Bt))
    f.check()
    tol = 1e-11 if prec == "fp64" else 1e-9
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref = S.solve(Bm[i].T).T
        refh = S.solve_adjoint(Bm[i].T).T
        assert np.linalg.norm(X[i] - ref) <= tol * np.linalg.norm(ref)
        assert np.linalg.norm(Z[i] - refh) <= tol * np.linalg.norm(refh)


def run_pipeline(w, prec, tile=64, omegas=None, response="av"):
    prob = rr().BurgersProblem.from_workload(w)
    oms = list(omegas if omegas is not None else w.omegas)
    out = rr().resolvent(prob, oms, k=w.k, q=w.q, seed=w.seed, precision=prec,
                         response=response, tile=tile)
    return {key: (to_np(v) if isinstance(v, torch.Tensor) else v) for key, v in out.items()}


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_cfg0_pipeline_matches_oracle(prec, tol):
    w = W.CONFIGS["cfg0"]
    U, coef, L, phi, hx, hy = oracle_problem(w)
    g = run_pipeline(w, prec)
    ref = ores.randomized_resolvent(L, w.omegas[0], osk.test_matrix(w.n, w.k, phi, w.seed), q=w.q)
    assert gain_errors(g["sigma_B"][0], ref.sigma_B).max() <= tol
    assert gain_errors(g["sigma_AV"][0], ref.sigma_AV).max() <= tol
    V = g["V"][0].T
    Uav = g["U"][0].T
    assert mode_angles(V, ref.V, ref.sigma_B, 5) < 1e-6
    assert mode_angles(Uav, ref.U_AV, ref.sigma_B, 5) < 1e-6
    Q = g["Q"][0].T
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(w.k), atol=1e-13)


def test_power_iteration_matches_oracle():
    w = W.small("p", 24, 16, nu=1e-2, omegas=(0.8, 2.0), k=8, q=1)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-8)):
        g = run_pipeline(w, prec, tile=32)
        Om = osk.test_matrix(w.n, w.k, phi, w.seed)
        for i, om in enumerate(w.omegas):
            ref = ores.randomized_resolvent(L, om, Om, q=1)
            assert gain_errors(g["sigma_B"][i], ref.sigma_B).max() <= tol
            assert gain_errors(g["sigma_AV"][i], ref.sigma_AV).max() <= tol


def test_halko_response_matches_oracle():
    w = W.small("h", 20, 12, nu=1e-2, omegas=(1.0,), k=6)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    g = run_pipeline(w, "fp64", tile=32, response="qu")
    ref = ores.randomized_resolvent(L, 1.0, osk.test_matrix(w.n, w.k, phi, w.seed))
    assert mode_angles(g["U"][0].T, ref.U_QU, ref.sigma_B, 4) < 1e-6


def test_diagonal_operator_closed_form():
    nx, ny = 8, 8
    n = 2 * nx * ny
    c = np.zeros((nx, ny, op.NCOEF))
    lam = -1e5 * (1.0 + np.arange(n) / n)
    lam[[3, 10, 17, 40]] = [-0.1, -0.25, -0.7, -1.5]
    c[..., 0] = lam[0::2].reshape(nx, ny)
    c[..., 6] = lam[1::2].reshape(nx, ny)
    prob = rr().BurgersProblem.from_coefficients(c)
    omega = 0.8
    exact = np.sort(1.0 / np.abs(1j * omega - lam))[::-1]
    out = rr().resolvent(prob, [omega], k=6, q=1, tile=32)
    np.testing.assert_allclose(to_np(out["sigma_B"])[0, :4], exact[:4], rtol=1e-10)
    np.testing.assert_allclose(to_np(out["sigma_AV"])[0, :4], exact[:4], rtol=1e-10)


def test_gradient_matches_oracle_formula():
    w = W.small("g", 16, 12, nu=3e-2, omegas=(0.9, 1.7), k=8, domain=(0.0, 8.0, -1.3, 2.2))
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=1, tile=32)
    f = out["factors"]
    s1 = out["sigma_AV"][:, 0].contiguous()
    dU, dnu, dom = f.grad(s1, out["U"], out["V"], stride=w.k * w.n)
    f.check()
    for i in range(len(w.omegas)):
        u = to_np(out["U"][i, 0])
        v = to_np(out["V"][i, 0])
        g, gnu, gom = ograd.gradient_full(float(s1[i]), u, v, w.nx, w.ny, hx, hy)
        np.testing.assert_allclose(to_np(dU[i]), g, rtol=0, atol=1e-12 * np.abs(g).max())
        assert abs(float(dnu[i]) - gnu) <= 1e-12 * abs(gnu)
        assert abs(float(dom[i]) - gom) <= 1e-12 * max(abs(gom), float(s1[i]))


def test_repeatable_and_batch_equals_single():
    w = W.small("b", 20, 16, nu=1e-2, omegas=(0.5, 1.0, 3.0), k=6)
    a = run_pipeline(w, "fp64", tile=32)
    b = run_pipeline(w, "fp64", tile=32)
    np.testing.assert_array_equal(a["sigma_B"], b["sigma_B"])
    np.testing.assert_array_equal(a["V"], b["V"])
    s = run_pipeline(w, "fp64", tile=32, omegas=[1.0])
    np.testing.assert_array_equal(a["sigma_B"][1], s["sigma_B"][0])
    np.testing.assert_array_equal(a["U"][1], s["U"][0])


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_refactor_is_bitwise_repeatable(prec):
    """Every refactorisation of one handle gives the same factor, bit for bit.

    Each band tile is written twice per launch (partial, then final) and read
    from other workgroups, usually on other XCDs; a stale read of the partial
    version gives a factor that is wrong (in FP64) or refines slowly (mixed).
    The arithmetic order of every tile is fixed, so repeated refactorisations
    and solves must agree exactly.
    """
    w = W.small("r", 96, 64, nu=5e-3, omegas=tuple(0.3 * 1.5 ** i for i in range(8)), k=8)
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, list(w.omegas), prec, k_max=w.k, tile=64)
    th = rr().sketch(prob, w.k, seed=0)
    Bm = th.unsqueeze(0).expand(len(w.omegas), w.k, prob.n).contiguous()
    X0 = f.solve(Bm)
    f.check()
    X0 = X0.clone()
    for _ in range(4):
        f.refactor()
        X = f.solve(Bm)
        f.check()
        assert torch.equal(X, X0)
    # and the factor is right: the residual of the FP64 path is at rounding level
    if prec == "fp64":
        R = Bm - prob.apply(list(w.omegas), X0)
        rel = (torch.linalg.vector_norm(R, dim=2) / torch.linalg.vector_norm(Bm, dim=2)).max()
        assert float(rel) < 1e-12


SUPERBLOCK_CASES = [  # (nx, ny, tile, k, superblock): B tiles per half-band against P
    (16, 96, 32, 12, 1),    # B = 6, one block row per step (diagonal inverses only)
    (16, 96, 32, 12, 3),    # B = 6, ragged superblocks (NB = 96 = 32 x 3)
    (13, 70, 32, 20, 8),    # B = 5 < P: the superblock spans more than the half-band
    (12, 100, 64, 32, 4),   # B = 4 = P, ragged n, k = 32
    (9, 48, 64, 17, 2),     # B = 2 = P, NB odd
    (10, 6, 32, 3, 5),      # B = 1, a partial last superblock
    (24, 40, 32, 5, -1),    # the tile-by-tile solve with chain tiles
]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("nx,ny,tile,k,sb", SUPERBLOCK_CASES)
def test_superblock_solve_matches_oracle(prec, nx, ny, tile, k, sb):
    """Forward and adjoint solves with every superblock size against LAPACK's
    banded solve (zgbtrs), FP64 (1e-11) and FP32 without refinement
    corrections (a 1e-4 bound on the normwise error: an FP32 LU, kappa ~ 1e2)."""
    w = W.small("sb", nx, ny, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.4, 2.5, 1.1]
    f = rr().factor(prob, oms, prec, k_max=k, tile=tile, superblock=sb, refine_tol=1.0)
    rng = np.random.Generator(np.random.PCG64(12))
    Bm = rng.standard_normal((3, k, w.n)) + 1j * rng.standard_normal((3, k, w.n))
    Bt = torch.tensor(Bm, device="cuda")
    X = to_np(f.solve(Bt))
    Z = to_np(f.adjoint_solve(Bt))
    f.check()
    tol = 1e-11 if prec == "fp64" else 1e-4
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref = S.solve(Bm[i].T).T
        refh = S.solve_adjoint(Bm[i].T).T
        ex = np.linalg.norm(X[i] - ref) / np.linalg.norm(ref)
        ez = np.linalg.norm(Z[i] - refh) / np.linalg.norm(refh)
        assert ex <= tol and ez <= tol, (i, ex, ez)
    f.free()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("tile,sb", [(32, 3), (64, 4)])
def test_superblock_solve_with_a_team_per_xcd_matches_oracle(prec, tile, sb):
    """Nine shifts: the solve's workgroups form a team per XCD, each serving
    only its own shifts (one team holds two) and handing blocks over through
    its XCD's L2 with plain stores.  Forward and adjoint solves against
    LAPACK's banded solve, at the tolerances of the test above."""
    w = W.small("sb9", 16, 96, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.25 * 1.45 ** i for i in range(9)]
    k = 20
    f = rr().factor(prob, oms, prec, k_max=k, tile=tile, superblock=sb, refine_tol=1.0)
    rng = np.random.Generator(np.random.PCG64(19))
    Bm = rng.standard_normal((len(oms), k, w.n)) + 1j * rng.standard_normal((len(oms), k, w.n))
    Bt = torch.tensor(Bm, device="cuda")
    X = to_np(f.solve(Bt))
    Z = to_np(f.adjoint_solve(Bt))
    f.check()
    tol = 1e-11 if prec == "fp64" else 1e-4
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref = S.solve(Bm[i].T).T
        refh = S.solve_adjoint(Bm[i].T).T
        ex = np.linalg.norm(X[i] - ref) / np.linalg.norm(ref)
        ez = np.linalg.norm(Z[i] - refh) / np.linalg.norm(refh)
        assert ex <= tol and ez <= tol, (i, ex, ez)
    f.free()


@pytest.mark.parametrize("k,probed", [(10, True), (20, True), (16, False)])
def test_first_refined_solve_measures_contraction(k, probed):
    """The first refined mixed solve after a factorisation measures the
    refinement's contraction.  With spare solve columns (k = 10 of 16, 20 of
    32) probe systems with known solutions ride along and measure it exactly
    on the first correction, so one correction is enough; with none spare
    (k = 16) a second correction measures it.  Every solve meets the
    tolerance against LAPACK's banded solve, also after a refactorisation
    (which measures again)."""
    w = W.small("pr", 40, 24, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.4, 2.5, 1.1]
    f = rr().factor(prob, oms, "mixed", k_max=k, tile=32, refine_tol=1e-8)
    rng = np.random.Generator(np.random.PCG64(31))
    Bm = rng.standard_normal((3, k, w.n)) + 1j * rng.standard_normal((3, k, w.n))
    Bt = torch.tensor(Bm, device="cuda")
    refs = []
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        refs.append((S.solve(Bm[i].T).T, S.solve_adjoint(Bm[i].T).T))

    def err(X, adj):
        return max(np.linalg.norm(X[i] - refs[i][adj]) / np.linalg.norm(refs[i][adj])
                   for i in range(3))

    counts = []
    for rep in range(2):
        X = to_np(f.solve(Bt))
        f.check()
        counts.append(f.refine_count())
        Z = to_np(f.adjoint_solve(Bt))
        f.check()
        counts.append(f.refine_count())
        X2 = to_np(f.solve(Bt))
        f.check()
        counts.append(f.refine_count())
        assert err(X, 0) <= 1e-8 and err(X2, 0) <= 1e-8 and err(Z, 1) <= 1e-8, \
            (rep, err(X, 0), err(X2, 0), err(Z, 1))
        f.refactor()
    print(f"\nk = {k}: corrections per solve {counts}")
    first = 1 if probed else 2
    assert counts == [first, 1, 1] * 2, counts
    f.free()


def test_adjoint_first_refined_solve_measures_with_a_second_correction():
    """Probe columns ride only in forward solves: a first refined solve that
    is an adjoint one measures the contraction by a second correction, and
    the solves after it stop after one; both meet the tolerance against
    LAPACK's banded solve."""
    w = W.small("pa", 40, 24, nu=2e-2)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    prob = rr().BurgersProblem.from_workload(w)
    oms = [0.4, 2.5, 1.1]
    k = 20
    f = rr().factor(prob, oms, "mixed", k_max=k, tile=32, refine_tol=1e-8)
    rng = np.random.Generator(np.random.PCG64(37))
    Bm = rng.standard_normal((3, k, w.n)) + 1j * rng.standard_normal((3, k, w.n))
    Bt = torch.tensor(Bm, device="cuda")
    Z = to_np(f.adjoint_solve(Bt))
    f.check()
    first = f.refine_count()
    X = to_np(f.solve(Bt))
    f.check()
    second = f.refine_count()
    for i, om in enumerate(oms):
        S = ShiftedSolver(op.shifted(L, om), "gb")
        ref, refh = S.solve(Bm[i].T).T, S.solve_adjoint(Bm[i].T).T
        assert np.linalg.norm(X[i] - ref) / np.linalg.norm(ref) <= 1e-8
        assert np.linalg.norm(Z[i] - refh) / np.linalg.norm(refh) <= 1e-8
    assert (first, second) == (2, 1), (first, second)
    f.free()
