"""Pins for the unpivoted band-LU probe and the spectral-norm estimate."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import operator as op, probe


def test_unpivoted_lu_reproduces_matrix():
    w = W.small("p", 6, 4, nu=2e-2)
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    M = op.shifted(op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu)), 0.7)
    growth, minpiv, A = probe.unpivoted_band_lu(M)
    n, b = M.shape[0], 2 * w.ny
    Lf = np.eye(n, dtype=complex)
    Uf = np.zeros((n, n), dtype=complex)
    for i in range(n):
        for d in range(-b, b + 1):
            j = i + d
            if 0 <= j < n:
                (Lf if d < 0 else Uf)[i, j] = A[i, d + b]
    np.testing.assert_allclose(Lf @ Uf, M.toarray(), atol=1e-12 * abs(M).max())
    assert 1.0 <= growth < 1e3 and minpiv > 0


def test_spectral_norm_matches_dense():
    rng = np.random.Generator(np.random.PCG64(9))
    A = sp.random(60, 60, density=0.2, random_state=1) + 1j * sp.random(60, 60, density=0.2,
                                                                       random_state=2)
    est = probe.spectral_norm(sp.csr_matrix(A), iters=2000)
    assert abs(est - np.linalg.norm(A.toarray(), 2)) <= 1e-6 * est


def diagonal_operator(lams, ny=4):
    """Diagonal L in the coefficient format: eigenvalue lams[2p + c] on row 2p + c."""
    lams = np.asarray(lams, dtype=float)
    nx = lams.size // (2 * ny)
    c = np.zeros((nx, ny, op.NCOEF))
    c[..., 0] = lams[0::2].reshape(nx, ny)
    c[..., 6] = lams[1::2].reshape(nx, ny)
    return op.assemble(c)


def test_conditioning_report_closed_form_on_a_normal_operator():
    # M = i omega I - diag(lam): ||M|| = max |i omega - lam|, sigma_1(H) = 1 /
    # min |i omega - lam|, so kappa is their ratio; with k = n the randomized
    # gains are exact, the eq. 9 triplet is an exact singular triplet (zero
    # residual), a diagonal has no element growth and both LUs agree exactly
    from oracle import sketch
    lam = np.concatenate([-np.linspace(0.05, 2.0, 31), [-6.0]])  # a well separated top
    L = diagonal_operator(lam)
    omega = 0.7
    d = np.abs(1j * omega - lam)
    Om = sketch.test_matrix(32, 32, None, seed=0)
    rep = probe.conditioning_report(L, omega, Om, q=0)
    assert abs(rep["norm_M"] - d.max()) <= 1e-10 * d.max()
    assert abs(rep["kappa"] - d.max() / d.min()) <= 1e-9 * d.max() / d.min()
    g = np.sort(1.0 / d)[::-1]
    assert abs(rep["gap12"] - g[0] / g[1]) <= 1e-12 * g[0] / g[1]
    assert abs(rep["gapk"] - g[-1] / g[0]) <= 1e-12
    assert rep["triplet_res"] <= 1e-13
    assert rep["growth"] == 1.0 and abs(rep["minpiv"] - d.min()) <= 1e-15
    assert rep["floor_measured"] <= 1e-14
    assert abs(rep["floor_pred"] - rep["kappa"] * 2.0 ** -53) <= 1e-30
    # below the floor the tolerance stays; above it it widens to 10x the measured floor
    assert probe.parity_tolerance(1e-10, rep) == 1e-10
    rep2 = dict(rep, floor_pred=1.0, floor_measured=3e-9)
    assert probe.parity_tolerance(1e-10, rep2) == 3e-8


def test_triplet_residual_matches_dense_resolvent():
    # non-normal Burgers operator with k < n: the residual through the
    # adjoint band solve against the same quantity with the dense inverse
    from oracle import resolvent, sketch
    w = W.small("p", 6, 4, nu=2e-2)
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    Om = sketch.test_matrix(w.n, 3, None, seed=0)
    rep = probe.conditioning_report(L, 0.7, Om, q=0)
    r = resolvent.randomized_resolvent(L, 0.7, Om, q=0)
    H = np.linalg.inv(op.shifted(L, 0.7).toarray())
    want = np.linalg.norm(H.conj().T @ r.U_AV[:, 0] - r.sigma_AV[0] * r.V[:, 0]) / r.sigma_AV[0]
    assert want > 1e-6                     # a genuinely inexact triplet
    assert abs(rep["triplet_res"] - want) <= 1e-8 * want
    assert rep["floor_measured"] < 1e-12   # unpivoted and pivoted LU agree here


def test_unpivoted_solver_matches_dense():
    w = W.small("p", 6, 4, nu=2e-2)
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    M = op.shifted(op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu)), 1.1)
    S = probe.UnpivotedSolver(M)
    rng = np.random.Generator(np.random.PCG64(2))
    B = rng.standard_normal((M.shape[0], 2)) + 1j * rng.standard_normal((M.shape[0], 2))
    Md = M.toarray()
    np.testing.assert_allclose(S.solve(B), np.linalg.solve(Md, B), rtol=1e-11)
    np.testing.assert_allclose(S.solve_adjoint(B), np.linalg.solve(Md.conj().T, B), rtol=1e-11)
