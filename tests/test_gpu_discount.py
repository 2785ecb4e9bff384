"""The discounted resolvent of Section 2.1 on the GPU: complex shifts
omega_r - i beta (the growth rates of L lowered by beta), against a closed
form, the oracle, and the identity that moves a diagonal shift of L into the
discount."""
import numpy as np
import pytest

import workloads as W
from oracle import operator as op
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import gain_errors, mode_angles, oracle_problem, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


def test_unstable_diagonal_operator_discounted_closed_form():
    """A normal operator with growing modes (Re lambda > 0): discounted by
    beta above the largest growth rate its gains are 1 / |i omega + beta -
    lambda|."""
    nx, ny = 8, 8
    n = 2 * nx * ny
    c = np.zeros((nx, ny, op.NCOEF))
    lam = -1e5 * (1.0 + np.arange(n) / n)
    lam[[3, 10, 17, 40]] = [0.3, 0.05, -0.2, -0.9]
    c[..., 0] = lam[0::2].reshape(nx, ny)
    c[..., 6] = lam[1::2].reshape(nx, ny)
    prob = rr().BurgersProblem.from_coefficients(c)
    omega, beta = 0.8, 0.5
    exact = np.sort(1.0 / np.abs(1j * omega + beta - lam))[::-1]
    for prec, tol in (("fp64", 1e-10), ("mixed", 1e-8)):
        out = rr().resolvent(prob, [omega], k=6, q=1, tile=32, precision=prec, discount=beta)
        np.testing.assert_allclose(out["factors"].omegas, [omega - 1j * beta])
        np.testing.assert_allclose(to_np(out["sigma_B"])[0, :4], exact[:4], rtol=tol)
        np.testing.assert_allclose(to_np(out["sigma_AV"])[0, :4], exact[:4], rtol=tol)
        out["factors"].free()


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-8)])
def test_discounted_pipeline_matches_oracle(prec, tol):
    w = W.small("d", 32, 24, nu=1e-2, omegas=(0.5, 2.0), k=8, q=1)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    beta = 0.3
    prob = rr().BurgersProblem.from_workload(w)
    out = rr().resolvent(prob, list(w.omegas), k=w.k, q=w.q, seed=w.seed, precision=prec,
                         tile=32, discount=beta)
    Om = osk.test_matrix(w.n, w.k, phi, w.seed)
    for i, om in enumerate(w.omegas):
        ref = ores.randomized_resolvent(L, om - 1j * beta, Om, q=w.q)
        assert gain_errors(to_np(out["sigma_B"][i]), ref.sigma_B).max() <= tol
        assert gain_errors(to_np(out["sigma_AV"][i]), ref.sigma_AV).max() <= tol
        assert mode_angles(to_np(out["V"][i]).T, ref.V, ref.sigma_B, 5) < 1e-6
        assert mode_angles(to_np(out["U"][i]).T, ref.U_AV, ref.sigma_B, 5) < 1e-6
    out["factors"].free()


def test_diagonal_shift_moves_into_the_discount():
    """L + gamma I discounted by beta is the same operator as L discounted by
    beta - gamma: M = i omega I - (L + gamma I - beta I)."""
    w = W.small("g", 24, 16, nu=1e-2, omegas=(0.7, 1.6), k=6, q=1)
    U, coef, L, phi, hx, hy = oracle_problem(w)
    gamma, beta = 0.4, 0.9
    c = coef.copy().reshape(w.nx, w.ny, op.NCOEF)
    c[..., 0] += gamma
    c[..., 6] += gamma
    shifted = rr().BurgersProblem.from_coefficients(c, phi=phi)
    base = rr().BurgersProblem.from_coefficients(coef.reshape(w.nx, w.ny, op.NCOEF), phi=phi)
    a = rr().resolvent(shifted, list(w.omegas), k=w.k, q=w.q, seed=w.seed, tile=32,
                       discount=beta)
    b = rr().resolvent(base, list(w.omegas), k=w.k, q=w.q, seed=w.seed, tile=32,
                       discount=beta - gamma)
    for key in ("sigma_B", "sigma_AV"):
        np.testing.assert_allclose(to_np(a[key]), to_np(b[key]), rtol=1e-10)
    a["factors"].free()
    b["factors"].free()
