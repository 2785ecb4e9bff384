"""Pins for the oracle's gradient of the leading gain.

The stencil reduction is checked against a node-by-node differentiation of the
coefficient array; the first-order perturbation formula (and its signs) against
central finite differences of the exact sigma_1 from the dense SVD (eq. 5);
the randomized triplet at full width against the dense one.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, grad, operator as op, resolvent, sketch


def problem(nx=7, ny=5, nu=3e-2):
    # an off-centre domain breaks the near up-down symmetry of the shear layer,
    # so sigma_1 is simple (sigma_1 / sigma_2 ~ 1.56)
    w = W.small("g", nx, ny, nu=nu, domain=(0.0, 8.0, -1.3, 2.2))
    U = W.base_flow(w)
    hx, hy = op.spacing(nx, ny, w.domain)
    return w, U, hx, hy


def sigma1(U, nx, ny, hx, hy, nu, omega):
    L = op.assemble(op.burgers_coefficients(U, nx, ny, hx, hy, nu))
    Ud, s, Vd = dense.resolvent_svd(L, omega)
    return s, Ud, Vd


def test_stencil_reduction_matches_bruteforce():
    w, U, hx, hy = problem()
    rng = np.random.Generator(np.random.PCG64(5))
    n = w.n
    u = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    v = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    g, _, _ = grad.gradient(1.7, u, v, w.nx, w.ny, hx, hy)
    gb = grad.gradient_bruteforce(1.7, u, v, U, w.nx, w.ny, hx, hy, w.nu)
    np.testing.assert_allclose(g, gb, rtol=1e-12, atol=1e-12 * np.abs(gb).max())


def test_formula_matches_finite_differences_of_exact_gain():
    w, U, hx, hy = problem()
    omega = 0.9
    s, Ud, Vd = sigma1(U, w.nx, w.ny, hx, hy, w.nu, omega)
    assert s[0] / s[1] > 1.01      # simple leading singular value
    g, gnu, gom = grad.gradient(s[0], Ud[:, 0], Vd[:, 0], w.nx, w.ny, hx, hy)
    h = 1e-6
    for (i, j) in [(0, 0), (3, 2), (6, 4), (2, 0), (5, 3)]:
        Up, Um = U.copy(), U.copy()
        Up[i + 1, j + 1] += h
        Um[i + 1, j + 1] -= h
        fd = (sigma1(Up, w.nx, w.ny, hx, hy, w.nu, omega)[0][0]
              - sigma1(Um, w.nx, w.ny, hx, hy, w.nu, omega)[0][0]) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * np.abs(g).max()
    fd_nu = (sigma1(U, w.nx, w.ny, hx, hy, w.nu + h, omega)[0][0]
             - sigma1(U, w.nx, w.ny, hx, hy, w.nu - h, omega)[0][0]) / (2 * h)
    assert abs(fd_nu - gnu) <= 1e-6 * abs(gnu)
    fd_om = (sigma1(U, w.nx, w.ny, hx, hy, w.nu, omega + h)[0][0]
             - sigma1(U, w.nx, w.ny, hx, hy, w.nu, omega - h)[0][0]) / (2 * h)
    assert abs(fd_om - gom) <= 1e-6 * max(abs(gom), 1e-3 * s[0])


def test_full_width_randomized_triplet_gives_dense_gradient():
    w, U, hx, hy = problem()
    omega = 0.9
    s, Ud, Vd = sigma1(U, w.nx, w.ny, hx, hy, w.nu, omega)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    r = resolvent.randomized_resolvent(L, omega, sketch.test_matrix(w.n, w.n, None), q=0)
    g_r = grad.gradient(r.sigma_AV[0], r.U_AV[:, 0], r.V[:, 0], w.nx, w.ny, hx, hy)
    g_d = grad.gradient(s[0], Ud[:, 0], Vd[:, 0], w.nx, w.ny, hx, hy)
    np.testing.assert_allclose(g_r[0], g_d[0], atol=1e-8 * np.abs(g_d[0]).max())
    assert abs(g_r[1] - g_d[1]) <= 1e-8 * abs(g_d[1])
    assert abs(g_r[2] - g_d[2]) <= 1e-8 * max(abs(g_d[2]), s[0])


def test_gradient_is_phase_invariant():
    w, U, hx, hy = problem()
    rng = np.random.Generator(np.random.PCG64(6))
    u = rng.standard_normal(w.n) + 1j * rng.standard_normal(w.n)
    v = rng.standard_normal(w.n) + 1j * rng.standard_normal(w.n)
    a = grad.gradient(2.0, u, v, w.nx, w.ny, hx, hy)
    ph = np.exp(0.7j)
    b = grad.gradient(2.0, u * ph, v * ph, w.nx, w.ny, hx, hy)
    np.testing.assert_allclose(a[0], b[0], atol=1e-13 * np.abs(a[0]).max())
    assert abs(a[1] - b[1]) < 1e-12 * abs(a[1]) and abs(a[2] - b[2]) < 1e-12 * (abs(a[2]) + 1)


def test_ring_terms_match_bruteforce():
    # every node of the (nx+2, ny+2) array, ring included: the term-by-term
    # formula against the node-by-node differentiation of the coefficients
    w, U, hx, hy = problem()
    rng = np.random.Generator(np.random.PCG64(8))
    u = rng.standard_normal(w.n) + 1j * rng.standard_normal(w.n)
    v = rng.standard_normal(w.n) + 1j * rng.standard_normal(w.n)
    g, dnu, dom = grad.gradient_full(1.3, u, v, w.nx, w.ny, hx, hy)
    gb = grad.gradient_bruteforce(1.3, u, v, U, w.nx, w.ny, hx, hy, w.nu, ring=True)
    np.testing.assert_allclose(g, gb, rtol=1e-12, atol=1e-12 * np.abs(gb).max())
    assert np.abs(g[0, 1:-1]).max() > 0 and np.abs(g[1:-1, -1]).max() > 0
    assert g[0, 0] == g[0, -1] == g[-1, 0] == g[-1, -1] == 0.0
    g0, dnu0, dom0 = grad.gradient(1.3, u, v, w.nx, w.ny, hx, hy)
    np.testing.assert_array_equal(g[1:-1, 1:-1], g0)
    assert (dnu, dom) == (dnu0, dom0)


def test_ring_formula_matches_finite_differences_of_exact_gain():
    w, U, hx, hy = problem()
    omega = 0.9
    s, Ud, Vd = sigma1(U, w.nx, w.ny, hx, hy, w.nu, omega)
    g, _, _ = grad.gradient_full(s[0], Ud[:, 0], Vd[:, 0], w.nx, w.ny, hx, hy)
    h = 1e-6
    for (i, j) in [(0, 2), (w.nx + 1, 3), (4, 0), (2, w.ny + 1), (0, 0)]:
        Up, Um = U.copy(), U.copy()
        Up[i, j] += h
        Um[i, j] -= h
        fd = (sigma1(Up, w.nx, w.ny, hx, hy, w.nu, omega)[0][0]
              - sigma1(Um, w.nx, w.ny, hx, hy, w.nu, omega)[0][0]) / (2 * h)
        assert abs(fd - g[i, j]) <= 1e-6 * np.abs(g).max(), (i, j, fd, g[i, j])
