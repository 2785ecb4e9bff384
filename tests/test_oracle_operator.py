"""Pins for the oracle's Burgers operator and solver.

Central differences are exact on quadratics; pure convection of x gives -1;
the rows of a 3x3 grid are worked by hand; the half-bandwidth is 2*ny; the
band and sparse LU back-ends agree with a dense solve; the adjoint solve
passes the dot test.
"""
import numpy as np
import pytest

from oracle import operator as op
from oracle.solver import ShiftedSolver, SingularShift


def grid_fields(nx, ny, domain):
    hx, hy = op.spacing(nx, ny, domain)
    x = domain[0] + hx * np.arange(nx + 2)
    y = domain[2] + hy * np.arange(ny + 2)
    X, Y = np.meshgrid(x, y, indexing="ij")
    return hx, hy, X, Y


@pytest.mark.parametrize("nx,ny", [(3, 3), (7, 5), (16, 8), (5, 11)])
def test_half_bandwidth_is_two_ny(nx, ny):
    hx, hy, X, Y = grid_fields(nx, ny, (0, 8, -2, 2))
    U = np.tanh(Y / 0.5) + 0.1 * np.sin(X)
    L = op.assemble(op.burgers_coefficients(U, nx, ny, hx, hy, 1e-2))
    assert op.half_bandwidth(L) == 2 * ny
    assert L.shape == (2 * nx * ny, 2 * nx * ny)


def test_diffusion_exact_on_quadratic():
    nx, ny = 9, 7
    hx, hy, X, Y = grid_fields(nx, ny, (0.0, 2.0, -1.0, 0.5))
    U = np.zeros((nx + 2, ny + 2))
    L = op.assemble(op.burgers_coefficients(U, nx, ny, hx, hy, 1.0))
    f = (X ** 2 + Y ** 2)[1:-1, 1:-1].ravel()
    q = np.empty(2 * nx * ny)
    q[0::2] = f
    q[1::2] = f
    r = (L @ q).reshape(nx, ny, 2)
    inner = r[1:-1, 1:-1]              # nodes whose whole stencil is interior
    np.testing.assert_allclose(inner, 4.0, rtol=1e-10)


def test_convection_of_x():
    nx, ny = 8, 6
    hx, hy, X, Y = grid_fields(nx, ny, (0.0, 1.0, 0.0, 1.0))
    U = np.ones((nx + 2, ny + 2))      # U_x = U_y = 0
    L = op.assemble(op.burgers_coefficients(U, nx, ny, hx, hy, 0.0))
    q = np.empty(2 * nx * ny)
    q[0::2] = X[1:-1, 1:-1].ravel()
    q[1::2] = X[1:-1, 1:-1].ravel()
    r = (L @ q).reshape(nx, ny, 2)
    np.testing.assert_allclose(r[1:-1, :, :], -1.0, rtol=1e-12)


def test_hand_worked_3x3_rows():
    # domain [0,4]^2 on a 3x3 interior grid: h = 1.  nu = 0.5, U(i, j) = i + 2 j
    # on all 5x5 nodes, so U_x = 1 and U_y = 2 everywhere.  By hand:
    # centre node (1-based (2,2), p = 4): U = 6
    #   u-row 8: C = -2*0.5*(1+1) - 1 = -3, E = 0.5 - 6/2 = -2.5 (col 14),
    #            W = 0.5 + 3 = 3.5 (col 2), N = S = 0.5 (cols 10, 6), Cpl = -2 (col 9)
    #   v-row 9: C = -2, E = -2.5 (col 15), W = 3.5 (col 3), N = S = 0.5 (11, 7),
    #            no coupling to u
    # corner node (1,1), p = 0: U = 3
    #   u-row 0: C = -3, E = 0.5 - 1.5 = -1 (col 6), N = 0.5 (col 2), Cpl = -2 (col 1)
    I, J = np.meshgrid(np.arange(5), np.arange(5), indexing="ij")
    U = (I + 2 * J).astype(float)
    L = op.assemble(op.burgers_coefficients(U, 3, 3, 1.0, 1.0, 0.5)).toarray()
    row8 = {8: -3.0, 14: -2.5, 2: 3.5, 10: 0.5, 6: 0.5, 9: -2.0}
    row9 = {9: -2.0, 15: -2.5, 3: 3.5, 11: 0.5, 7: 0.5}
    row0 = {0: -3.0, 6: -1.0, 2: 0.5, 1: -2.0}
    for r, want in ((8, row8), (9, row9), (0, row0)):
        expect = np.zeros(18)
        for c, v in want.items():
            expect[c] = v
        np.testing.assert_array_equal(L[r], expect)


def small_problem(nx=10, ny=6, nu=2e-2, omega=1.3):
    hx, hy, X, Y = grid_fields(nx, ny, (0, 8, -2, 2))
    U = np.tanh(Y / 0.5) + 0.1 * np.exp(-Y ** 2) * np.sin(np.pi * X / 4)
    L = op.assemble(op.burgers_coefficients(U, nx, ny, hx, hy, nu))
    return L, op.shifted(L, omega)


def test_solver_backends_agree_with_dense():
    L, M = small_problem()
    rng = np.random.Generator(np.random.PCG64(0))
    B = rng.standard_normal((M.shape[0], 3)) + 1j * rng.standard_normal((M.shape[0], 3))
    Md = M.toarray()
    X0 = np.linalg.solve(Md, B)
    X0h = np.linalg.solve(Md.conj().T, B)
    for be in ("gb", "splu"):
        S = ShiftedSolver(M, be)
        np.testing.assert_allclose(S.solve(B), X0, rtol=1e-11, atol=1e-12 * np.abs(X0).max())
        np.testing.assert_allclose(S.solve_adjoint(B), X0h, rtol=1e-11,
                                   atol=1e-12 * np.abs(X0h).max())


def test_adjoint_dot_test():
    L, M = small_problem(12, 8)
    S = ShiftedSolver(M, "gb")
    rng = np.random.Generator(np.random.PCG64(1))
    n = M.shape[0]
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    lhs = np.vdot(S.solve(x), y)
    rhs = np.vdot(x, S.solve_adjoint(y))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    # and the operator itself: <M x, y> = <x, M^H y>
    assert abs(np.vdot(M @ x, y) - np.vdot(x, M.conj().T @ y)) <= 1e-12 * abs(np.vdot(M @ x, y))


def test_singular_shift_detected():
    # diagonal L with a zero eigenvalue and omega = 0: M has an exactly zero pivot
    c = np.zeros((2, 2, op.NCOEF))
    c[..., 0] = [[-1.0, -2.0], [0.0, -3.0]]
    c[..., 6] = -1.0
    L = op.assemble(c)
    M = op.shifted(L, 0.0)
    for be in ("gb", "splu"):
        with pytest.raises(SingularShift):
            ShiftedSolver(M, be)


def test_anisotropic_grid_closed_form():
    # h_x != h_y (0.5 against 0.6) and U = x^2 + 3y, whose central differences
    # are exact: U_x = 2x, U_y = 3, Phi = sqrt(4x^2 + 9) + 0.1.  A swap of h_x
    # and h_y anywhere in the coefficients or the weights fails here.
    from oracle import sketch
    nx, ny, nu = 5, 4, 0.3
    dom = (0.0, 3.0, -1.0, 2.0)
    hx, hy, X, Y = grid_fields(nx, ny, dom)
    assert abs(hx - 0.5) < 1e-15 and abs(hy - 0.6) < 1e-15
    U = X ** 2 + 3.0 * Y
    c = op.burgers_coefficients(U, nx, ny, hx, hy, nu)
    x = X[1:-1, 1:-1]
    Ui = U[1:-1, 1:-1]
    ax, ay = nu / hx ** 2, nu / hy ** 2
    want = np.empty_like(c)
    want[..., 0] = -2 * (ax + ay) - 2 * x
    want[..., 1] = ax - Ui / (2 * hx)
    want[..., 2] = ax + Ui / (2 * hx)
    want[..., 3] = want[..., 4] = ay
    want[..., 5] = -3.0
    want[..., 6] = -2 * (ax + ay)
    want[..., 7] = want[..., 1]
    want[..., 8] = want[..., 2]
    want[..., 9] = want[..., 10] = ay
    want[..., 11] = 0.0
    np.testing.assert_allclose(c, want, rtol=1e-13, atol=1e-13)
    phi = sketch.gradient_weight(U, hx, hy)
    np.testing.assert_allclose(phi, np.sqrt(4 * x ** 2 + 9) + 0.1, rtol=1e-14)


def test_anisotropic_diffusion_directions():
    # nu = 1, U = 0 on h_x = 0.5, h_y = 0.6: L x^2 = 2 and L y^2 = 2 at nodes
    # whose stencil is interior; with the spacings swapped they would be
    # 2 (0.6/0.5)^2 and 2 (0.5/0.6)^2
    nx, ny = 7, 6
    hx, hy, X, Y = grid_fields(nx, ny, (0.0, 4.0, -1.0, 3.2))
    assert abs(hx - 0.5) < 1e-15 and abs(hy - 0.6) < 1e-15
    L = op.assemble(op.burgers_coefficients(np.zeros((nx + 2, ny + 2)), nx, ny, hx, hy, 1.0))
    for f in (X ** 2, Y ** 2):
        q = np.zeros(2 * nx * ny)
        q[0::2] = f[1:-1, 1:-1].ravel()
        q[1::2] = f[1:-1, 1:-1].ravel()
        r = (L @ q).reshape(nx, ny, 2)
        np.testing.assert_allclose(r[1:-1, 1:-1], 2.0, rtol=1e-11)
