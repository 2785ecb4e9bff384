"""Pins of the oracle's preconditioners (oracle/precond.py) against what their
definitions fix: block ILU(0) with a full pattern is the exact block LU; on a
one-line grid the pattern has no fill, so ILU(0) reproduces M; in 2-D,
(L U) equals M on every block of the pattern and differs from it off the
pattern; block Jacobi inverts node blocks exactly when M has nothing else."""
import numpy as np
import scipy.linalg as sla

import workloads as W
from oracle import operator as op
from oracle import precond as opc


def shifted_dense(nx, ny, nu=2e-2, omega=0.9 + 0.1j):
    w = W.small("pc", nx, ny, nu=nu)
    U = W.base_flow(w)
    hx, hy = op.spacing(nx, ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, nx, ny, hx, hy, nu))
    return op.shifted(L, omega).toarray()


def test_full_pattern_is_the_exact_block_lu():
    rng = np.random.default_rng(1)
    nb = 5
    M = rng.standard_normal((2 * nb, 2 * nb)) + 1j * rng.standard_normal((2 * nb, 2 * nb))
    M += 6 * np.eye(2 * nb)
    full = {(I, J) for I in range(nb) for J in range(nb)}
    L, U = opc.block_ilu0(M, full)
    np.testing.assert_allclose(L @ U, M, atol=1e-12)
    # the no-pivot block LU: identity diagonal blocks in L, nothing above them,
    # and nothing below the diagonal blocks of U
    for I in range(nb):
        np.testing.assert_allclose(L[2 * I:2 * I + 2, 2 * I:2 * I + 2], np.eye(2))
        assert not L[2 * I:2 * I + 2, 2 * I + 2:].any()
        assert not U[2 * I + 2:, 2 * I:2 * I + 2].any()


def test_one_line_grid_has_no_fill():
    for nx, ny in ((1, 9), (7, 1)):
        M = shifted_dense(nx, ny)
        L, U = opc.block_ilu0(M, opc.stencil_pattern(nx, ny))
        np.testing.assert_allclose(L @ U, M, atol=1e-12 * np.abs(M).max())


def test_product_matches_M_on_the_pattern_only():
    nx, ny = 4, 5
    M = shifted_dense(nx, ny)
    pat = opc.stencil_pattern(nx, ny)
    L, U = opc.block_ilu0(M, pat)
    P = L @ U
    on = np.zeros_like(M, dtype=bool)
    for (I, J) in pat:
        on[2 * I:2 * I + 2, 2 * J:2 * J + 2] = True
    np.testing.assert_allclose(P[on], M[on], atol=1e-12 * np.abs(M).max())
    # the dropped fill sits at (p, p + ny - 1)-type blocks, outside the pattern
    assert np.abs(P[~on]).max() > 1e-6 * np.abs(M).max()
    # L keeps M's own lower blocks scaled by the inverse pivots; U keeps M's
    # upper off-diagonal blocks unchanged (the 5-point structure)
    for (I, J) in pat:
        if J > I:
            np.testing.assert_allclose(U[2 * I:2 * I + 2, 2 * J:2 * J + 2],
                                       M[2 * I:2 * I + 2, 2 * J:2 * J + 2], atol=1e-14)


def test_block_jacobi_inverts_node_blocks():
    rng = np.random.default_rng(2)
    nb = 6
    M = np.zeros((2 * nb, 2 * nb), dtype=np.complex128)
    for I in range(nb):
        M[2 * I:2 * I + 2, 2 * I:2 * I + 2] = rng.standard_normal((2, 2)) + 1j * rng.standard_normal((2, 2)) + 3 * np.eye(2)
    X = rng.standard_normal((2 * nb, 3)) + 1j * rng.standard_normal((2 * nb, 3))
    K = opc.block_jacobi(M)
    np.testing.assert_allclose(K, M)
    np.testing.assert_allclose(opc.apply_inverse(K, X), sla.solve(M, X), atol=1e-13)
    np.testing.assert_allclose(opc.apply_inverse(K, X, adjoint=True), sla.solve(M.conj().T, X),
                               atol=1e-13)
