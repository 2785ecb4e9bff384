"""Preconditioners for LU-free solves (test infrastructure).

Section 3.2 ends by noting that BiCGStab or GMRES with an incomplete-LU or a
Jacobi preconditioner can take the place of the direct solves of Algorithm 1.
This module states the two preconditioners by their plain definitions, on the
shifted operator M = i*omega*I - L assembled as a dense matrix at small n, with
the unknowns grouped in 2 x 2 node blocks (u_p, v_p):

  block Jacobi   K = blockdiag(M_pp)
  block ILU(0)   K = L U, where L (unit block-lower) and U (block-upper) come
                 from block Gaussian elimination in natural node order in
                 which every update landing outside the block sparsity pattern
                 of M is dropped (Saad, Iterative Methods for Sparse Linear
                 Systems, 2nd ed., Sec. 10.3 and 10.7).  Its defining
                 property: (L U)_IJ = M_IJ on every block (I, J) of the pattern.

The pattern is structural (the stencil's node adjacency: the node itself and
its E, W, N, S neighbours inside the grid), not the numerical nonzeros.

Pins (tests/test_oracle_precond.py): ILU(0) with a full pattern is the exact
block LU; on a one-line grid (block tridiagonal, no fill) ILU(0) reproduces M;
(L U) = M on the pattern for a 2-D grid; block Jacobi against the inverted
node blocks of a diagonal-only operator.
"""
from __future__ import annotations

import numpy as np


def stencil_pattern(nx: int, ny: int) -> set:
    """Block pattern (I, J) of the 5-point node stencil, node p = j + ny*i."""
    pat = set()
    for i in range(nx):
        for j in range(ny):
            p = j + ny * i
            pat.add((p, p))
            if i > 0:
                pat.add((p, p - ny))
            if i < nx - 1:
                pat.add((p, p + ny))
            if j > 0:
                pat.add((p, p - 1))
            if j < ny - 1:
                pat.add((p, p + 1))
    return pat


def _blk(A, I, J, bs):
    return A[bs * I:bs * (I + 1), bs * J:bs * (J + 1)]


def block_jacobi(M: np.ndarray, bs: int = 2) -> np.ndarray:
    """K = the block diagonal of M (blocks of size bs)."""
    K = np.zeros_like(M)
    for I in range(M.shape[0] // bs):
        K[bs * I:bs * (I + 1), bs * I:bs * (I + 1)] = _blk(M, I, I, bs)
    return K


def block_ilu0(M: np.ndarray, pattern: set, bs: int = 2):
    """Block ILU(0) of M restricted to `pattern`: returns (L, U) dense, L unit
    block-lower, U block-upper, by the IKJ form of Gaussian elimination:
    for each block row I, for K < I in the pattern, L_IK = A_IK A_KK^-1 and
    A_IJ -= L_IK A_KJ for the J > K with (I, J) in the pattern."""
    nb = M.shape[0] // bs
    A = np.array(M, dtype=np.complex128, copy=True)
    rows = [sorted(J for (I, J) in pattern if I == r) for r in range(nb)]
    for I in range(nb):
        for K in [J for J in rows[I] if J < I]:
            lik = _blk(A, I, K, bs) @ np.linalg.inv(_blk(A, K, K, bs))
            A[bs * I:bs * (I + 1), bs * K:bs * (K + 1)] = lik
            for J in rows[I]:
                if J > K and (K, J) in pattern:
                    A[bs * I:bs * (I + 1), bs * J:bs * (J + 1)] -= lik @ _blk(A, K, J, bs)
    L = np.eye(M.shape[0], dtype=np.complex128)
    U = np.zeros_like(A)
    for (I, J) in pattern:
        if J < I:
            L[bs * I:bs * (I + 1), bs * J:bs * (J + 1)] = _blk(A, I, J, bs)
        else:
            U[bs * I:bs * (I + 1), bs * J:bs * (J + 1)] = _blk(A, I, J, bs)
    return L, U


def apply_inverse(K_or_LU, X: np.ndarray, adjoint: bool = False) -> np.ndarray:
    """K^-1 X (or K^-H X) for a dense K or an (L, U) pair, by a dense solve."""
    if isinstance(K_or_LU, tuple):
        L, U = K_or_LU
        K = L @ U
    else:
        K = K_or_LU
    if adjoint:
        K = K.conj().T
    return np.linalg.solve(K, X)
