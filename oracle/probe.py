"""Unpivoted band-LU probe and conditioning report (informs the GPU design).

Not used for parity.  The paper (Section 3.1) only says that one LU of the
shifted operator is reused by the three solves.  A band LU without pivoting
keeps the band at kl = ku = b, but is only safe if element growth stays small;
this probe runs the textbook column-by-column elimination (no pivoting, no
blocking) on the band of M and reports growth and the smallest pivot, and the
conditioning report estimates ||M||_2 and kappa(M) = ||M||_2 sigma_1(H).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operator import half_bandwidth


def unpivoted_band_lu(M: sp.spmatrix):
    """Return (growth, min |pivot|, factored band) for the no-pivot LU of band M.

    Stores the band in a dense (n, 2b+1) array, row i holding M[i, i-b .. i+b].
    growth = max |U_ij| / max |M_ij| over the band.
    """
    n = M.shape[0]
    b = half_bandwidth(M)
    C = M.tocoo()
    A = np.zeros((n, 2 * b + 1), dtype=np.complex128)
    A[C.row, C.col - C.row + b] = C.data
    amax = np.abs(A).max()
    minpiv = np.inf
    for j in range(n):
        piv = A[j, b]
        minpiv = min(minpiv, abs(piv))
        if piv == 0:
            return np.inf, 0.0, A
        r1 = min(n, j + b + 1)
        rows = np.arange(j + 1, r1)
        if rows.size == 0:
            continue
        # multipliers: column j below the pivot sits at A[i, j - i + b]
        l = A[rows, j - rows + b] / piv
        A[rows, j - rows + b] = l
        # rank-1 update of rows j+1..j+b, columns j+1..j+b (inside the band)
        cols = np.arange(j + 1, min(n, j + b + 1))
        urow = A[j, cols - j + b]
        A[rows[:, None], cols[None, :] - rows[:, None] + b] -= l[:, None] * urow[None, :]
    umax = np.abs(A[:, b:]).max()
    return umax / amax, minpiv, A


def spectral_norm(M: sp.spmatrix, iters: int = 200, seed: int = 1) -> float:
    """||M||_2 by power iteration on M^H M with sparse products."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.standard_normal(M.shape[1]) + 1j * rng.standard_normal(M.shape[1])
    x /= np.linalg.norm(x)
    MH = M.conj().T.tocsr()
    s = 0.0
    for _ in range(iters):
        y = MH @ (M @ x)
        s_new = np.sqrt(np.linalg.norm(y))
        x = y / np.linalg.norm(y)
        if abs(s_new - s) <= 1e-10 * s_new:
            s = s_new
            break
        s = s_new
    return float(s)
