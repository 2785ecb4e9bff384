"""Brute-force resolvent SVD at small n (eq. 4 and eq. 5).

The resolvent H = M^-1 is formed explicitly and its full SVD H = U S V^H
taken with LAPACK.  This is the O(m^3) route the paper's method avoids; it is
only used to pin the randomized oracle on small problems.
"""
from __future__ import annotations

import numpy as np

from .operator import shifted


def resolvent_svd(L, omega: complex):
    """Full SVD of H(omega): (U, s, V) with H = U diag(s) V^H, s descending."""
    M = shifted(L, omega).toarray()
    H = np.linalg.inv(M)
    U, s, Vh = np.linalg.svd(H)
    return U, s, Vh.conj().T


def sin_angle(A: np.ndarray, B: np.ndarray) -> float:
    """sin of the largest principal angle between range(A) and range(B).

    Both are orthonormalised first; the value is ||(I - Qa Qa^H) Qb||_2, which
    is phase-free like the paper's cosine similarity (Section 3.2) and keeps
    its digits for nearly parallel subspaces.
    """
    A = np.asarray(A).reshape(A.shape[0], -1)
    B = np.asarray(B).reshape(B.shape[0], -1)
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    R = Qb - Qa @ (Qa.conj().T @ Qb)
    return float(np.linalg.norm(R, 2))
