"""Randomized resolvent analysis: Algorithm 1 with subspace iteration.

For one frequency omega and a test matrix Omega (n x k, Alg. 1 step 1 / eq. 10):
  step 2   Y = M^-1 Omega                  (sketch of the resolvent, eq. 6)
  step 3   Q = orth(Y)                     (economy QR, Section 2.2)
  (2.2.1)  q subspace iterations: Q <- orth(M^-1 orth(M^-H Q))
  step 4   B = Q^H M^-1 = Z^H with Z = M^-H Q
  step 5   B = Ut S V^H                    (reduced SVD, eq. 7)
  eq. 8    U_QU = Q Ut                     (Halko et al.'s response modes)
  step 6   U^Sigma = M^-1 V                (eq. 9: H v_j = sigma_j u_j)
  7-9      sigma_AV_j = ||U^Sigma_j||, u_j = U^Sigma_j / sigma_AV_j
  10-11    optional: svd(U^Sigma) = U S Vt, V <- V Vt

Here M = i*omega*I - L and H = M^-1 (see operator.shifted for the sign).
orth() is Householder QR with the phases of R's diagonal made real positive,
which makes Q unique and equal (in exact arithmetic) to any other QR of Y with
that normalisation, e.g. Cholesky QR.

Pins: closed-form gains of normal operators, the dense SVD of H at small n, the
bounds sigma_j(randomized) <= sigma_j(H), nesting in k, exactness at k = n
(tests/test_oracle_resolvent.py).
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

from .operator import shifted
from .solver import ShiftedSolver


def orth(Y: np.ndarray) -> np.ndarray:
    """Orthonormal basis of range(Y): Householder QR with diag(R) > 0."""
    Q, R = np.linalg.qr(Y, mode="reduced")
    d = np.diag(R)
    ph = np.where(np.abs(d) > 0, d / np.where(np.abs(d) > 0, np.abs(d), 1.0), 1.0)
    return Q * ph[None, :]


@dataclasses.dataclass
class Result:
    omega: complex
    sigma_B: np.ndarray      # k gains from the SVD of B (step 5)
    V: np.ndarray            # n x k forcing modes (step 5, or 11 if refined)
    U_QU: np.ndarray         # n x k response modes Q Ut (eq. 8)
    sigma_AV: np.ndarray     # k gains ||H v_j|| (steps 7-8)
    U_AV: np.ndarray         # n x k response modes H v_j / sigma_j (step 9)
    Q: np.ndarray            # n x k final orthonormal basis
    U_svd: Optional[np.ndarray] = None     # step 10 (optional)
    sigma_svd: Optional[np.ndarray] = None
    V_svd: Optional[np.ndarray] = None     # step 11 (optional)


def randomized_resolvent(L, omega: complex, Omega: np.ndarray, q: int = 0,
                         optional_svd: bool = False, backend: str = "auto",
                         solver: Optional[ShiftedSolver] = None) -> Result:
    M = shifted(L, omega)
    S = solver if solver is not None else ShiftedSolver(M, backend)
    Y = S.solve(Omega)                                  # step 2
    Q = orth(Y)                                         # step 3
    for _ in range(q):                                  # Section 2.2.1
        Q = orth(S.solve_adjoint(Q))
        Q = orth(S.solve(Q))
    Z = S.solve_adjoint(Q)                              # step 4: B = Z^H
    B = Z.conj().T
    Ut, s, Vh = np.linalg.svd(B, full_matrices=False)   # step 5
    V = Vh.conj().T
    US = S.solve(V)                                     # step 6
    sig_av = np.linalg.norm(US, axis=0)                 # step 8
    U_av = US / sig_av[None, :]                         # step 9
    res = Result(omega, s, V, Q @ Ut, sig_av, U_av, Q)
    if optional_svd:                                    # steps 10-11
        Uo, so, Vto = np.linalg.svd(US, full_matrices=False)
        res.U_svd, res.sigma_svd, res.V_svd = Uo, so, V @ Vto.conj().T
    return res


def run(L, omegas, Omega: np.ndarray, q: int = 0, **kw):
    """Algorithm 1 for each omega of a sweep, all sharing one L and one Omega."""
    return [randomized_resolvent(L, w, Omega, q=q, **kw) for w in omegas]
