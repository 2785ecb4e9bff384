"""Factor once, solve many: linear solves with M(omega) = i*omega*I - L.

Section 3.1 notes that the three linear solves of Algorithm 1 (steps 2, 4, 6)
share one LU factorisation of the shifted operator, computed once and reused.
Two library back-ends serve as that step:
  "gb"    LAPACK zgbtrf / zgbtrs (band LU with partial pivoting, kl = ku = b)
  "splu"  SuperLU (sparse LU with partial pivoting and a fill-reducing order)
The band back-end is the default for small n; SuperLU keeps large problems
(n ~ 1e5-1e6) tractable on a CPU, where a band solve would stream the full
band once per right-hand side.

Pins: residual of M X - B, agreement of the two back-ends, dense solve at small
n, and the adjoint dot test <M^-1 x, y> = <x, M^-H y>.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla
from scipy.linalg import lapack

from .operator import half_bandwidth, lapack_band


class SingularShift(RuntimeError):
    """The shifted operator has an exactly zero pivot (omega hits an eigenvalue)."""


class ShiftedSolver:
    def __init__(self, M: sp.spmatrix, backend: str = "auto"):
        self.n = M.shape[0]
        if backend == "auto":
            backend = "gb" if self.n <= 20000 else "splu"
        self.backend = backend
        if backend == "gb":
            b = half_bandwidth(M)
            self.kl = self.ku = b
            AB = lapack_band(M, b, b)
            lu, ipiv, info = lapack.zgbtrf(AB, b, b)
            if info > 0:
                raise SingularShift(f"zero pivot at column {info}")
            if info < 0:
                raise ValueError(f"zgbtrf argument {-info}")
            self.lu, self.ipiv = lu, ipiv
        elif backend == "splu":
            try:
                self.lu = spla.splu(sp.csc_matrix(M), permc_spec="COLAMD")
            except RuntimeError as e:  # SuperLU reports exact singularity this way
                raise SingularShift(str(e)) from e
        else:
            raise ValueError(backend)

    def solve(self, B: np.ndarray) -> np.ndarray:
        """X = M^-1 B (Algorithm 1 steps 2 and 6)."""
        return self._solve(B, 0)

    def solve_adjoint(self, B: np.ndarray) -> np.ndarray:
        """X = M^-H B, so that X^H = B^H M^-1 (Algorithm 1 step 4)."""
        return self._solve(B, 2)

    def _solve(self, B: np.ndarray, trans: int) -> np.ndarray:
        B = np.asarray(B, dtype=np.complex128)
        vec = B.ndim == 1
        B2 = B.reshape(self.n, -1)
        if self.backend == "gb":
            X, info = lapack.zgbtrs(self.lu, self.kl, self.ku, np.asfortranarray(B2),
                                    self.ipiv, trans=trans)
            if info != 0:
                raise ValueError(f"zgbtrs info {info}")
        else:
            X = self.lu.solve(np.asfortranarray(B2), trans={0: "N", 2: "H"}[trans])
        return X.reshape(-1) if vec else X
