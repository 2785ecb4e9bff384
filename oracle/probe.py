"""Unpivoted band-LU probe and conditioning report.

The paper (Section 3.1) only says that one LU of the shifted operator is
reused by the three solves.  A band LU without pivoting keeps the band at
kl = ku = b, but is only safe if element growth stays small; this probe runs
the textbook column-by-column elimination (no pivoting, no blocking) on the
band of M and reports growth and the smallest pivot.  The conditioning report
estimates ||M||_2 and kappa(M) = ||M||_2 sigma_1(H), the gaps of the gains,
the quality of the eq. 9 triplet, and the parity floor that the choice of
pivoting alone sets (Algorithm 1 run once with each LU); `parity_tolerance`
turns it into the tolerance a parity test may use.

Pins (tests/test_oracle_probe.py): L U reproduces M; the norm estimate
against a dense 2-norm; on a diagonal (normal) operator kappa, the gaps, a
zero triplet residual, unit growth and a zero floor are known in closed form;
the unpivoted solver against a dense solve.

Command line (the figures quoted for the benchmark operator come from it):
    python -m oracle.probe cfg1 2.0 [--unpivoted]
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from scipy.linalg import lapack

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


class UnpivotedSolver:
    """Solves with the unpivoted band LU of `unpivoted_band_lu` (the GPU
    path's factorisation without pivoting), by two LAPACK band triangular
    solves (ztbtrs) per application: L (unit lower) then U for M, U^H then
    L^H for M^H.  Same interface as solver.ShiftedSolver."""

    def __init__(self, M: sp.spmatrix):
        growth, minpiv, A = unpivoted_band_lu(M)
        if not np.isfinite(growth):
            raise ZeroDivisionError("zero pivot in the unpivoted band LU")
        self.growth, self.minpiv = growth, minpiv
        n, w = A.shape
        b = (w - 1) // 2
        self.n, self.b = n, b
        # LAPACK triangular band storage: upper AB[b + i - j, j] = U[i, j],
        # lower AB[i - j, j] = L[i, j]; the probe's row i holds M[i, i + d] at d + b
        self.ABu = np.zeros((b + 1, n), dtype=np.complex128, order="F")
        self.ABl = np.zeros((b + 1, n), dtype=np.complex128, order="F")
        for d in range(0, b + 1):        # U[i, i + d] -> ABu[b - d, i + d]
            i = np.arange(0, n - d)
            self.ABu[b - d, i + d] = A[i, d + b]
        self.ABl[0, :] = 1.0
        for d in range(1, b + 1):        # L[i, i - d] -> ABl[d, i - d]
            i = np.arange(d, n)
            self.ABl[d, i - d] = A[i, b - d]

    def _tb(self, AB, X, uplo, trans):
        diag = b"U" if uplo == b"L" else b"N"
        Y, info = lapack.ztbtrs(AB, np.asfortranarray(X), uplo=uplo, trans=trans, diag=diag)
        if info != 0:
            raise ValueError(f"ztbtrs info {info}")
        return Y

    def solve(self, B):
        B2 = np.asarray(B, dtype=np.complex128).reshape(self.n, -1)
        X = self._tb(self.ABu, self._tb(self.ABl, B2, b"L", b"N"), b"U", b"N")
        return X.reshape(np.shape(B))

    def solve_adjoint(self, B):
        B2 = np.asarray(B, dtype=np.complex128).reshape(self.n, -1)
        X = self._tb(self.ABl, self._tb(self.ABu, B2, b"U", b"C"), b"L", b"C")
        return X.reshape(np.shape(B))


EPS64 = 2.0 ** -53   # unit roundoff, FP64
EPS32 = 2.0 ** -24   # unit roundoff, FP32


def conditioning_report(L: sp.spmatrix, omega: complex, Omega: np.ndarray, q: int = 0,
                        unpivoted: bool = True, norm_iters: int = 200) -> dict:
    """What bounds parity at one shift: conditioning, gaps and the accuracy floor.

    From one run of Algorithm 1 (resolvent.randomized_resolvent, pivoted LU)
    with test matrix Omega and q subspace iterations:
      norm_M          ||M||_2, power iteration on M^H M (sparse products)
      sigma           the gains sigma_B; sigma[0] stands in for sigma_1(H)
      kappa           ||M||_2 sigma_1: the condition number of M to leading order
      floor_pred      kappa * u64, the relative accuracy FP64 solves can promise
      gap12, gapk     sigma_1 / sigma_2 and sigma_k / sigma_1
      triplet_res     ||H^H u_1 - sigma_1 v_1|| / sigma_1 with the eq. 9 triplet
                      (sigma_AV_1, u_AV_1, v_1): one adjoint solve.  H v_1 =
                      sigma u_1 holds by construction, so this measures how far
                      the triplet is from a singular triplet of H
    and, with unpivoted=True (the unpivoted band LU, as the GPU factors):
      growth, minpiv  element growth max|U| / max|M| and the smallest pivot
      contraction_pred  kappa * growth * u32: the error left per correction by
                      FP32 iterative refinement
      floor_measured  max_j |sigma_B,j(unpivoted) - sigma_B,j(pivoted)| / sigma_1:
                      the same algorithm with the two LUs, i.e. the parity floor
                      the pivoting choice alone sets
    """
    from .resolvent import randomized_resolvent
    from .operator import shifted
    from .solver import ShiftedSolver

    M = shifted(L, omega)
    S = ShiftedSolver(M)
    r = randomized_resolvent(L, omega, Omega, q=q, solver=S)
    norm_M = spectral_norm(M, iters=norm_iters)
    s = r.sigma_B
    kappa = norm_M * s[0]
    res = S.solve_adjoint(r.U_AV[:, 0]) - r.sigma_AV[0] * r.V[:, 0]
    out = {
        "omega": complex(omega), "norm_M": norm_M, "sigma": s, "kappa": kappa,
        "floor_pred": kappa * EPS64, "gap12": s[0] / s[1] if s.size > 1 else np.inf,
        "gapk": s[-1] / s[0],
        "triplet_res": float(np.linalg.norm(res) / r.sigma_AV[0]),
    }
    if unpivoted:
        Su = UnpivotedSolver(M)
        ru = randomized_resolvent(L, omega, Omega, q=q, solver=Su)
        out["growth"], out["minpiv"] = Su.growth, Su.minpiv
        out["contraction_pred"] = kappa * Su.growth * EPS32
        out["floor_measured"] = float(np.max(np.abs(ru.sigma_B - s)) / s[0])
    return out


def parity_tolerance(tol: float, report: dict) -> float:
    """The tolerance a parity test may use at this shift.  When
    the predicted floor exceeds tol / 10 it is max(tol, 10 x the measured
    floor between the pivoted and the unpivoted LU), otherwise tol."""
    if report["floor_pred"] <= tol / 10 or "floor_measured" not in report:
        return tol
    return max(tol, 10.0 * report["floor_measured"])


def _main(argv):
    import argparse
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import workloads as W
    from . import operator as op
    from . import sketch
    ap = argparse.ArgumentParser(description="conditioning report of one shift")
    ap.add_argument("workload")
    ap.add_argument("omega", type=float)
    ap.add_argument("--unpivoted", action="store_true",
                    help="also run the unpivoted LU (slow beyond n ~ 2e4)")
    a = ap.parse_args(argv)
    w = W.CONFIGS[a.workload]
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    Om = sketch.test_matrix(w.n, w.k, sketch.gradient_weight(U, hx, hy).ravel(), seed=w.seed)
    rep = conditioning_report(L, a.omega, Om, q=w.q, unpivoted=a.unpivoted)
    for key, val in rep.items():
        if key == "sigma":
            val = " ".join(f"{x:.6e}" for x in val)
        print(f"{key:18s} {val}")


if __name__ == "__main__":
    import sys
    _main(sys.argv[1:])
