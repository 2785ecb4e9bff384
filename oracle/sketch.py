"""Physics-informed complex Gaussian test matrix (Algorithm 1 step 1, eq. 10).

Algorithm 1 draws a random normal test matrix; Section 3.4 scales its rows by
Phi, the 2-norm of the base-flow velocity gradient at each grid point, stacked
over the variables (eq. 10: Omega_p = diag(Phi) Omega).  With the base flow
(U, V = 0) the gradient tensor has a single non-zero row, so its 2-norm is
sqrt(U_x^2 + U_y^2); an offset of 0.1 keeps weak-gradient rows in the sketch.

Entry (r, j) of the unweighted matrix is a standard complex normal number
(E|w|^2 = 1) made by the Box-Muller transform from one Philox4x32-10 call at
counter (r, j, stream, 0) under key (seed low word, seed high word):
    u1 = (m1 + 1) 2^-53 in (0, 1],  u2 = m2 2^-53 in [0, 1)
    w  = sqrt(-ln u1) * exp(2 pi i u2)
where m1, m2 are the top 53 bits of the 64-bit words (x0:x1) and (x2:x3).
Column j does not depend on k, so sketches of growing width are nested.

Other test matrices named in Section 2.2.2 (our readings; the paper gives no
formulas):
  * Rademacher: real +-1 entries, the sign being the top bit of x0 at the
    same counter (r, j, stream, 0); nested in k like the Gaussian one.
  * ultrasparse Rademacher (sparse sign): each row has zeta nonzeros, +-1 as
    above, in the zeta columns whose selection keys (word x0 at counter
    (r, j, stream + 1, 0)) are smallest, ties to the lower column; other
    entries 0.  zeta = 0 means min(k, 8).
  * orthonormal: the Gaussian matrix with orthonormal columns (QR with a
    positive real diagonal of R), before the eq. 10 weighting.
The weighting diag(Phi) of eq. 10 applies to each of them alike.

Pins: known-answer Philox vectors; moments of w; Phi = 1.1 for U = y; the
structure of each kind (values, nonzeros per row, orthonormality, nesting).
"""
from __future__ import annotations

import numpy as np

from .philox import philox4x32_10

TWO_M53 = 2.0 ** -53


def uniforms(rows, cols, stream: int, seed: int):
    """The two 53-bit uniforms (u1 in (0,1], u2 in [0,1)) for each (row, col)."""
    x0, x1, x2, x3 = philox4x32_10(rows, cols, stream, 0, seed & 0xFFFFFFFF, seed >> 32)
    m1 = ((x0.astype(np.uint64) << np.uint64(32)) | x1.astype(np.uint64)) >> np.uint64(11)
    m2 = ((x2.astype(np.uint64) << np.uint64(32)) | x3.astype(np.uint64)) >> np.uint64(11)
    u1 = (m1.astype(np.float64) + 1.0) * TWO_M53
    u2 = m2.astype(np.float64) * TWO_M53
    return u1, u2


def complex_normal(n: int, k: int, seed: int = 0, stream: int = 0) -> np.ndarray:
    """n x k standard complex normal matrix (E|w|^2 = 1) by Box-Muller."""
    r = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(k, dtype=np.uint64)[None, :]
    u1, u2 = uniforms(r, c, stream, seed)
    return np.sqrt(-np.log(u1)) * np.exp(2j * np.pi * u2)


KINDS = ("gaussian", "rademacher", "sparse", "orthonormal")


def rademacher(n: int, k: int, seed: int = 0, stream: int = 0) -> np.ndarray:
    """n x k matrix of +-1 (sign: top bit of x0 at counter (r, j, stream, 0))."""
    r = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(k, dtype=np.uint64)[None, :]
    x0, _, _, _ = philox4x32_10(r, c, stream, 0, seed & 0xFFFFFFFF, seed >> 32)
    return np.where((x0 >> np.uint32(31)) != 0, -1.0, 1.0)


def sparse_sign(n: int, k: int, zeta: int = 0, seed: int = 0, stream: int = 0) -> np.ndarray:
    """n x k ultrasparse Rademacher matrix: zeta entries +-1 per row, in the
    columns with the smallest selection keys (ties to the lower column)."""
    z = min(k, 8) if zeta <= 0 else min(zeta, k)
    r = np.arange(n, dtype=np.uint64)[:, None]
    c = np.arange(k, dtype=np.uint64)[None, :]
    keys, _, _, _ = philox4x32_10(r, c, stream + 1, 0, seed & 0xFFFFFFFF, seed >> 32)
    keys = np.broadcast_to(keys, (n, k))
    order = np.argsort(keys, axis=1, kind="stable")  # equal keys keep column order
    mask = np.zeros((n, k), dtype=bool)
    np.put_along_axis(mask, order[:, :z], True, axis=1)
    return np.where(mask, rademacher(n, k, seed, stream), 0.0)


def gradient_weight(U: np.ndarray, hx: float, hy: float) -> np.ndarray:
    """Phi per interior node: |grad U| + 0.1 with central differences (nx, ny)."""
    Ux = (U[2:, 1:-1] - U[:-2, 1:-1]) / (2.0 * hx)
    Uy = (U[1:-1, 2:] - U[1:-1, :-2]) / (2.0 * hy)
    return np.sqrt(Ux * Ux + Uy * Uy) + 0.1


def test_matrix(n: int, k: int, phi_nodes, seed: int = 0, kind: str = "gaussian",
                zeta: int = 0) -> np.ndarray:
    """Omega_p = diag(Phi stacked over (u, v)) Omega (eq. 10).

    phi_nodes: Phi per node in node order p (length n/2), or None for the plain
    matrix of Algorithm 1 step 1; kind: one of KINDS.
    """
    if kind == "gaussian":
        W = complex_normal(n, k, seed=seed, stream=0)
    elif kind == "rademacher":
        W = rademacher(n, k, seed=seed, stream=0).astype(np.complex128)
    elif kind == "sparse":
        W = sparse_sign(n, k, zeta, seed=seed, stream=0).astype(np.complex128)
    elif kind == "orthonormal":
        Qm, R = np.linalg.qr(complex_normal(n, k, seed=seed, stream=0), mode="reduced")
        d = np.diag(R)
        W = Qm * (d / np.abs(d))[None, :]
    else:
        raise ValueError(f"unknown test matrix kind {kind!r}")
    if phi_nodes is None:
        return W
    w = np.repeat(np.asarray(phi_nodes, dtype=np.float64).reshape(-1), 2)
    return w[:, None] * W
