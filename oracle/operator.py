"""2-D linearised viscous Burgers operator L (the stand-in for eq. (1)'s L).

Eq. (1) needs a real linear operator L about a base state; eq. (4) builds the
resolvent from it.  Here L is the linearisation of
    u_t + u u_x + v u_y = nu Lap(u),   v_t + u v_x + v v_y = nu Lap(v)
about the base flow (U(x, y), V = 0):
    u'_t = nu Lap(u') - U u'_x - U_x u' - U_y v'
    v'_t = nu Lap(v') - U v'_x
discretised with second-order central differences on the interior nodes of a
uniform grid, homogeneous Dirichlet perturbations on the ring around them.

Ordering: node p = j + ny*i (0-based interior indices, y fastest); u_p is
unknown 2p and v_p is unknown 2p+1.  The half-bandwidth is then 2*ny.

Coefficient layout (12 per node, the format the library consumes too):
  u-row: C, E, W, N, S, Cpl (Cpl multiplies v_p)
  v-row: C, E, W, N, S, Cpl (Cpl multiplies u_p)
Neighbours on the ring contribute nothing.

Pins: exactness on quadratics (nu = 1, U = 0), pure convection of x
(nu = 0, U = 1), rows of a 3x3 grid worked by hand, half-bandwidth, and the
adjoint dot test (tests/test_oracle_operator.py).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

NCOEF = 12


def spacing(nx: int, ny: int, domain):
    x0, x1, y0, y1 = domain
    return (x1 - x0) / (nx + 1), (y1 - y0) / (ny + 1)


def burgers_coefficients(U: np.ndarray, nx: int, ny: int, hx: float, hy: float,
                         nu: float) -> np.ndarray:
    """Stencil coefficients, shape (nx, ny, 12), from U on (nx+2, ny+2) nodes."""
    assert U.shape == (nx + 2, ny + 2)
    Ui = U[1:-1, 1:-1]
    Ux = (U[2:, 1:-1] - U[:-2, 1:-1]) / (2.0 * hx)
    Uy = (U[1:-1, 2:] - U[1:-1, :-2]) / (2.0 * hy)
    ax = nu / (hx * hx)
    ay = nu / (hy * hy)
    c = np.empty((nx, ny, NCOEF))
    # u-row
    c[..., 0] = -2.0 * (ax + ay) - Ux
    c[..., 1] = ax - Ui / (2.0 * hx)
    c[..., 2] = ax + Ui / (2.0 * hx)
    c[..., 3] = ay
    c[..., 4] = ay
    c[..., 5] = -Uy
    # v-row
    c[..., 6] = -2.0 * (ax + ay)
    c[..., 7] = ax - Ui / (2.0 * hx)
    c[..., 8] = ax + Ui / (2.0 * hx)
    c[..., 9] = ay
    c[..., 10] = ay
    c[..., 11] = 0.0
    return c


def assemble(coef: np.ndarray) -> sp.csr_matrix:
    """Real sparse L (n x n) from the (nx, ny, 12) coefficient array."""
    nx, ny, _ = coef.shape
    n = 2 * nx * ny
    I, J = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    p = (J + ny * I).ravel()
    rows, cols, vals = [], [], []

    def add(row_off, mask, nbr_p, col_off, values):
        m = mask.ravel()
        rows.append(2 * p[m] + row_off)
        cols.append(2 * nbr_p.ravel()[m] + col_off)
        vals.append(values.ravel()[m])

    every = np.ones((nx, ny), dtype=bool)
    pE = (J + ny * (I + 1))
    pW = (J + ny * (I - 1))
    pN = (J + 1 + ny * I)
    pS = (J - 1 + ny * I)
    hasE, hasW = I < nx - 1, I > 0
    hasN, hasS = J < ny - 1, J > 0
    pp = p.reshape(nx, ny)
    for comp in (0, 1):
        o = 6 * comp
        add(comp, every, pp, comp, coef[..., o + 0])
        add(comp, hasE, pE, comp, coef[..., o + 1])
        add(comp, hasW, pW, comp, coef[..., o + 2])
        add(comp, hasN, pN, comp, coef[..., o + 3])
        add(comp, hasS, pS, comp, coef[..., o + 4])
        add(comp, every, pp, 1 - comp, coef[..., o + 5])
    L = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    L.sum_duplicates()
    return L


def shifted(L: sp.spmatrix, omega: complex) -> sp.csr_matrix:
    """M(omega) = i*omega*I - L, whose inverse is the resolvent H(omega).

    Eq. (4) writes the resolvent as [-i omega I - L]^(-1) for the e^(-i omega t)
    convention; with e^(+i omega t) it is [i omega I - L]^(-1).  For real L and
    real omega the two are complex conjugates of each other: same gains, modes
    conjugated.  This oracle and the library both use the + sign.  The
    discounted resolvent of Section 2.1 (complex frequency omega_r + i beta
    there, the growth rates of L lowered by beta) is i omega_r I - (L - beta I)
    here, i.e. omega = omega_r - i beta.
    """
    n = L.shape[0]
    return (sp.identity(n, dtype=np.complex128, format="csr") * (1j * omega)
            - L.astype(np.complex128)).tocsr()


def half_bandwidth(A: sp.spmatrix) -> int:
    C = A.tocoo()
    if C.nnz == 0:
        return 0
    return int(np.max(np.abs(C.row.astype(np.int64) - C.col.astype(np.int64))))


def lapack_band(A: sp.spmatrix, kl: int, ku: int) -> np.ndarray:
    """LAPACK general-band storage for ?gbtrf: (2kl+ku+1, n), AB[kl+ku+i-j, j] = A[i, j]."""
    C = A.tocoo()
    n = A.shape[0]
    AB = np.zeros((2 * kl + ku + 1, n), dtype=np.complex128, order="F")
    AB[kl + ku + C.row - C.col, C.col] = C.data
    return AB


def laplacian(nx: int, ny: int, hx: float, hy: float) -> sp.csr_matrix:
    """Dirichlet 5-point Laplacian acting on both components (d L / d nu)."""
    c = np.zeros((nx, ny, NCOEF))
    for o in (0, 6):
        c[..., o + 0] = -2.0 / hx ** 2 - 2.0 / hy ** 2
        c[..., o + 1] = c[..., o + 2] = 1.0 / hx ** 2
        c[..., o + 3] = c[..., o + 4] = 1.0 / hy ** 2
    return assemble(c)
