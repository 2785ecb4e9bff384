"""Gradient of the leading gain with respect to the base flow, nu and omega.

Not part of the paper's algorithm: a first-order perturbation of eq. (5).  For
a simple singular value with H v = s u and u^H H = s v^H,
    ds = Re(u^H dH v),  dH = -H dM H   =>   ds = -s^2 Re(v^H dM u).
With M = i*omega*I - L:
  parameter p of L (dM = -dL/dp dp):  ds/dp = s^2 Re(v^H (dL/dp) u)
  omega (dM = i d omega I):           ds/d omega = s^2 Im(v^H u)
  nu (dL/dnu = Dirichlet Laplacian on both components):
                                      ds/d nu = s^2 Re(v^H Lap_h u)
L depends on the interior nodal values of U through the convection coefficient
at the node itself and through U_x, U_y at its four neighbours (central
differences), so ds/dU_p is a short stencil reduction over u and v.  A value
of U on the boundary ring enters L only through the central difference of its
one interior neighbour (U_x for the west and east rings, U_y for the south
and north ones; the corners through none), so its derivative is one term of
that neighbour's row (`gradient_full`).

Two implementations are kept on purpose: `gradient` / `gradient_full` write
that reduction out term by term; `gradient_bruteforce` differentiates the
coefficient array numerically exactly (it is affine in U) and forms
v^H (dL/dU_p) u with a sparse matrix per node, ring nodes included when asked.  They pin each other at small n; the dense SVD pins the
triplet.
"""
from __future__ import annotations

import numpy as np

from .operator import assemble, burgers_coefficients, laplacian


def gradient(sigma: float, u: np.ndarray, v: np.ndarray, nx: int, ny: int,
             hx: float, hy: float):
    """(dsigma/dU on the (nx, ny) interior nodes, dsigma/dnu, dsigma/domega)
    from the triplet (sigma, u = response, v = forcing); u, v length 2*nx*ny."""
    uu = u[0::2].reshape(nx, ny)   # u-component of the response
    uv = u[1::2].reshape(nx, ny)   # v-component of the response
    vu = np.conj(v[0::2].reshape(nx, ny))
    vv = np.conj(v[1::2].reshape(nx, ny))

    def shift(a, di, dj):
        """a at neighbour (i+di, j+dj), zero where that neighbour is on the ring."""
        out = np.zeros_like(a)
        nxa, nya = a.shape
        si = slice(max(di, 0), nxa + min(di, 0))
        so = slice(max(-di, 0), nxa + min(-di, 0))
        sj = slice(max(dj, 0), nya + min(dj, 0))
        sjo = slice(max(-dj, 0), nya + min(-dj, 0))
        out[so, sjo] = a[si, sj]
        return out

    E = lambda a: shift(a, 1, 0)
    W = lambda a: shift(a, -1, 0)
    N = lambda a: shift(a, 0, 1)
    S = lambda a: shift(a, 0, -1)
    g = (vu * (-(E(uu) - W(uu)) / (2 * hx))          # -U_p du/dx in the u-row at p
         + vv * (-(E(uv) - W(uv)) / (2 * hx))        # -U_p dv/dx in the v-row at p
         - W(vu * uu) / (2 * hx)                     # -U_x u at W: U_x(W) has +U_p/2hx
         + E(vu * uu) / (2 * hx)                     # -U_x u at E: U_x(E) has -U_p/2hx
         - S(vu * uv) / (2 * hy)                     # -U_y v at S: U_y(S) has +U_p/2hy
         + N(vu * uv) / (2 * hy))                    # -U_y v at N: U_y(N) has -U_p/2hy
    dU = sigma ** 2 * np.real(g)
    Lap = laplacian(nx, ny, hx, hy)
    dnu = sigma ** 2 * np.real(np.vdot(v, Lap @ u))
    domega = sigma ** 2 * np.imag(np.vdot(v, u))
    return dU, float(dnu), float(domega)


def gradient_full(sigma: float, u: np.ndarray, v: np.ndarray, nx: int, ny: int,
                  hx: float, hy: float):
    """dsigma/dU on every node of the (nx+2, ny+2) base-flow array, ring
    included, plus dsigma/dnu and dsigma/domega as in `gradient`.

    Ring terms (1-based interior neighbour in brackets):
      west  (0, j):     U_x(1, j) = (U(2, j) - U(0, j)) / 2hx, and the u-row
                        centre coefficient carries -U_x, so
                        dsigma = +s^2 Re(conj(v_u) u_u) / 2hx at (1, j)
      east  (nx+1, j):  -s^2 Re(conj(v_u) u_u) / 2hx at (nx, j)
      south (i, 0):     U_y(i, 1) = (U(i, 2) - U(i, 0)) / 2hy, and the u-row
                        coupling coefficient is -U_y, so
                        dsigma = +s^2 Re(conj(v_u) u_v) / 2hy at (i, 1)
      north (i, ny+1):  -s^2 Re(conj(v_u) u_v) / 2hy at (i, ny)
      corners:          no central difference reads them: 0.
    """
    g, dnu, domega = gradient(sigma, u, v, nx, ny, hx, hy)
    uu = u[0::2].reshape(nx, ny)
    uv = u[1::2].reshape(nx, ny)
    vu = np.conj(v[0::2].reshape(nx, ny))
    s2 = sigma ** 2
    full = np.zeros((nx + 2, ny + 2))
    full[1:-1, 1:-1] = g
    full[0, 1:-1] = s2 * np.real(vu[0, :] * uu[0, :]) / (2 * hx)
    full[-1, 1:-1] = -s2 * np.real(vu[-1, :] * uu[-1, :]) / (2 * hx)
    full[1:-1, 0] = s2 * np.real(vu[:, 0] * uv[:, 0]) / (2 * hy)
    full[1:-1, -1] = -s2 * np.real(vu[:, -1] * uv[:, -1]) / (2 * hy)
    return full, dnu, domega


def gradient_bruteforce(sigma: float, u: np.ndarray, v: np.ndarray, U: np.ndarray,
                        nx: int, ny: int, hx: float, hy: float, nu: float,
                        ring: bool = False):
    """Same quantity by differentiating the coefficient array node by node:
    on the (nx, ny) interior nodes, or with ring=True on all (nx+2, ny+2)."""
    c0 = burgers_coefficients(U, nx, ny, hx, hy, nu)
    o = 0 if ring else 1
    dU = np.zeros((nx + 2 - 2 * o, ny + 2 - 2 * o))
    for i in range(dU.shape[0]):
        for j in range(dU.shape[1]):
            U1 = U.copy()
            U1[i + o, j + o] += 1.0
            dc = burgers_coefficients(U1, nx, ny, hx, hy, nu) - c0  # exact: affine in U
            dL = assemble(dc)
            dU[i, j] = sigma ** 2 * np.real(np.vdot(v, dL @ u))
    return dU
