"""Seeded synthetic workloads shared by the oracle and the GPU path.

This module only produces *inputs*: grid sizes, domains, viscosities, the
base-flow field sampled on the nodes (ghost ring included), the lists of
frequencies and the sketch parameters.  It holds none of the method's
arithmetic (no operator, no sketch, no solve), so both the oracle and the HIP
library can take their inputs from here without sharing any computation.

The configurations are synthetic stand-ins for the paper's airfoil problem
(Section 3.1: a compressible linearised Navier-Stokes operator of size about
0.75 million about a LES mean flow, swept over Strouhal number).  That operator,
mesh and mean flow are not available, so a 2-D linearised viscous Burgers
operator about a shear-layer base flow is used instead (a stand-in with the
same kind of shear-driven non-normality the paper's Section 3.1 points at).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Tuple

import numpy as np


@dataclasses.dataclass(frozen=True)
class Workload:
    """One synthetic resolvent workload.

    nx, ny      interior nodes in x and y (unknowns are u, v at each node)
    domain      (x0, x1, y0, y1); nodes sit at x0 + i*hx, i = 0..nx+1, with
                hx = (x1 - x0)/(nx + 1); i = 0 and nx+1 form the Dirichlet ring
    nu          viscosity
    omegas      frequencies (real, rad per unit time)
    k           sketch width
    q           number of subspace (power) iterations
    base        name of the base flow ("shear" or "shear_noise")
    """
    name: str
    nx: int
    ny: int
    domain: Tuple[float, float, float, float]
    nu: float
    omegas: Tuple[float, ...]
    k: int
    q: int
    base: str = "shear"
    stretch: float = 1.0  # base flow U0(x/stretch, y/stretch)
    seed: int = 0

    @property
    def n(self) -> int:
        return 2 * self.nx * self.ny

    @property
    def b(self) -> int:
        return 2 * self.ny


def _logspace(lo: float, hi: float, count: int) -> Tuple[float, ...]:
    return tuple(float(lo * (hi / lo) ** (i / (count - 1))) for i in range(count))


def headline_omegas() -> Tuple[float, ...]:
    """16 shifts 2^((i-6)/3), i = 0..15: log-spaced over [0.25, 8], holding 2.0."""
    return tuple(float(2.0 ** ((i - 6) / 3.0)) for i in range(16))


CONFIGS = {
    # 64x32 grid on [0,8]x[-2,2], nu = 1e-2, single omega = 1, k = 10
    "cfg0": Workload("cfg0", 64, 32, (0.0, 8.0, -2.0, 2.0), 1e-2, (1.0,), 10, 0),
    # 512x256 grid on [0,16]x[-4,4], nu = 2e-3, base flow stretched by 2
    "cfg1": Workload("cfg1", 512, 256, (0.0, 16.0, -4.0, 4.0), 2e-3, (2.0,), 20, 1,
                     stretch=2.0),
    # the measured batch: the 512x256 operator swept over 16 shifts
    "cfg1_batch16": Workload("cfg1_batch16", 512, 256, (0.0, 16.0, -4.0, 4.0), 2e-3,
                             headline_omegas(), 20, 1, stretch=2.0),
    # 256x128 sweep of 64 log-spaced omegas in [0.1, 10], k = 10
    "cfg2": Workload("cfg2", 256, 128, (0.0, 8.0, -2.0, 2.0), 1e-2,
                     _logspace(0.1, 10.0, 64), 10, 0),
    # 256x128 gradient workload, nu = 5e-3
    "cfg3": Workload("cfg3", 256, 128, (0.0, 8.0, -2.0, 2.0), 5e-3,
                     (0.5, 1.0, 2.0, 4.0), 12, 0),
    # 1024x512, nu = 1e-3, noisy base flow, 16 omegas in [0.2, 8], k = 32, q = 1
    "cfg4": Workload("cfg4", 1024, 512, (0.0, 8.0, -2.0, 2.0), 1e-3,
                     _logspace(0.2, 8.0, 16), 32, 1, base="shear_noise"),
}


def node_coords(w: Workload) -> Tuple[np.ndarray, np.ndarray]:
    """Coordinates of all (nx+2) x (ny+2) nodes, ring included."""
    x0, x1, y0, y1 = w.domain
    hx = (x1 - x0) / (w.nx + 1)
    hy = (y1 - y0) / (w.ny + 1)
    x = x0 + hx * np.arange(w.nx + 2)
    y = y0 + hy * np.arange(w.ny + 2)
    return x, y


def shear_flow(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """U0(x, y) = tanh(y/0.5) + 0.1 exp(-y^2) sin(pi x / 4), on a tensor grid."""
    X, Y = np.meshgrid(x, y, indexing="ij")
    return np.tanh(Y / 0.5) + 0.1 * np.exp(-Y * Y) * np.sin(np.pi * X / 4.0)


def smooth_noise(shape: Tuple[int, int], seed: int = 2, width: float = 8.0,
                 amplitude: float = 0.05) -> np.ndarray:
    """Seeded Gaussian-filtered white noise, normalised to max |.| = amplitude.

    White N(0,1) noise (numpy PCG64, given seed) is smoothed with a separable
    Gaussian of standard deviation `width` nodes truncated at 4 widths.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    g = rng.standard_normal(shape)
    r = int(math.ceil(4 * width))
    t = np.arange(-r, r + 1)
    ker = np.exp(-0.5 * (t / width) ** 2)
    ker /= ker.sum()
    for ax in (0, 1):
        g = np.apply_along_axis(lambda v: np.convolve(v, ker, mode="same"), ax, g)
    return amplitude * g / np.abs(g).max()


def base_flow(w: Workload) -> np.ndarray:
    """Base-flow streamwise velocity U on all nodes, shape (nx+2, ny+2), y fastest."""
    x, y = node_coords(w)
    U = shear_flow(x / w.stretch, y / w.stretch)
    if w.base == "shear_noise":
        U = U + smooth_noise(U.shape)
    elif w.base != "shear":
        raise ValueError(f"unknown base flow {w.base!r}")
    return np.ascontiguousarray(U, dtype=np.float64)


def small(name: str, nx: int, ny: int, nu: float = 1e-2, omegas=(1.0,), k: int = 10,
          q: int = 0, domain=(0.0, 8.0, -2.0, 2.0)) -> Workload:
    """A reduced-size workload with config 0's domain and base flow."""
    return Workload(name, nx, ny, tuple(domain), nu, tuple(omegas), k, q)


def sub_grid(U: np.ndarray, i0: int, j0: int, m: int) -> np.ndarray:
    """An m x m block of interior nodes starting at interior index (i0, j0) (1-based),
    returned with its ring taken from the neighbouring nodes of the big grid."""
    return np.ascontiguousarray(U[i0 - 1:i0 + m + 1, j0 - 1:j0 + m + 1])
