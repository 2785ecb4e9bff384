"""Randomized resolvent analysis on the MI355X (gfx950).

The hot path of Ribeiro, Yeh & Taira, "Randomized resolvent analysis"
(arXiv:1902.01458), Algorithm 1: a physics-weighted Gaussian sketch, one band
LU of i*omega*I - L per frequency, forward and adjoint multi-RHS solves,
Cholesky-QR orthonormalisation, the reduced SVD and the recovery of gains and
modes through eq. (9); plus mixed-precision refinement, batched frequency
sweeps and the gradient of the leading gain.  All numerical work runs in the
HIP kernels of librr.so; this package only marshals arguments.
"""
from .api import (BurgersProblem, Factors, Graph, autotune, capture, factor,  # noqa: F401
                  factor_bytes, philox_raw, resolvent, sketch, sweep, use_torch_allocator)
from ._lib import RRError, lib  # noqa: F401
from .autograd import SigmaOne, sigma_one  # noqa: F401

__all__ = ["BurgersProblem", "Factors", "Graph", "factor", "resolvent", "sketch", "philox_raw",
           "capture", "autotune", "sweep", "factor_bytes", "use_torch_allocator", "RRError", "lib",
           "SigmaOne",
           "sigma_one"]
