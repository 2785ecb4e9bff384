"""Pins for the unpivoted band-LU probe and the spectral-norm estimate."""
import numpy as np
import scipy.sparse as sp

import workloads as W
from oracle import operator as op, probe


def test_unpivoted_lu_reproduces_matrix():
    w = W.small("p", 6, 4, nu=2e-2)
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    M = op.shifted(op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu)), 0.7)
    growth, minpiv, A = probe.unpivoted_band_lu(M)
    n, b = M.shape[0], 2 * w.ny
    Lf = np.eye(n, dtype=complex)
    Uf = np.zeros((n, n), dtype=complex)
    for i in range(n):
        for d in range(-b, b + 1):
            j = i + d
            if 0 <= j < n:
                (Lf if d < 0 else Uf)[i, j] = A[i, d + b]
    np.testing.assert_allclose(Lf @ Uf, M.toarray(), atol=1e-12 * abs(M).max())
    assert 1.0 <= growth < 1e3 and minpiv > 0


def test_spectral_norm_matches_dense():
    rng = np.random.Generator(np.random.PCG64(9))
    A = sp.random(60, 60, density=0.2, random_state=1) + 1j * sp.random(60, 60, density=0.2,
                                                                       random_state=2)
    est = probe.spectral_norm(sp.csr_matrix(A), iters=2000)
    assert abs(est - np.linalg.norm(A.toarray(), 2)) <= 1e-6 * est
