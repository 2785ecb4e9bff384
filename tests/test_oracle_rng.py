"""Pins for the oracle's counter-based generator and test matrix.

Philox4x32-10 is checked against the published known-answer vectors; the
Box-Muller complex normals against their moments; the weighting of eq. (10)
against a base flow with a known gradient.
"""
import os

import numpy as np

from oracle import operator as op
from oracle import sketch
from oracle.philox import philox4x32_10

GOLD = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_known_answers():
    n = 0
    for line in open(GOLD):
        if line.startswith("#") or not line.strip():
            continue
        w = [int(x, 16) for x in line.split()]
        out = philox4x32_10(w[0], w[1], w[2], w[3], w[4], w[5])
        assert [int(o) for o in out] == w[6:]
        n += 1
    assert n == 3


def test_philox_vectorised_matches_scalar():
    r = np.arange(7, dtype=np.uint64)
    a = philox4x32_10(r, 3, 0, 0, 5, 0)
    for i in range(7):
        s = philox4x32_10(i, 3, 0, 0, 5, 0)
        assert all(int(a[t][i]) == int(s[t]) for t in range(4))


def test_complex_normal_moments():
    N = 200_000
    w = sketch.complex_normal(N, 1, seed=0).ravel()
    tol = 5.0 / np.sqrt(N)
    assert abs(w.mean()) < tol
    assert abs(np.mean(np.abs(w) ** 2) - 1.0) < 5 * tol
    assert abs(np.mean(w * w)) < 5 * tol          # circular: E[w^2] = 0
    assert abs(np.mean(w.real ** 2) - 0.5) < 5 * tol


def test_uniform_ranges():
    u1, u2 = sketch.uniforms(np.arange(100_000, dtype=np.uint64), 0, 0, 0)
    assert u1.min() > 0.0 and u1.max() <= 1.0
    assert u2.min() >= 0.0 and u2.max() < 1.0


def test_sketch_columns_nested_and_seeded():
    a = sketch.complex_normal(50, 6, seed=3)
    b = sketch.complex_normal(50, 4, seed=3)
    np.testing.assert_array_equal(a[:, :4], b)
    c = sketch.complex_normal(50, 4, seed=4)
    assert np.abs(b - c).min() > 0


def test_gradient_weight_linear_flow():
    # U = y has |grad U| = 1 exactly under central differences: Phi = 1.1
    nx, ny = 5, 4
    hx, hy = op.spacing(nx, ny, (0.0, 3.0, -1.0, 1.0))
    y = -1.0 + hy * np.arange(ny + 2)
    U = np.tile(y, (nx + 2, 1))
    phi = sketch.gradient_weight(U, hx, hy)
    np.testing.assert_allclose(phi, 1.1, rtol=1e-14)
    Om = sketch.test_matrix(2 * nx * ny, 3, phi.ravel(), seed=0)
    np.testing.assert_allclose(Om, 1.1 * sketch.complex_normal(2 * nx * ny, 3), rtol=1e-15)


def test_rademacher_signs_balanced_and_nested():
    W = sketch.rademacher(20000, 8, seed=5)
    assert set(np.unique(W)) == {-1.0, 1.0}
    assert abs(W.mean()) < 0.02
    # the sign is the top bit of word x0 of the Gaussian's counter: columns nest
    np.testing.assert_array_equal(sketch.rademacher(20000, 3, seed=5), W[:, :3])
    # and the signs of neighbouring columns are uncorrelated
    assert abs(np.mean(W[:, 0] * W[:, 1])) < 0.03


def test_sparse_sign_structure():
    n, k = 4000, 10
    for zeta, z in ((3, 3), (0, 8), (25, 10)):
        S = sketch.sparse_sign(n, k, zeta, seed=2)
        nz = S != 0
        assert np.all(nz.sum(axis=1) == z)
        # nonzeros carry the Rademacher signs of the same entries
        R = sketch.rademacher(n, k, seed=2)
        np.testing.assert_array_equal(S[nz], R[nz])
    # every column is chosen about equally often (zeta / k of the rows)
    S = sketch.sparse_sign(n, k, 3, seed=2)
    frac = (S != 0).mean(axis=0)
    assert np.all(np.abs(frac - 0.3) < 0.04)


def test_orthonormal_test_matrix():
    n, k = 500, 7
    W = sketch.test_matrix(n, k, None, seed=4, kind="orthonormal")
    np.testing.assert_allclose(W.conj().T @ W, np.eye(k), atol=1e-13)
    G = sketch.complex_normal(n, k, seed=4)
    # same column space as the Gaussian matrix, and W^H G upper triangular
    # with a positive real diagonal (the R of G = W R)
    R = W.conj().T @ G
    np.testing.assert_allclose(np.tril(R, -1), 0, atol=1e-12)
    assert np.all(np.abs(np.diag(R).imag) < 1e-12) and np.all(np.diag(R).real > 0)
    # eq. 10's weights apply after the orthonormalisation
    phi = np.linspace(0.5, 2.0, n // 2)
    Wp = sketch.test_matrix(n, k, phi, seed=4, kind="orthonormal")
    np.testing.assert_allclose(Wp, np.repeat(phi, 2)[:, None] * W, rtol=1e-15)
