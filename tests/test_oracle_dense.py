"""Pins for the subspace sine of the oracle (oracle.dense.sin_angle) and of
the GPU tests' helper (tests.gpu_util.sin_angle).

Every mode-parity claim rests on this function, so it is checked against
subspaces whose principal angles are known by construction: a line at angle
theta, a plane with two different angles (the 2-norm gives the larger sine,
a Frobenius norm would give the root sum of squares), bases that are not
orthonormal (scaled, mixed columns: the subspace decides, not the basis), a
common complex phase, and identical subspaces.
"""
import numpy as np
import pytest

from oracle import dense
from tests import gpu_util

FUNCS = [dense.sin_angle, gpu_util.sin_angle]


def rotated_pair(n, thetas, seed):
    """Orthonormal A and B = A cos(theta) + A_perp sin(theta), column-wise,
    embedded in C^n by a random unitary: principal angles exactly `thetas`."""
    m = len(thetas)
    rng = np.random.Generator(np.random.PCG64(seed))
    Z = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Qf, _ = np.linalg.qr(Z)
    A = Qf[:, :m]
    Ap = Qf[:, m:2 * m]
    c = np.cos(np.asarray(thetas))
    s = np.sin(np.asarray(thetas))
    return A, A * c[None, :] + Ap * s[None, :]


@pytest.mark.parametrize("f", FUNCS)
def test_line_at_known_angle(f):
    for th in (1e-9, 1e-4, 0.3, 1.2, np.pi / 2):
        e1 = np.zeros((5, 1), dtype=complex)
        e1[0] = 1
        b = np.zeros((5, 1), dtype=complex)
        b[0], b[1] = np.cos(th), np.sin(th)
        assert abs(f(e1, b) - np.sin(th)) <= 1e-15 + 1e-12 * np.sin(th)


@pytest.mark.parametrize("f", FUNCS)
def test_plane_takes_the_largest_angle_in_2_norm(f):
    t1, t2 = 0.5, 0.6
    A, B = rotated_pair(12, [t1, t2], 3)
    got = f(A, B)
    assert abs(got - np.sin(t2)) <= 1e-13
    # the Frobenius variant would give this instead: far from the 2-norm one
    assert abs(np.hypot(np.sin(t1), np.sin(t2)) - got) > 0.1


@pytest.mark.parametrize("f", FUNCS)
def test_basis_does_not_matter(f):
    t = [1e-6, 3e-3, 0.05]
    A, B = rotated_pair(20, t, 4)
    rng = np.random.Generator(np.random.PCG64(5))
    G1 = rng.standard_normal((3, 3)) + 1j * rng.standard_normal((3, 3))
    G2 = np.diag([1e3, 1.0, 1e-3]) @ (rng.standard_normal((3, 3)) + 0j)
    assert abs(f(A @ G1, B @ G2) - np.sin(t[-1])) <= 1e-10
    assert abs(f(A * np.exp(0.9j), B) - np.sin(t[-1])) <= 1e-13   # a common phase
    assert f(A @ G1, A) <= 1e-14                                   # same subspace


@pytest.mark.parametrize("f", FUNCS)
def test_small_angles_keep_their_digits(f):
    # arccos(|a^H b|) would lose everything below ~1e-8; the projection keeps it
    A, B = rotated_pair(30, [2e-11], 6)
    assert abs(f(A, B) - 2e-11) <= 1e-3 * 2e-11
