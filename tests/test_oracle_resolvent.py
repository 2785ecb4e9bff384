"""Pins for the oracle's Algorithm 1.

Closed forms (normal operators fed through the same 12-coefficient format),
brute force (dense SVD of the resolvent, eq. 5), the inequalities that hold
for any range basis, nesting in k, exactness at k = n, and the Halko bound
quoted in Section 2.2.
"""
import numpy as np
import pytest

import workloads as W
from oracle import dense, operator as op, resolvent, sketch


def coef_zero(nx, ny):
    return np.zeros((nx, ny, op.NCOEF))


def test_orth_matches_cholesky_qr():
    rng = np.random.Generator(np.random.PCG64(2))
    Y = rng.standard_normal((200, 7)) + 1j * rng.standard_normal((200, 7))
    Q = resolvent.orth(Y)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(7), atol=1e-14)
    # Cholesky QR (a textbook route to the same Q when diag(R) > 0)
    G = Y.conj().T @ Y
    R = np.linalg.cholesky(G).conj().T
    Qc = Y @ np.linalg.inv(R)
    np.testing.assert_allclose(Q, Qc, atol=1e-12)


def test_diagonal_operator_closed_form():
    # normal L = diag(lambda): gains 1/|i omega - lambda|.  Four eigenvalues
    # near zero give large gains; the rest are far away (gap > 1e4).
    nx, ny = 8, 4
    n = 2 * nx * ny
    c = coef_zero(nx, ny)
    lam = -1e5 * (1.0 + np.arange(n) / n)
    lam[[3, 10, 17, 40]] = [-0.1, -0.25, -0.7, -1.5]
    c[..., 0] = lam[0::2].reshape(nx, ny)
    c[..., 6] = lam[1::2].reshape(nx, ny)
    L = op.assemble(c)
    omega = 0.8
    exact = np.sort(1.0 / np.abs(1j * omega - lam))[::-1]
    Om = sketch.test_matrix(n, 6, None, seed=0)
    r = resolvent.randomized_resolvent(L, omega, Om, q=1)
    np.testing.assert_allclose(r.sigma_B[:4], exact[:4], rtol=1e-12)
    np.testing.assert_allclose(r.sigma_AV[:4], exact[:4], rtol=1e-12)
    # forcing modes of a diagonal operator are unit vectors
    for j, idx in enumerate(np.argsort(np.abs(1j * omega - lam))[:4]):
        e = np.zeros(n)
        e[idx] = 1
        assert dense.sin_angle(r.V[:, j:j + 1], e[:, None]) < 1e-10


def test_discounted_unstable_diagonal_closed_form():
    # Section 2.1: growing modes (Re lambda > 0) discounted by beta above the
    # largest growth rate; here the shift omega - i beta, so M = (i omega +
    # beta) I - L and the gains are 1 / |i omega + beta - lambda|
    nx, ny = 8, 8
    n = 2 * nx * ny
    c = coef_zero(nx, ny)
    lam = -1e5 * (1.0 + np.arange(n) / n)
    lam[[3, 10, 17, 40]] = [0.3, 0.05, -0.2, -0.9]
    c[..., 0] = lam[0::2].reshape(nx, ny)
    c[..., 6] = lam[1::2].reshape(nx, ny)
    L = op.assemble(c)
    omega, beta = 0.8, 0.5
    exact = np.sort(1.0 / np.abs(1j * omega + beta - lam))[::-1]
    r = resolvent.randomized_resolvent(L, omega - 1j * beta, sketch.test_matrix(n, 6, None, 0),
                                       q=1)
    np.testing.assert_allclose(r.sigma_B[:4], exact[:4], rtol=1e-12)
    np.testing.assert_allclose(r.sigma_AV[:4], exact[:4], rtol=1e-12)
    # the growing mode lambda = 0.3 is the most amplified one after discounting
    e = np.zeros(n)
    e[3] = 1
    assert dense.sin_angle(r.V[:, :1], e[:, None]) < 1e-10


def test_rotation_blocks_closed_form():
    # per node [[a, -c], [c, a]] through the coupling coefficients: normal,
    # eigenvalues a +- i c, gains 1/sqrt(a^2 + (omega -+ c)^2)
    nx, ny = 6, 5
    rng = np.random.Generator(np.random.PCG64(3))
    a = -rng.uniform(50.0, 100.0, (nx, ny))
    cc = rng.uniform(-3.0, 3.0, (nx, ny))
    a[2, 3], cc[2, 3] = -0.05, 1.0     # one node with a near-resonant pair
    C = coef_zero(nx, ny)
    C[..., 0] = a
    C[..., 5] = -cc
    C[..., 6] = a
    C[..., 11] = cc
    L = op.assemble(C)
    omega = 1.02
    gains = np.concatenate([1 / np.sqrt(a.ravel() ** 2 + (omega - cc.ravel()) ** 2),
                            1 / np.sqrt(a.ravel() ** 2 + (omega + cc.ravel()) ** 2)])
    exact = np.sort(gains)[::-1]
    n = 2 * nx * ny
    r = resolvent.randomized_resolvent(L, omega, sketch.test_matrix(n, 4, None), q=1)
    np.testing.assert_allclose(r.sigma_B[0], exact[0], rtol=1e-12)
    np.testing.assert_allclose(r.sigma_AV[0], exact[0], rtol=1e-12)
    # and with k = n the whole spectrum is exact
    r = resolvent.randomized_resolvent(L, omega, sketch.test_matrix(n, n, None), q=0)
    np.testing.assert_allclose(r.sigma_B, exact, rtol=1e-12)


def test_shifted_laplacian_closed_form():
    # L = nu Lap_h + alpha I on the real band shape: eigenvalues
    # alpha - 4 nu sin^2(k pi / 2(nx+1)) / hx^2 - 4 nu sin^2(l pi / 2(ny+1)) / hy^2,
    # each twice (u and v); alpha puts the lowest mode close to zero
    nx, ny, nu = 12, 8, 0.05
    hx, hy = op.spacing(nx, ny, (0, 8, -2, 2))
    kx = np.arange(1, nx + 1)
    ky = np.arange(1, ny + 1)
    lam_d = (-4 * nu * np.sin(kx * np.pi / (2 * (nx + 1))) ** 2 / hx ** 2)[:, None] + \
            (-4 * nu * np.sin(ky * np.pi / (2 * (ny + 1))) ** 2 / hy ** 2)[None, :]
    alpha = -lam_d.max() - 1e-4
    lam = np.concatenate([lam_d.ravel(), lam_d.ravel()]) + alpha
    C = coef_zero(nx, ny)
    for o in (0, 6):
        C[..., o + 0] = -2 * nu / hx ** 2 - 2 * nu / hy ** 2 + alpha
        C[..., o + 1] = C[..., o + 2] = nu / hx ** 2
        C[..., o + 3] = C[..., o + 4] = nu / hy ** 2
    L = op.assemble(C)
    assert op.half_bandwidth(L) == 2 * ny
    omega = 0.0
    exact = np.sort(1 / np.abs(1j * omega - lam))[::-1]
    n = 2 * nx * ny
    r = resolvent.randomized_resolvent(L, omega, sketch.test_matrix(n, n, None), q=0)
    np.testing.assert_allclose(r.sigma_B, exact, rtol=1e-11)
    r = resolvent.randomized_resolvent(L, omega, sketch.test_matrix(n, 6, None), q=1)
    # the top pair (u and v copies of the lowest mode) has a gain ratio of ~2e2
    np.testing.assert_allclose(r.sigma_B[:2], exact[:2], rtol=1e-9)


@pytest.fixture(scope="module")
def small_burgers():
    w = W.small("s", 16, 8, nu=1e-2, omegas=(1.0,), k=10)
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    phi = sketch.gradient_weight(U, hx, hy).ravel()
    Ud, sd, Vd = dense.resolvent_svd(L, 1.0)
    return w, L, phi, Ud, sd, Vd


def test_bruteforce_inequalities(small_burgers):
    w, L, phi, Ud, sd, Vd = small_burgers
    k = 10
    for q in (0, 1):
        r = resolvent.randomized_resolvent(L, 1.0, sketch.test_matrix(w.n, k, phi), q=q)
        slack = 1e-13 * sd[0]
        assert np.all(r.sigma_B <= sd[:k] + slack)           # sigma_j(Q^H H) <= sigma_j(H)
        assert np.all(r.sigma_B <= r.sigma_AV + slack)       # sigma_j(B) <= ||H v_j||
        assert np.all(r.sigma_AV <= sd[0] + slack)
        # the paper's recovery is never worse for sigma_1 (Section 2.2)
        assert abs(r.sigma_AV[0] - sd[0]) <= abs(r.sigma_B[0] - sd[0]) + slack
        # steps 2-9 reproduce H v_j = sigma_j u_j (eq. 9)
        M = op.shifted(L, 1.0)
        np.testing.assert_allclose(M @ (r.U_AV * r.sigma_AV[None, :]), r.V, atol=1e-12)


def test_bruteforce_exact_at_full_width(small_burgers):
    w, L, phi, Ud, sd, Vd = small_burgers
    r = resolvent.randomized_resolvent(L, 1.0, sketch.test_matrix(w.n, w.n, phi), q=0,
                                       optional_svd=True)
    np.testing.assert_allclose(r.sigma_B, sd, rtol=1e-10)
    np.testing.assert_allclose(r.sigma_AV[:4], sd[:4], rtol=1e-10)
    gap = sd[:-1] / sd[1:]
    for j in range(4):
        if gap[j] > 1.001 and (j == 0 or gap[j - 1] > 1.001):
            assert dense.sin_angle(r.V[:, j:j + 1], Vd[:, j:j + 1]) < 1e-8
            assert dense.sin_angle(r.U_AV[:, j:j + 1], Ud[:, j:j + 1]) < 1e-8


def test_halko_bound_and_error_shrinks(small_burgers):
    w, L, phi, Ud, sd, Vd = small_burgers
    M = op.shifted(L, 1.0).toarray()
    H = np.linalg.inv(M)
    errs = []
    for k in (4, 8, 16):
        r = resolvent.randomized_resolvent(L, 1.0, sketch.test_matrix(w.n, k, phi), q=0)
        E = H - r.Q @ (r.Q.conj().T @ H)
        assert np.linalg.norm(E, 2) <= (1 + 9 * np.sqrt(k) * np.sqrt(w.n)) * sd[k]
        errs.append(abs(r.sigma_AV[0] - sd[0]) / sd[0])
    assert errs[2] <= errs[0]


def test_nested_sketches(small_burgers):
    w, L, phi, Ud, sd, Vd = small_burgers
    prev = None
    for k in (3, 5, 8):
        r = resolvent.randomized_resolvent(L, 1.0, sketch.test_matrix(w.n, k, phi), q=0)
        if prev is not None:
            assert np.all(prev[:len(prev)] <= r.sigma_B[:len(prev)] + 1e-13 * sd[0])
        prev = r.sigma_B


def test_optional_steps_10_11(small_burgers):
    w, L, phi, Ud, sd, Vd = small_burgers
    r = resolvent.randomized_resolvent(L, 1.0, sketch.test_matrix(w.n, 8, phi), q=1,
                                       optional_svd=True)
    np.testing.assert_allclose(r.U_svd.conj().T @ r.U_svd, np.eye(8), atol=1e-12)
    np.testing.assert_allclose(r.V_svd.conj().T @ r.V_svd, np.eye(8), atol=1e-12)
    # H V_svd = U_svd diag(sigma_svd) exactly (step 10 is an SVD of H V)
    M = op.shifted(L, 1.0)
    np.testing.assert_allclose(M @ (r.U_svd * r.sigma_svd[None, :]), r.V_svd, atol=1e-11)


def test_recovery_accuracy_ordering():
    """Section 3.2 on the Burgers operator at n = 1024 (nu = 1e-3, k = 10,
    q = 1), against the dense SVD: sigma_B <= sigma_AV <= sigma_svd <=
    sigma_1 (norms of H over nested subspaces), and on the leading cluster
    the response modes of eq. 9 beat Halko's Q Ut, the optional re-SVD beats
    both, and its forcing modes beat those of step 5."""
    w = W.small("a", 32, 16, nu=1e-3, k=10, q=1)
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    L = op.assemble(op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu))
    phi = sketch.gradient_weight(U, hx, hy).ravel()
    Om = sketch.test_matrix(w.n, w.k, phi, w.seed)
    for om in (0.3, 1.0):
        Ud, sd, Vd = dense.resolvent_svd(L, om)
        r = resolvent.randomized_resolvent(L, om, Om, q=1, optional_svd=True)
        assert r.sigma_B[0] <= r.sigma_AV[0] * (1 + 1e-12)
        assert r.sigma_AV[0] <= r.sigma_svd[0] * (1 + 1e-12)
        assert r.sigma_svd[0] <= sd[0] * (1 + 1e-12)
        m = 2  # the leading pair (sigma_1 / sigma_2 < 1.02, sigma_2 / sigma_3 > 1.9)
        assert sd[0] / sd[1] < 1.02 and sd[1] / sd[2] > 1.9
        e = [dense.sin_angle(Ud[:, :m], X[:, :m]) for X in (r.U_QU, r.U_AV, r.U_svd)]
        assert e[1] < e[0] and e[2] < e[1]
        assert dense.sin_angle(Vd[:, :m], r.V_svd[:, :m]) < dense.sin_angle(Vd[:, :m], r.V[:, :m])
