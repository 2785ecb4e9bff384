"""GPU gradient of the leading gain through torch.autograd (SigmaOne).

d sigma_1 / d(U, nu, omega) from sigma_1^2 Re(v_1^H dL/dp u_1) (and
sigma_1^2 Im(v_1^H u_1) for omega), evaluated in rr_grad with the recovered
triplet of eq. (9).  Three checks:
  * against the oracle: the FP64 CPU pipeline on the same sketch gives the
    triplet, oracle.grad.gradient the gradient (FP64: 1e-8 of the largest
    entry; mixed: 1e-6 against the same FP64 oracle, since a 1e-8 error on the
    triplet is amplified by the derivative);
  * central finite differences of sigma_1 itself (h = 1e-6, FP64 only: a
    mixed-precision sigma_1 carries ~1e-8 relative noise) on 32 seeded nodes,
    nu and omega;
  * the dense SVD: on an 8 x 8 sub-grid copy of the problem the exact
    triplet from LAPACK gives the exact gradient.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense as odense
from oracle import grad as ograd
from oracle import operator as op
from oracle import resolvent as ores
from oracle import sketch as osk
from tests.gpu_util import oracle_problem, to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


def cfg3_small():
    # config 3's operator (nu = 5e-3, omega in {0.5, 1, 2, 4}, k = 12) on a
    # 64 x 48 grid, so that the FP64 oracle runs in seconds
    return W.small("g3", 64, 48, nu=5e-3, omegas=(0.5, 1.0, 2.0, 4.0), k=12, q=2,
                   domain=(0.0, 8.0, -2.0, 2.0))


def oracle_gradients(w, weights):
    U, coef, L, phi, hx, hy = oracle_problem(w)
    Om = osk.test_matrix(w.n, w.k, phi, seed=0)
    gU = np.zeros((w.nx, w.ny))
    gnu = 0.0
    gom = np.zeros(len(w.omegas))
    for i, om in enumerate(w.omegas):
        r = ores.randomized_resolvent(L, om, Om, q=w.q)
        s1, u1, v1 = r.sigma_AV[0], r.U_AV[:, 0], r.V[:, 0]
        d, dn, do = ograd.gradient(s1, u1, v1, w.nx, w.ny, hx, hy)
        gU += weights[i] * d
        gnu += weights[i] * dn
        gom[i] = weights[i] * do
    return gU, gnu, gom


def gpu_gradients(w, weights, precision):
    U = torch.as_tensor(W.base_flow(w), device="cuda").requires_grad_(True)
    nu = torch.tensor(w.nu, dtype=torch.float64, device="cuda", requires_grad=True)
    om = torch.tensor(w.omegas, dtype=torch.float64, device="cuda", requires_grad=True)
    s = rr().sigma_one(U, nu, om, w.nx, w.ny, w.domain, k=w.k, q=w.q, precision=precision)
    (s * torch.as_tensor(weights, device="cuda")).sum().backward()
    return to_np(U.grad), float(nu.grad), to_np(om.grad), to_np(s.detach())


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("mixed", 1e-6)])
def test_autograd_gradient_matches_oracle(precision, tol):
    w = cfg3_small()
    wts = np.array([1.0, -0.5, 0.25, 2.0])
    gU, gnu, gom, _ = gpu_gradients(w, wts, precision)
    oU, onu, oom = oracle_gradients(w, wts)
    scale = np.abs(oU).max()
    print(f"\n[{precision}] dU err {np.abs(gU[1:-1, 1:-1] - oU).max() / scale:.2e} "
          f"dnu err {abs(gnu - onu) / abs(onu):.2e} dom err {np.abs(gom - oom).max() / np.abs(oom).max():.2e}")
    assert np.abs(gU[0, :]).max() == 0 and np.abs(gU[-1, :]).max() == 0  # the ring is data
    assert np.abs(gU[1:-1, 1:-1] - oU).max() <= tol * scale
    assert abs(gnu - onu) <= tol * abs(onu)
    np.testing.assert_allclose(gom, oom, rtol=0, atol=tol * np.abs(oom).max())


def test_autograd_gradient_matches_central_differences():
    # The formula is the derivative of the exact sigma_1; the randomized
    # estimate's own derivative differs from it by the subspace error, first
    # order in the singular vectors (sigma itself only second order), so the
    # sketch is widened and iterated until that error is below the
    # finite-difference noise.
    w = W.small("g3fd", 64, 48, nu=5e-3, omegas=(0.5, 1.0, 2.0, 4.0), k=24, q=6,
                domain=(0.0, 8.0, -2.0, 2.0))
    wts = np.array([1.0, -0.5, 0.25, 2.0])
    gU, gnu, gom, s0 = gpu_gradients(w, wts, "fp64")
    U0 = W.base_flow(w)
    h = 1e-6

    def objective(U, nu, omegas):
        with torch.no_grad():
            s = rr().sigma_one(torch.as_tensor(U, device="cuda"),
                               torch.tensor(nu, dtype=torch.float64),
                               torch.tensor(omegas, dtype=torch.float64),
                               w.nx, w.ny, w.domain, k=w.k, q=w.q, precision="fp64")
        return float((to_np(s) * wts).sum())

    rng = np.random.default_rng(7)
    nodes = rng.choice(w.nx * w.ny, size=32, replace=False)
    scale = np.abs(gU).max()
    for p in nodes:
        i, j = divmod(int(p), w.ny)
        Up = U0.copy()
        Um = U0.copy()
        Up[i + 1, j + 1] += h
        Um[i + 1, j + 1] -= h
        fd = (objective(Up, w.nu, w.omegas) - objective(Um, w.nu, w.omegas)) / (2 * h)
        print(f"node ({i},{j}) fd {fd:.6e} grad {gU[i + 1, j + 1]:.6e} rel-to-max {abs(fd - gU[i + 1, j + 1]) / scale:.2e}")
        assert abs(fd - gU[i + 1, j + 1]) <= 1e-4 * scale, (i, j, fd, gU[i + 1, j + 1])
    fd_nu = (objective(U0, w.nu + h * w.nu, w.omegas)
             - objective(U0, w.nu - h * w.nu, w.omegas)) / (2 * h * w.nu)
    print(f"nu fd {fd_nu:.8e} grad {gnu:.8e}")
    assert abs(fd_nu - gnu) <= 1e-4 * abs(gnu)
    for i in range(len(w.omegas)):
        op_ = list(w.omegas)
        om_ = list(w.omegas)
        op_[i] += h
        om_[i] -= h
        fd = (objective(U0, w.nu, op_) - objective(U0, w.nu, om_)) / (2 * h)
        print(f"omega {i} fd {fd:.8e} grad {gom[i]:.8e}")
        assert abs(fd - gom[i]) <= 1e-4 * np.abs(gom).max()


def test_autograd_gradient_matches_dense_svd_on_subgrid():
    big = W.CONFIGS["cfg3"]
    Ub = W.base_flow(big)
    hx, hy = op.spacing(big.nx, big.ny, big.domain)
    m = 8
    Us = W.sub_grid(Ub, 100, 40, m)
    dom = (0.0, hx * (m + 1), 0.0, hy * (m + 1))  # the big grid's spacing
    nu = big.nu
    coef = op.burgers_coefficients(Us, m, m, hx, hy, nu)
    L = op.assemble(coef)
    omegas = (0.5, 2.0)
    wts = np.array([1.0, 1.0])
    oU = np.zeros((m, m))
    onu = 0.0
    oom = []
    for om in omegas:
        Uh, s, V = odense.resolvent_svd(L, om)
        d, dn, do = ograd.gradient(s[0], Uh[:, 0], V[:, 0], m, m, hx, hy)
        oU += d
        onu += dn
        oom.append(do)
    Ut = torch.as_tensor(Us, device="cuda").requires_grad_(True)
    nut = torch.tensor(nu, dtype=torch.float64, device="cuda", requires_grad=True)
    omt = torch.tensor(omegas, dtype=torch.float64, device="cuda", requires_grad=True)
    s = rr().sigma_one(Ut, nut, omt, m, m, dom, k=32, q=10, precision="fp64", tile=32)
    s.sum().backward()
    exact = [odense.resolvent_svd(L, om)[1][0] for om in omegas]
    np.testing.assert_allclose(to_np(s.detach()), exact, rtol=1e-10)
    g = to_np(Ut.grad)[1:-1, 1:-1]
    print(f"dense: dU err {np.abs(g - oU).max() / np.abs(oU).max():.2e} nu err {abs(float(nut.grad) - onu) / abs(onu):.2e}")
    assert np.abs(g - oU).max() <= 1e-8 * np.abs(oU).max()
    assert abs(float(nut.grad) - onu) <= 1e-8 * abs(onu)
    np.testing.assert_allclose(to_np(omt.grad), oom, rtol=1e-8, atol=1e-8 * max(map(abs, oom)))
