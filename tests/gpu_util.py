"""Helpers for the GPU parity tests: building oracle-side operators from the
same seeded workloads, comparing gains and subspaces."""
import numpy as np

import workloads as W
from oracle import operator as op
from oracle import sketch as osk


def oracle_problem(w):
    U = W.base_flow(w)
    hx, hy = op.spacing(w.nx, w.ny, w.domain)
    coef = op.burgers_coefficients(U, w.nx, w.ny, hx, hy, w.nu)
    L = op.assemble(coef)
    phi = osk.gradient_weight(U, hx, hy).ravel()
    return U, coef, L, phi, hx, hy


def to_np(t):
    return t.detach().cpu().numpy()


def max_rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b) / np.abs(b)))


def gain_errors(sig, ref, floor=1e-3):
    """Relative errors |d sigma_j| / sigma_j for sigma_j >= floor*sigma_1, else
    |d sigma_j| / sigma_1 (a backward-stable SVD is only absolutely accurate
    to eps*sigma_1 for the small ones)."""
    sig = np.asarray(sig)
    ref = np.asarray(ref)
    den = np.where(ref >= floor * ref[0], ref, ref[0])
    return np.abs(sig - ref) / den


def clusters(sig, rel_gap=1e-3):
    """Index groups of singular values separated by relative gaps > rel_gap."""
    groups, cur = [], [0]
    for j in range(1, len(sig)):
        if (sig[j - 1] - sig[j]) / sig[j - 1] > rel_gap:
            groups.append(cur)
            cur = [j]
        else:
            cur.append(j)
    groups.append(cur)
    return groups


def sin_angle(A, B):
    Qa, _ = np.linalg.qr(A)
    Qb, _ = np.linalg.qr(B)
    return float(np.linalg.norm(Qb - Qa @ (Qa.conj().T @ Qb), 2))


def mode_angles(V_gpu, V_ref, sig_ref, upto):
    """Largest sine angle over the clusters fully inside the first `upto` modes."""
    worst = 0.0
    for g in clusters(sig_ref):
        if g[-1] >= upto:
            break
        worst = max(worst, sin_angle(V_gpu[:, g], V_ref[:, g]))
    return worst
