"""The largest configuration: 1024 x 512 Burgers operator (n = 1048576,
half-bandwidth 1024), base flow with smoothed noise, nu = 1e-3, k = 32, one
subspace iteration, shifts from the 16-point sweep in [0.2, 8].

The FP64 oracle cannot run here (its band array alone is 51.6 GB per shift),
so this size is checked GPU against GPU: the mixed-precision sweep against the
FP64 sweep (sigma_1 relative 1e-8, the mixed-path tolerance) and the mixed
gradient against the FP64 gradient; both paths are pinned to the oracle at
the smaller configurations.  All sixteen shifts of the sweep are compared;
sweep() sizes the shift chunks from the free device memory.
"""
import numpy as np
import pytest
import torch

import workloads as W
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


def test_cfg4_mixed_sweep_matches_fp64_sweep():
    w = W.CONFIGS["cfg4"]
    oms = list(w.omegas)
    prob = rr().BurgersProblem.from_workload(w)
    mixed = rr().sweep(prob, oms, w.k, q=w.q, seed=w.seed, precision="mixed")
    fp64 = rr().sweep(prob, oms, w.k, q=w.q, seed=w.seed, precision="fp64")
    s_m = to_np(mixed["sigma_AV"])
    s_d = to_np(fp64["sigma_AV"])
    assert np.all(np.isfinite(s_m)) and np.all(np.isfinite(s_d))
    assert s_m.shape == (16, w.k)
    rel = np.abs(s_m[:, 0] - s_d[:, 0]) / s_d[:, 0]
    print(f"\ncfg4 16 shifts: max sigma_1 mixed vs fp64 {rel.max():.2e}, chunks "
          f"{mixed['chunk']} / {fp64['chunk']}")
    assert rel.max() <= 1e-8, rel
    rel_b = np.abs(to_np(mixed["sigma_B"])[:, :5] - to_np(fp64["sigma_B"])[:, :5]) / \
        to_np(fp64["sigma_B"])[:, :1]
    assert rel_b.max() <= 1e-8


def test_cfg4_mixed_gradient_matches_fp64_gradient():
    w = W.CONFIGS["cfg4"]
    om = torch.tensor([w.omegas[5]], dtype=torch.float64)
    grads = {}
    for prec in ("fp64", "mixed"):
        U = torch.as_tensor(W.base_flow(w), device="cuda").requires_grad_(True)
        nu = torch.tensor(w.nu, dtype=torch.float64, requires_grad=True)
        s = rr().sigma_one(U, nu, om, w.nx, w.ny, w.domain, k=w.k, q=w.q, precision=prec)
        s.sum().backward()
        grads[prec] = (to_np(U.grad), float(nu.grad), float(s.detach()[0]))
        del U, s
        torch.cuda.empty_cache()
    gd, nd, sd = grads["fp64"]
    gm, nm, sm = grads["mixed"]
    assert abs(sm - sd) <= 1e-8 * sd
    assert np.abs(gm - gd).max() <= 1e-6 * np.abs(gd).max()
    assert abs(nm - nd) <= 1e-6 * abs(nd)
