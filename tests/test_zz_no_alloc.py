"""rr_grad_noalloc: the gradient without any device allocation (a file-scope
scratch array per GPU), through the C ABI, against rr_grad on the same
triplets: bitwise equal (same kernels, same reduction order), on two calls in
a row, the second with a smaller problem; the size limit is rejected on the
host.  Runs alone in a fresh process and after the other tests."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W
from paper_1902_01458_amd import _lib
from tests.gpu_util import to_np

pytestmark = pytest.mark.gpu


def rr():
    import paper_1902_01458_amd as m
    return m


def reference(w, omegas, k):
    """A pass of Algorithm 1 and rr_grad on its handle; returns the triplets
    (kept alive) and the handle's gradient."""
    prob = rr().BurgersProblem.from_workload(w)
    f = rr().factor(prob, omegas, "fp64", k_max=k, tile=32)
    Q = f.sketch_solve(k, 0, 0)
    Z = f.adjoint_solve(Q)
    out = f.gains(Q, Z, "av")
    s1 = out["sigma_AV"][:, 0].contiguous()
    dU, dnu, dom = f.grad(s1, out["U"], out["V"], k * prob.n)
    f.check()
    f.free()
    return prob, s1, out["U"], out["V"], to_np(dU), to_np(dnu), to_np(dom)


def noalloc(prob, n_omega, s1, u, v, stride):
    L = _lib.lib()
    dU = torch.full((n_omega, prob.nx + 2, prob.ny + 2), float("nan"), dtype=torch.float64,
                    device="cuda")
    dnu = torch.full((n_omega,), float("nan"), dtype=torch.float64, device="cuda")
    dom = torch.full((n_omega,), float("nan"), dtype=torch.float64, device="cuda")
    ps = prob.c_struct()
    st = L.rr_grad_noalloc(ctypes.byref(ps), n_omega, ctypes.c_void_p(s1.data_ptr()),
                           ctypes.c_void_p(u.data_ptr()), ctypes.c_void_p(v.data_ptr()), stride,
                           ctypes.c_void_p(dU.data_ptr()), ctypes.c_void_p(dnu.data_ptr()),
                           ctypes.c_void_p(dom.data_ptr()),
                           ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == 0, L.rr_last_error()
    torch.cuda.synchronize()
    return to_np(dU), to_np(dnu), to_np(dom)


def test_noalloc_gradient_equals_handle_gradient_twice():
    big = W.small("na1", 40, 24, nu=1e-2, omegas=(0.5, 1.7, 3.1), k=8)
    small = W.small("na2", 12, 10, nu=2e-2, omegas=(0.9,), k=4)
    for w in (big, small):   # the second call is smaller than the first
        prob, s1, u, v, gU, gnu, gom = reference(w, list(w.omegas), w.k)
        dU, dnu, dom = noalloc(prob, len(w.omegas), s1, u, v, w.k * prob.n)
        np.testing.assert_array_equal(dU, gU)
        np.testing.assert_array_equal(dnu, gnu)
        np.testing.assert_array_equal(dom, gom)


def test_noalloc_rejects_sizes_beyond_its_scratch():
    L = _lib.lib()
    w = W.CONFIGS["cfg4"]                       # 2060 chunks per shift at 1024 x 512
    ps = _lib.Problem(w.nx, w.ny, None, None, None, *w.domain, w.nu)
    one = torch.zeros(1, dtype=torch.float64, device="cuda")
    args = [ctypes.c_void_p(one.data_ptr())] * 3
    st = L.rr_grad_noalloc(ctypes.byref(ps), 64, *args, 2 * w.n * 32, *args, None)
    assert st == 1 and b"scratch" in L.rr_last_error()
    assert L.rr_grad_noalloc(None, 1, *args, 0, *args, None) == 1
