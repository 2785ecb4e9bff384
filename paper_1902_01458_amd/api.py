"""Python front end over the C ABI: device buffers are torch tensors, the
stream is torch's current stream, every step runs in librr.so's kernels.

    prob = BurgersProblem.from_workload(w)               # U, coefficients, Phi on the GPU
    f = factor(prob, omegas, precision="mixed", k_max=20) # one LU per shift (Section 3.1)
    Q = f.sketch_solve(k, seed, q)                        # Alg. 1 steps 1-3 (+ Section 2.2.1)
    Z = f.adjoint_solve(Q)                                # step 4
    out = f.gains(Q, Z, "av")                             # steps 5-9 (eq. 8, eq. 9)
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib
from ._lib import RRError, check, lib

PRECISIONS = {"fp64": _lib.RR_FP64, "mixed": _lib.RR_MIXED}
RESPONSES = {"av": _lib.RR_RESP_AV, "qu": _lib.RR_RESP_QU, "none": _lib.RR_RESP_NONE}

# numerical failures of a mixed-precision pass that an FP64 factorisation can
# cure: a zero or non-finite FP32 pivot, refinement that missed its tolerance,
# a CholeskyQR breakdown or non-finite values downstream of a stalled solve
_FP64_CURABLE = (2, 3, 4, 5)
# Factors() options that only the mixed path reads
_MIXED_ONLY = ("refine_iters", "refine_tol", "refine_tol_sketch", "refine_method", "gmres_restart")


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must be on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


@dataclasses.dataclass
class BurgersProblem:
    """The operator of eq. (1) as the library consumes it (all on the GPU)."""
    nx: int
    ny: int
    coef: torch.Tensor                 # (nx*ny*12,) float64
    phi: Optional[torch.Tensor]        # (nx*ny,) float64 or None
    U: Optional[torch.Tensor] = None   # ((nx+2)*(ny+2),) float64
    domain: tuple = (0.0, 1.0, 0.0, 1.0)
    nu: float = 0.0

    @property
    def n(self) -> int:
        return 2 * self.nx * self.ny

    @classmethod
    def from_base_flow(cls, U, nx: int, ny: int, domain, nu: float,
                       weighted: bool = True, device="cuda") -> "BurgersProblem":
        """Coefficients and Phi computed on the GPU (rr_burgers_coeffs).  U is the
        (nx+2, ny+2) base flow with its boundary ring, host array or GPU tensor."""
        if isinstance(U, torch.Tensor) and U.is_cuda:
            Ud = U.detach().to(torch.float64).contiguous().reshape(-1)
        else:
            Ud = torch.as_tensor(np.ascontiguousarray(U, dtype=np.float64).reshape(-1),
                                 device=device)
        if Ud.numel() != (nx + 2) * (ny + 2):
            raise ValueError("U must have (nx+2)*(ny+2) values")
        coef = torch.empty(nx * ny * 12, dtype=torch.float64, device=device)
        phi = torch.empty(nx * ny, dtype=torch.float64, device=device) if weighted else None
        check(lib().rr_burgers_coeffs(nx, ny, _ptr(Ud), *map(float, domain), float(nu),
                                      _ptr(coef), _ptr(phi), ctypes.c_void_p(_stream())))
        return cls(nx, ny, coef, phi, Ud, tuple(map(float, domain)), float(nu))

    @classmethod
    def from_workload(cls, w, weighted: bool = True, device="cuda") -> "BurgersProblem":
        import workloads
        return cls.from_base_flow(workloads.base_flow(w), w.nx, w.ny, w.domain, w.nu,
                                  weighted=weighted, device=device)

    @classmethod
    def from_coefficients(cls, coef: np.ndarray, phi=None, device="cuda") -> "BurgersProblem":
        """Any operator in the 12-coefficient stencil format, shape (nx, ny, 12)."""
        nx, ny, _ = coef.shape
        c = torch.as_tensor(np.ascontiguousarray(coef, dtype=np.float64).reshape(-1), device=device)
        p = None if phi is None else torch.as_tensor(
            np.ascontiguousarray(phi, dtype=np.float64).reshape(-1), device=device)
        return cls(nx, ny, c, p)

    def c_struct(self) -> _lib.Problem:
        x0, x1, y0, y1 = self.domain
        return _lib.Problem(self.nx, self.ny, self.coef.data_ptr(),
                            self.phi.data_ptr() if self.phi is not None else None,
                            self.U.data_ptr() if self.U is not None else None,
                            x0, x1, y0, y1, self.nu)

    def apply(self, omegas: Sequence[complex], X: torch.Tensor, adjoint: bool = False):
        """Y = M(omega) X (or M^H X) for X of shape (n_omega, k, n) complex128."""
        om = np.asarray(omegas, dtype=np.complex128).reshape(-1)
        n_om, k, n = X.shape
        if n != self.n or n_om != om.size:
            raise ValueError("shape mismatch")
        Y = torch.empty_like(X)
        re = np.ascontiguousarray(om.real)
        im = np.ascontiguousarray(om.imag)
        ps = self.c_struct()
        check(lib().rr_apply(ctypes.byref(ps), re.ctypes.data_as(ctypes.c_void_p),
                             im.ctypes.data_as(ctypes.c_void_p), n_om, k, int(adjoint),
                             _ptr(X), _ptr(Y), ctypes.c_void_p(_stream())))
        return Y


class Factors:
    """One band LU per shift (M(omega) = i omega I - L), owned by the library.
    With discount = beta > 0 the shifts become omega - i beta: the discounted
    resolvent of Section 2.1, the growth rates of L lowered by beta (the
    paper's complex frequency omega + i beta in its e^{-i omega t} convention).
    `omegas` keeps the shifts as factored."""

    def __init__(self, prob: BurgersProblem, omegas, precision: str = "fp64", k_max: int = 32,
                 tile: int = 0, grid: int = 0, refine_iters: int = 0, refine_tol: float = 0.0,
                 refine_tol_sketch: float = 0.0, stream=None, discount: float = 0.0,
                 test_matrix: str = "gaussian", zeta: int = 0, refine_method: str = "plain",
                 gmres_restart: int = 0, superblock: int = 0, solver: str = "lu",
                 precond: str = "jacobi", krylov_maxit: int = 0, krylov_tol: float = 0.0):
        # discount beta: the paper's discounted resolvent (Section 2.1),
        # M = i omega I - (L - beta I), i.e. the shift omega - i beta here
        om = np.asarray(omegas, dtype=np.complex128).reshape(-1) - 1j * discount
        self.prob = prob
        self.omegas = om
        self.n_omega = om.size
        self.n = prob.n
        self.k_max = k_max
        self.precision = precision
        self._h = ctypes.c_void_p()
        re = np.ascontiguousarray(om.real)
        im = np.ascontiguousarray(om.imag)
        # refine_method "gmres": GMRES-IR corrections (mixed precision), for
        # shifts where plain refinement with the FP32 LU stalls
        # superblock: block rows per solve step (0: default, < 0: one at a time)
        # solver "bicgstab" / "gmres": no band LU; every solve is a Krylov
        # iteration preconditioned by `precond` ("jacobi" or "ilu0"), FP64
        tune = _lib.Tuning(tile, grid, refine_iters, refine_tol, refine_tol_sketch,
                           _lib.REFINE_METHODS[refine_method], gmres_restart, superblock,
                           _lib.SOLVERS[solver], _lib.PRECONDS[precond], krylov_maxit,
                           krylov_tol)
        ps = prob.c_struct()
        check(lib().rr_factor(ctypes.byref(ps), re.ctypes.data_as(ctypes.c_void_p),
                              im.ctypes.data_as(ctypes.c_void_p), self.n_omega, k_max,
                              PRECISIONS[precision], ctypes.byref(tune),
                              ctypes.c_void_p(_stream(stream)), ctypes.byref(self._h)))
        if test_matrix != "gaussian":
            self.set_test_matrix(test_matrix, zeta)

    def set_test_matrix(self, kind: str, zeta: int = 0):
        """Test matrix of later sketches (Section 2.2.2): "gaussian",
        "rademacher", "sparse" (zeta nonzeros per row, 0: min(k, 8)) or
        "orthonormal"; each weighted by the problem's Phi (eq. 10) if set."""
        check(lib().rr_set_test_matrix(self.handle, _lib.TEST_MATRICES[kind], zeta))

    def set_timing_events(self, factor=None, solve=None):
        """Record torch.cuda.Event pairs (begin, end) around the factorisation
        kernel and the main launch of every solve call (rr_set_timing_events);
        None clears a pair.  The events must outlive their use."""
        def raw(ev):
            return ctypes.c_void_p(ev.cuda_event) if ev is not None else None
        fb, fe = factor if factor is not None else (None, None)
        sb, se = solve if solve is not None else (None, None)
        check(lib().rr_set_timing_events(self.handle, raw(fb), raw(fe), raw(sb), raw(se)))

    def set_jacobi_sweeps(self, sweeps: int):
        """Sweep cap of the k x k Jacobi SVD (default 40); a sweep that still
        rotates at the cap is reported as RR_ERR_NOT_CONVERGED by check()."""
        check(lib().rr_set_jacobi_sweeps(self.handle, sweeps))

    def precond_apply(self, X: torch.Tensor, adjoint: bool = False, out=None) -> torch.Tensor:
        """Y = K^-1 X (or K^-H X) with the Krylov handle's preconditioner, for a
        (n_omega, k, n) complex128 block (rr_precond_apply; a test hook)."""
        X = X.contiguous()
        Y = torch.empty_like(X) if out is None else out
        check(lib().rr_precond_apply(self.handle, X.shape[1], 1 if adjoint else 0,
                                     ctypes.c_void_p(X.data_ptr()), ctypes.c_void_p(Y.data_ptr()),
                                     ctypes.c_void_p(_stream(None))))
        return Y

    # -- lifetime ----------------------------------------------------------
    def free(self):
        if self._h:
            lib().rr_factors_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass

    @property
    def handle(self):
        if not self._h:
            raise RuntimeError("factors were freed")
        return self._h

    def nbytes(self) -> int:
        return int(lib().rr_bytes(self.handle))

    def check(self, stream=None):
        """Synchronise and raise on any device-side error latched so far."""
        check(lib().rr_check(self.handle, ctypes.c_void_p(_stream(stream))))

    def refine_count(self) -> int:
        return int(lib().rr_refine_count(self.handle))

    def refactor(self, stream=None):
        check(lib().rr_refactor(self.handle, ctypes.c_void_p(_stream(stream))))

    # -- Algorithm 1 ---------------------------------------------------------
    def empty_block(self, k: int) -> torch.Tensor:
        return torch.empty((self.n_omega, k, self.n), dtype=torch.complex128, device="cuda")

    def sketch_solve(self, k: int, seed: int = 0, q: int = 0, out=None, stream=None):
        Q = out if out is not None else self.empty_block(k)
        check(lib().rr_sketch_solve(self.handle, k, seed, q, _ptr(Q),
                                    ctypes.c_void_p(_stream(stream))))
        return Q

    def adjoint_solve(self, Q: torch.Tensor, out=None, stream=None):
        k = Q.shape[1]
        Z = out if out is not None else self.empty_block(k)
        check(lib().rr_adjoint_solve(self.handle, k, _ptr(Q), _ptr(Z),
                                     ctypes.c_void_p(_stream(stream))))
        return Z

    def solve(self, Bm: torch.Tensor, out=None, stream=None):
        k = Bm.shape[1]
        X = out if out is not None else self.empty_block(k)
        check(lib().rr_solve(self.handle, k, _ptr(Bm), _ptr(X), ctypes.c_void_p(_stream(stream))))
        return X

    def gains(self, Q: Optional[torch.Tensor], Z: torch.Tensor, response: str = "av",
              out: Optional[dict] = None, stream=None) -> dict:
        k = Z.shape[1]
        dev = "cuda"
        o = out or {}
        sB = o.get("sigma_B", torch.empty((self.n_omega, k), dtype=torch.float64, device=dev))
        V = o.get("V", self.empty_block(k))
        sAV = U = None
        if response == "av":
            sAV = o.get("sigma_AV", torch.empty((self.n_omega, k), dtype=torch.float64, device=dev))
            U = o.get("U", self.empty_block(k))
        elif response == "qu":
            U = o.get("U", self.empty_block(k))
        check(lib().rr_gains(self.handle, k, _ptr(Q) if Q is not None else None, _ptr(Z),
                             RESPONSES[response], _ptr(sB), _ptr(sAV), _ptr(V), _ptr(U),
                             ctypes.c_void_p(_stream(stream))))
        return {"sigma_B": sB, "sigma_AV": sAV, "V": V, "U": U}

    def resvd(self, Us: torch.Tensor, V: torch.Tensor, scale: Optional[torch.Tensor] = None,
              out: Optional[dict] = None, stream=None) -> dict:
        """Optional steps 10-11 of Algorithm 1 (rr_resvd): the SVD of U^Sigma
        (Us, or Us scaled per column by `scale`, e.g. the unit modes U and
        sigma_AV of gains()) gives sigma_svd, orthonormal U_svd and the
        refined forcing modes V_svd = V W."""
        k = Us.shape[1]
        o = out or {}
        sig = o.get("sigma_svd", torch.empty((self.n_omega, k), dtype=torch.float64,
                                             device="cuda"))
        U = o.get("U_svd", self.empty_block(k))
        Vn = o.get("V_svd", self.empty_block(k))
        check(lib().rr_resvd(self.handle, k, _ptr(Us), _ptr(scale), _ptr(V), _ptr(sig), _ptr(U),
                             _ptr(Vn), ctypes.c_void_p(_stream(stream))))
        return {"sigma_svd": sig, "U_svd": U, "V_svd": Vn}

    def grad(self, sigma1: torch.Tensor, u1: torch.Tensor, v1: torch.Tensor, stride: int,
             stream=None):
        """(dU (n_omega, nx+2, ny+2), dnu (n_omega,), domega (n_omega,)) of
        sigma_1; dU covers every node of the base-flow array, ring included."""
        nx, ny = self.prob.nx, self.prob.ny
        dU = torch.empty((self.n_omega, nx + 2, ny + 2), dtype=torch.float64, device="cuda")
        dnu = torch.empty(self.n_omega, dtype=torch.float64, device="cuda")
        dom = torch.empty(self.n_omega, dtype=torch.float64, device="cuda")
        check(lib().rr_grad(self.handle, ctypes.c_void_p(sigma1.data_ptr()),
                            ctypes.c_void_p(u1.data_ptr()), ctypes.c_void_p(v1.data_ptr()),
                            stride, _ptr(dU), _ptr(dnu), _ptr(dom),
                            ctypes.c_void_p(_stream(stream))))
        return dU, dnu, dom


class Graph:
    """One captured pass of Algorithm 1 over every shift of a handle
    (rr_graph_capture); launch() replays it on a stream.  Holds references to
    the handle and the buffers the graph writes."""

    def __init__(self, f: "Factors", k: int, seed: int, q: int, response: str, refactor: bool):
        self.f = f
        self.k = k
        self.Q = f.empty_block(k)
        self.Z = f.empty_block(k)
        self.sigma_B = torch.empty((f.n_omega, k), dtype=torch.float64, device="cuda")
        self.sigma_AV = (torch.empty((f.n_omega, k), dtype=torch.float64, device="cuda")
                         if response == "av" else None)
        self.V = f.empty_block(k)
        self.U = f.empty_block(k) if response in ("av", "qu") else None
        self._g = ctypes.c_void_p()
        check(lib().rr_graph_capture(f.handle, int(refactor), k, seed, q, RESPONSES[response],
                                     _ptr(self.Q), _ptr(self.Z), _ptr(self.sigma_B),
                                     _ptr(self.sigma_AV), _ptr(self.V), _ptr(self.U),
                                     ctypes.byref(self._g)))

    def launch(self, stream=None):
        check(lib().rr_graph_launch(self._g, ctypes.c_void_p(_stream(stream))))
        return {"sigma_B": self.sigma_B, "sigma_AV": self.sigma_AV, "V": self.V, "U": self.U,
                "Q": self.Q}

    def free(self):
        if self._g:
            lib().rr_graph_free(self._g)
            self._g = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def capture(f: Factors, k: int, seed: int = 0, q: int = 0, response: str = "av",
            refactor: bool = True) -> Graph:
    """Record one pass of Algorithm 1 (optionally with the refactorisation) for
    replay with one graph launch."""
    return Graph(f, k, seed, q, response, refactor)


_ALLOCATOR = None  # the registered ctypes callbacks (kept alive here)


def use_torch_allocator(enable: bool = True):
    """Route the device memory of new handles through PyTorch's caching
    allocator (rr_set_allocator), or back to hipMalloc / hipFree."""
    global _ALLOCATOR
    if not enable:
        check(lib().rr_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None))
        _ALLOCATOR = None
        return

    def _alloc(nbytes, stream, ctx):
        try:
            return torch.cuda.caching_allocator_alloc(int(nbytes), stream=stream or 0)
        except Exception:
            return None

    def _free(ptr, ctx):
        torch.cuda.caching_allocator_delete(ptr)

    cbs = (_lib.ALLOC_FN(_alloc), _lib.FREE_FN(_free))
    check(lib().rr_set_allocator(cbs[0], cbs[1], None))
    _ALLOCATOR = cbs


def factor_bytes(nx: int, ny: int, n_omega: int, k_max: int, precision: str = "fp64",
                 tile: int = 0) -> int:
    return int(lib().rr_factor_bytes(nx, ny, n_omega, k_max, PRECISIONS[precision], tile))


def autotune(prob: BurgersProblem, omegas, k: int, precision: str = "fp64",
             max_shifts: int = 0, stream=None) -> dict:
    """The library's autotuner (rr_autotune): fastest band tile, persistent
    grid and solve superblock for this operator, shift batch, width and
    precision (cached in the file RR_AUTOTUNE_CACHE names, if set)."""
    om = np.asarray(omegas, dtype=np.complex128).reshape(-1)
    re = np.ascontiguousarray(om.real)
    im = np.ascontiguousarray(om.imag)
    t = _lib.Tuning()
    ms = ctypes.c_double()
    ps = prob.c_struct()
    check(lib().rr_autotune(ctypes.byref(ps), re.ctypes.data_as(ctypes.c_void_p),
                            im.ctypes.data_as(ctypes.c_void_p), om.size, k,
                            PRECISIONS[precision], max_shifts, ctypes.c_void_p(_stream(stream)),
                            ctypes.byref(t), ctypes.byref(ms)))
    return {"tile": t.tile, "grid": t.grid, "superblock": t.superblock, "ms": ms.value}


def _sweep_chunk(prob, om, k, seed, q, precision, tile, grid, superblock=0):
    f = factor(prob, om, precision, k_max=k, tile=tile, grid=grid, superblock=superblock)
    g = None
    try:
        g = capture(f, k, seed, q, "av", refactor=False)
        out = g.launch()
        f.check()
        return out["sigma_B"].clone(), out["sigma_AV"].clone()
    finally:
        if g is not None:
            g.free()
        f.free()


def _chunk_size(prob, k, precision, tile, memory_fraction, n_omega):
    free, _ = torch.cuda.mem_get_info()
    per = factor_bytes(prob.nx, prob.ny, 1, k, precision, tile) + 6 * k * prob.n * 16
    return max(1, min(n_omega, int(memory_fraction * free // per)))


def sweep(prob: BurgersProblem, omegas, k: int, q: int = 0, seed: int = 0,
          precision: str = "fp64", tune: Optional[dict] = None, chunk: int = 0,
          memory_fraction: float = 0.8, on_failure: str = "raise") -> dict:
    """Frequency sweep sharing one L: the shifts are processed in chunks that
    fit in device memory (rr_factor_bytes), each chunk as one captured graph
    (factorisation, sketch, subspace iteration, adjoint solve, SVD, eq. 9).
    With on_failure="fp64", a mixed-precision chunk that reports a numerical
    failure is refactored and run again in FP64 (in sub-chunks sized for the
    FP64 factors). Returns sigma_B, sigma_AV (n_omega, k) on the GPU, the chunk
    size and the first shift index of every chunk redone in FP64."""
    if on_failure not in ("raise", "fp64"):
        raise ValueError("on_failure must be 'raise' or 'fp64'")
    om = np.asarray(omegas, dtype=np.complex128).reshape(-1)
    tile = int(tune["tile"]) if tune else 0
    grid = int(tune["grid"]) if tune else 0
    sb = int(tune.get("superblock", 0)) if tune else 0
    if chunk <= 0:
        chunk = _chunk_size(prob, k, precision, tile, memory_fraction, om.size)
    sB = torch.empty((om.size, k), dtype=torch.float64, device="cuda")
    sAV = torch.empty((om.size, k), dtype=torch.float64, device="cuda")
    redone = []
    for c0 in range(0, om.size, chunk):
        c1 = min(om.size, c0 + chunk)
        try:
            sB[c0:c1], sAV[c0:c1] = _sweep_chunk(prob, om[c0:c1], k, seed, q, precision, tile,
                                                 grid, sb)
        except RRError as e:
            if on_failure != "fp64" or precision != "mixed" or e.status not in _FP64_CURABLE:
                raise
            sub = _chunk_size(prob, k, "fp64", 0, memory_fraction, c1 - c0)
            for s0 in range(c0, c1, sub):
                s1 = min(c1, s0 + sub)
                sB[s0:s1], sAV[s0:s1] = _sweep_chunk(prob, om[s0:s1], k, seed, q, "fp64", 0, 0)
            redone.append(c0)
    return {"sigma_B": sB, "sigma_AV": sAV, "chunk": chunk, "fp64_chunks": redone}


def factor(prob: BurgersProblem, omegas, precision: str = "fp64", k_max: int = 32, **kw) -> Factors:
    return Factors(prob, omegas, precision, k_max, **kw)


def resolvent(prob: BurgersProblem, omegas, k: int, q: int = 0, seed: int = 0,
              precision: str = "fp64", response: str = "av", factors: Optional[Factors] = None,
              check_status: bool = True, optional_svd: bool = False, on_failure: str = "raise",
              **kw) -> dict:
    """Algorithm 1 for every shift: returns sigma_B, sigma_AV, V, U, Q (GPU
    tensors), and with optional_svd (response "av" only) the optional steps
    10-11 as sigma_svd, U_svd, V_svd. out["precision"] names the path that
    produced the result.

    on_failure="fp64" is the policy for a mixed-precision pass that fails
    numerically (refinement not converged, a zero FP32 pivot, a CholeskyQR
    breakdown or non-finite values): every shift is refactored in FP64 and the
    pass runs again with the same sketch; out["fallback_status"] holds the
    status of the failed pass. It needs the factors to be made here and the
    status to be checked; on the FP64 path it changes nothing."""
    if optional_svd and response != "av":
        raise ValueError("the optional SVD refines the AV recovery (response='av')")
    if on_failure not in ("raise", "fp64"):
        raise ValueError("on_failure must be 'raise' or 'fp64'")
    if on_failure == "fp64" and (factors is not None or not check_status):
        raise ValueError("the FP64 fallback needs factors made here and check_status=True")
    f = factors if factors is not None else factor(prob, omegas, precision, k_max=k, **kw)
    try:
        Q = f.sketch_solve(k, seed, q)
        Z = f.adjoint_solve(Q)
        out = f.gains(Q, Z, response)
        if optional_svd:
            out.update(f.resvd(out["U"], out["V"], scale=out["sigma_AV"]))
        if check_status:
            f.check()
    except RRError as e:
        if on_failure != "fp64" or f.precision != "mixed" or e.status not in _FP64_CURABLE:
            raise
        f.free()
        kw64 = {key: v for key, v in kw.items() if key not in _MIXED_ONLY}
        out = resolvent(prob, omegas, k, q, seed, "fp64", response, None, True, optional_svd,
                        **kw64)
        out["fallback_status"] = e.status
        return out
    out["Q"] = Q
    out["factors"] = f
    out["precision"] = f.precision
    return out


def philox_raw(count: int, c1: int = 0, c2: int = 0, key=(0, 0)) -> torch.Tensor:
    """Raw Philox4x32-10 words from the device generator: (count, 4) uint32 as int64."""
    out = torch.empty(4 * count, dtype=torch.int32, device="cuda")
    check(lib().rr_philox_raw(_ptr(out), count, c1, c2, key[0], key[1],
                              ctypes.c_void_p(_stream())))
    return (out.to(torch.int64) & 0xFFFFFFFF).reshape(count, 4)


def sketch(prob: BurgersProblem, k: int, seed: int = 0, kind: str = "gaussian",
           zeta: int = 0) -> torch.Tensor:
    """The test matrix Theta (k, n) the sketch step draws (eq. 10 weighting),
    for the elementwise kinds ("gaussian", "rademacher", "sparse")."""
    out = torch.empty((k, prob.n), dtype=torch.complex128, device="cuda")
    ps = prob.c_struct()
    check(lib().rr_sketch(ctypes.byref(ps), k, seed, _lib.TEST_MATRICES[kind], zeta, _ptr(out),
                          ctypes.c_void_p(_stream())))
    return out
