"""Host-only checks of the C ABI: the library loads, exports every function
include/rr.h declares, and rejects bad arguments before touching the GPU."""
import ctypes
import os
import re

import pytest

from paper_1902_01458_amd import _lib

HEADER = os.path.join(os.path.dirname(os.path.dirname(__file__)), "include", "rr.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rr_[a-z_0-9]+)\s*\(", txt)))


def test_header_declares_the_entry_points():
    names = declared()
    for must in ("rr_factor", "rr_sketch_solve", "rr_adjoint_solve", "rr_gains", "rr_grad"):
        assert must in names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared():
        assert hasattr(L, name), name
    for name in _lib.EXPORTS:
        assert hasattr(L, name), name


def test_invalid_arguments_rejected_on_host():
    L = _lib.lib()
    h = ctypes.c_void_p()
    one = (ctypes.c_double * 1)(1.0)
    # NULL problem
    assert L.rr_factor(None, one, None, 1, 4, 0, None, None, ctypes.byref(h)) == 1
    assert b"NULL" in L.rr_last_error()
    # bad sizes
    p = _lib.Problem(0, 4, None, None, None, 0, 1, 0, 1, 0.01)
    assert L.rr_factor(ctypes.byref(p), one, None, 1, 4, 0, None, None, ctypes.byref(h)) == 1
    p = _lib.Problem(4, 4, 1, None, None, 0, 1, 0, 1, 0.01)
    assert L.rr_factor(ctypes.byref(p), one, None, 0, 4, 0, None, None, ctypes.byref(h)) == 1
    assert L.rr_factor(ctypes.byref(p), one, None, 1, 0, 0, None, None, ctypes.byref(h)) == 1
    assert L.rr_factor(ctypes.byref(p), one, None, 1, 33, 0, None, None, ctypes.byref(h)) == 1
    assert L.rr_factor(ctypes.byref(p), one, None, 1, 4, 7, None, None, ctypes.byref(h)) == 1
    nan = (ctypes.c_double * 1)(float("nan"))
    assert L.rr_factor(ctypes.byref(p), nan, None, 1, 4, 0, None, None, ctypes.byref(h)) == 1
    bad_tile = _lib.Tuning(48, 0, 0, 0.0)
    assert L.rr_factor(ctypes.byref(p), one, None, 1, 4, 0, ctypes.byref(bad_tile), None,
                       ctypes.byref(h)) == 1
    for bad in (_lib.Tuning(64, 0, 0, 0.0, 0.0, 2, 0), _lib.Tuning(64, 0, 0, 0.0, 0.0, 1, 17),
                _lib.Tuning(64, 0, 0, 0.0, 0.0, 1, -1)):
        assert L.rr_factor(ctypes.byref(p), one, None, 1, 4, 1, ctypes.byref(bad), None,
                           ctypes.byref(h)) == 1
        assert b"refine_method" in L.rr_last_error() or b"gmres_restart" in L.rr_last_error()
    assert not h
    assert L.rr_factor(ctypes.byref(p), one, None, 1, 4, 0, None, None, None) == 1
    # calls on a NULL handle
    assert L.rr_sketch_solve(None, 4, 0, 0, None, None) == 1
    assert L.rr_adjoint_solve(None, 4, None, None, None) == 1
    assert L.rr_gains(None, 4, None, None, 0, None, None, None, None, None) == 1
    assert L.rr_resvd(None, 4, None, None, None, None, None, None, None) == 1
    assert L.rr_set_test_matrix(None, 0, 0) == 1
    assert L.rr_set_jacobi_sweeps(None, 40) == 1
    assert L.rr_sketch(None, 4, 0, 0, 0, None, None) == 1
    assert L.rr_grad(None, None, None, None, 0, None, None, None, None) == 1
    assert L.rr_check(None, None) == 1
    assert L.rr_refine_count(None) == 0
    assert L.rr_bytes(None) == 0
    L.rr_factors_free(None)
    assert L.rr_burgers_coeffs(0, 3, None, 0, 1, 0, 1, 0.1, None, None, None) == 1
    assert L.rr_philox_raw(None, 4, 0, 0, 0, 0, None) == 1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "librr.so"))
    with pytest.raises(ImportError):
        _lib.lib()


def test_sweep_entry_points_reject_bad_arguments_on_host():
    L = _lib.lib()
    g = ctypes.c_void_p()
    assert L.rr_graph_capture(None, 1, 4, 0, 0, 0, None, None, None, None, None, None,
                              ctypes.byref(g)) == 1
    assert L.rr_graph_launch(None, None) == 1
    L.rr_graph_free(None)  # NULL-safe
    t = _lib.Tuning()
    one = (ctypes.c_double * 1)(1.0)
    assert L.rr_autotune(None, one, None, 1, 4, 0, 0, None, ctypes.byref(t), None) == 1
    p = _lib.Problem(4, 4, 1, None, None, 0, 1, 0, 1, 0.01)
    assert L.rr_autotune(ctypes.byref(p), one, None, 1, 33, 0, 0, None, ctypes.byref(t), None) == 1
    # allocator: both callbacks or neither
    assert L.rr_set_allocator(_lib.ALLOC_FN(lambda n, s, c: None), _lib.FREE_FN(), None) == 1
    assert L.rr_set_allocator(_lib.ALLOC_FN(), _lib.FREE_FN(), None) == 0


def test_factor_bytes_matches_the_layout():
    L = _lib.lib()
    assert L.rr_factor_bytes(0, 4, 1, 4, 0, 0) == 0
    assert L.rr_factor_bytes(4, 4, 1, 33, 1, 0) == 0    # mixed precision: k_max <= 32
    assert L.rr_factor_bytes(4, 4, 1, 513, 0, 0) == 0   # FP64: k_max <= 512
    # a wide FP64 sketch adds its k x k scratch and one wide block
    assert L.rr_factor_bytes(4, 4, 1, 33, 0, 0) > L.rr_factor_bytes(4, 4, 1, 32, 0, 0)
    assert L.rr_factor_bytes(4, 4, 1, 4, 0, 48) == 0
    nx, ny, nw, k, T = 512, 256, 16, 20, 64
    n, b = 2 * nx * ny, 2 * ny
    B, NB = -(-b // T), -(-n // T)
    P = min(B, 256 // T)  # the default superblock: 4 block rows of 64
    # the band, the block-inverse LU and P - 1 superblock-inverse tiles per row, complex FP64
    tiles = nw * NB * (2 * B + 1 + 1 + (P - 1)) * T * T * 16
    got = L.rr_factor_bytes(nx, ny, nw, k, 0, T)
    assert tiles < got < tiles * 1.2
    # FP32 factor: half the tile bytes, one more vector workspace
    assert L.rr_factor_bytes(nx, ny, nw, k, 1, T) < got


def test_fp64_fallback_policy_rejects_bad_options_on_the_host():
    """The failure policy of resolvent() and sweep() is checked before any
    factorisation, so bad options fail without a GPU."""
    import paper_1902_01458_amd as rr
    with pytest.raises(ValueError):
        rr.resolvent(None, [1.0], k=4, on_failure="retry")
    with pytest.raises(ValueError):  # the fallback needs factors it owns
        rr.resolvent(None, [1.0], k=4, precision="mixed", on_failure="fp64", factors=object())
    with pytest.raises(ValueError):  # and a checked status to act on
        rr.resolvent(None, [1.0], k=4, precision="mixed", on_failure="fp64", check_status=False)
    with pytest.raises(ValueError):
        rr.sweep(None, [1.0], 4, on_failure="retry")
