"""CPU checks of the built library: it loads and exports every entry point
declared in include/die_te.h (no compute call is made without a GPU)."""
import ctypes
import os

import pytest

from paper_1104_4263_amd import _lib


def test_header_declares_the_boundary():
    names = _lib.header_symbols()
    for n in ("die_te_setup", "die_te_setup_multi", "die_te_matvec", "die_te_regularize", "die_te_solve", "die_te_destroy",
              "die_te_last_error", "die_te_apply_deflation", "die_te_deflation_info", "die_te_fft2"):
        assert n in names


def test_library_loads_and_exports_every_symbol():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libdie_te.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(_lib.LIB_PATH)
    for n in _lib.header_symbols():
        assert hasattr(lib, n), n


def test_last_error_without_gpu_calls():
    lib = _lib.load()
    assert lib.die_te_last_error() == b""
    # a null context is rejected before any HIP call
    assert lib.die_te_matvec(None, None, None, 1, 0, None) == _lib.DIE_E_INVALID
    assert b"context" in lib.die_te_last_error()


def test_setup_multi_validates_before_any_gpu_call():
    lib = _lib.load()
    ctx = ctypes.c_void_p()
    g = _lib.DieTeGrid(8, 8, 0.05, 0.0, 0, 0)
    dummy = ctypes.c_void_p(16)  # never dereferenced: the object count is checked first
    assert lib.die_te_setup_multi(ctypes.byref(ctx), ctypes.byref(g), 0, dummy, None, None) == _lib.DIE_E_INVALID
    assert b"nobj" in lib.die_te_last_error()
    g.nx = 0
    assert lib.die_te_setup_multi(ctypes.byref(ctx), ctypes.byref(g), 2, dummy, None, None) == _lib.DIE_E_INVALID
    assert not ctx.value


def test_unet_create_validates_before_any_gpu_call():
    lib = _lib.load()
    net = ctypes.c_void_p()
    # the coarsest level of a 3-level network on 16 x 16 would be 4 wide (needs 8)
    assert lib.die_te_unet_create(ctypes.byref(net), 3, 8, 16, 16, 1, 0, None) == _lib.DIE_E_INVALID
    assert b"multiples" in lib.die_te_last_error()
    assert lib.die_te_unet_create(ctypes.byref(net), 2, 12, 16, 16, 1, 0, None) == _lib.DIE_E_INVALID
    assert lib.die_te_unet_create(ctypes.byref(net), 2, 8, 16, 16, 0, 0, None) == _lib.DIE_E_INVALID
    assert not net.value
    assert lib.die_te_unet_forward(None, None, None, 1, None) == _lib.DIE_E_INVALID


def test_solve_batch_validates_before_any_gpu_call():
    lib = _lib.load()
    vp = ctypes.c_void_p
    o = _lib.DieTeSolveOpts(30, 100, 1e-8, 0, 0, 0.0, 0, 0, 0)
    one = (ctypes.c_int * 2)(1, 1)
    dummy = (vp * 2)(vp(16), vp(32))  # never dereferenced: the argument checks come first
    assert lib.die_te_solve_batch(None, 2, dummy, dummy, one, ctypes.byref(o), None, None) == _lib.DIE_E_INVALID
    assert lib.die_te_solve_batch(dummy, 0, dummy, dummy, one, ctypes.byref(o), None, None) == _lib.DIE_E_INVALID
    same = (vp * 2)(vp(16), vp(16))
    assert lib.die_te_solve_batch(same, 2, dummy, dummy, one, ctypes.byref(o), None, None) == _lib.DIE_E_INVALID
    assert b"twice" in lib.die_te_last_error()
    nul = (vp * 2)(vp(16), None)
    assert lib.die_te_solve_batch(nul, 2, dummy, dummy, one, ctypes.byref(o), None, None) == _lib.DIE_E_INVALID
    assert b"null" in lib.die_te_last_error()
