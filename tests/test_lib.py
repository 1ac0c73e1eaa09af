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


def test_ctypes_structs_match_the_header(tmp_path):
    """The binding's mirrors of the header's structs have the C layout (size and every field
    offset), measured by a C program compiled against include/die_te.h."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    pairs = [("die_te_grid", _lib.DieTeGrid), ("die_te_setup_opts", _lib.DieTeSetupOpts),
             ("die_te_solve_opts", _lib.DieTeSolveOpts), ("die_te_solve_info", _lib.DieTeSolveInfo),
             ("die_te_plan", _lib.DieTePlan)]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "die_te.h"', 'int main(void) {']
    for cname, py in pairs:
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for f, _ in py._fields_:
            lines.append(f'  printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include")
    subprocess.run([cc, "-I", inc, str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, py in pairs:
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for f, _ in py._fields_:
            assert got[(cname, f)] == getattr(py, f).offset, (cname, f)
