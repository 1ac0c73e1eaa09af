"""ctypes declarations of the C ABI in include/die_te.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdie_te.so")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
HEADERS = [os.path.join(INCLUDE, "die_te.h"), os.path.join(INCLUDE, "die_te_learn.h")]

DIE_OK = 0
DIE_NOT_CONVERGED = 1
DIE_E_INVALID = -1
DIE_E_SINGULAR = -2
DIE_E_NOMEM = -3
DIE_E_HIP = -4
DIE_E_BREAKDOWN = -5
DIE_C128 = 0
DIE_C64 = 1
DIE_PROF_PRODUCT = 0
DIE_PROF_DOTS = 1
DIE_PROF_AXPY = 2
DIE_PROF_GEMM = 3


class DieTeGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("h", ctypes.c_double), ("k_b", ctypes.c_double),
                ("px", ctypes.c_int), ("py", ctypes.c_int)]


class DieTeSetupOpts(ctypes.Structure):
    _fields_ = [("regularize", ctypes.c_int), ("deflate_k", ctypes.c_int), ("eigs_tol", ctypes.c_double),
                ("eigs_krylov", ctypes.c_int), ("eigs_max_restarts", ctypes.c_int), ("seed", ctypes.c_ulonglong),
                ("fft_variant", ctypes.c_int), ("deflate_max", ctypes.c_int), ("polarization", ctypes.c_int),
                ("magnetic", ctypes.c_int), ("mu_r", ctypes.c_void_p)]


class DieTeSolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int), ("max_iters", ctypes.c_int), ("tol", ctypes.c_double),
                ("mixed", ctypes.c_int), ("x0_given", ctypes.c_int), ("reg_margin", ctypes.c_double),
                ("orth", ctypes.c_int), ("graph", ctypes.c_int), ("block", ctypes.c_int), ("method", ctypes.c_int)]


class DieTeSolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("products_A", ctypes.c_int),
                ("products_AR", ctypes.c_int), ("cycles", ctypes.c_int), ("rel_res_true", ctypes.c_double),
                ("finish_iters", ctypes.c_int)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class DieTePlan(ctypes.Structure):
    _fields_ = [("alpha", ctypes.c_double), ("n_max", ctypes.c_double), ("a_over_lambda_max", ctypes.c_double),
                ("nodes", ctypes.c_longlong), ("n", ctypes.c_longlong), ("unknowns", ctypes.c_longlong),
                ("r", ctypes.c_int), ("restart", ctypes.c_int), ("restart_unpreconditioned", ctypes.c_int),
                ("mem_system", ctypes.c_double), ("mem_preconditioner", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class DieTeError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"die_te error {code}: {msg}")
        self.code = code


_lib = None


def load() -> ctypes.CDLL:
    """Load libdie_te.so built in-tree; raise loudly when it is missing (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1104_4263_amd.build` "
                           "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, ip, i = ctypes.c_void_p, ctypes.c_int, ctypes.c_int
    lib.die_te_setup.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(DieTeGrid), vp, ctypes.POINTER(DieTeSetupOpts), vp]
    lib.die_te_setup_multi.argtypes = [ctypes.POINTER(vp), ctypes.POINTER(DieTeGrid), i, vp,
                                       ctypes.POINTER(DieTeSetupOpts), vp]
    lib.die_te_matvec.argtypes = [vp, vp, vp, i, i, vp]
    lib.die_te_matvec_noalloc.argtypes = [vp, vp, vp, i, i, vp]
    lib.die_te_regularize.argtypes = [vp, vp, vp, i, i, vp]
    lib.die_te_solve.argtypes = [vp, vp, vp, i, ctypes.POINTER(DieTeSolveOpts), ctypes.POINTER(DieTeSolveInfo), vp]
    lib.die_te_solve_batch.argtypes = [ctypes.POINTER(vp), i, ctypes.POINTER(vp), ctypes.POINTER(vp),
                                       ctypes.POINTER(ctypes.c_int), ctypes.POINTER(DieTeSolveOpts),
                                       ctypes.POINTER(vp), vp]
    lib.die_te_apply_deflation.argtypes = [vp, vp, vp, i, vp]
    lib.die_te_operator_dense.argtypes = [vp, i, i, vp, vp]
    lib.die_te_spectrum.argtypes = [vp, i, i, vp, vp]
    lib.die_te_fft_plan.argtypes = [vp, i, i, ctypes.POINTER(ctypes.c_int), vp]
    lib.die_te_deflation_info.argtypes = [vp, ctypes.POINTER(ip), vp, vp, vp, vp]
    lib.die_te_fft2.argtypes = [vp, i, i, i, i, i, vp]
    lib.die_te_destroy.argtypes = [vp]
    lib.die_te_deflation_radius.argtypes = [vp, ctypes.c_longlong, i, ctypes.POINTER(ctypes.c_double)]
    lib.die_te_plan_memory.argtypes = [ctypes.c_double] * 5 + [ctypes.POINTER(DieTePlan)]
    lib.die_te_profile.argtypes = [vp, i]
    lib.die_te_profile_read.argtypes = [vp, i, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong),
                                        ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]
    lib.die_te_profile_mem.argtypes = [vp, i, ctypes.POINTER(ctypes.c_double)]
    lib.die_te_last_error.argtypes = []
    lib.die_te_last_error.restype = ctypes.c_char_p
    fp, dp, ll, f, ull = (ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_double), ctypes.c_longlong,
                          ctypes.c_float, ctypes.c_ulonglong)
    lib.die_te_unet_create.argtypes = [ctypes.POINTER(vp), i, i, i, i, i, ull, vp]
    lib.die_te_unet_num_params.argtypes = [vp, ctypes.POINTER(ll)]
    lib.die_te_unet_get_params.argtypes = [vp, vp, vp]
    lib.die_te_unet_set_params.argtypes = [vp, vp, vp]
    lib.die_te_unet_get_grads.argtypes = [vp, vp, vp]
    lib.die_te_unet_forward.argtypes = [vp, vp, vp, i, vp]
    lib.die_te_unet_loss_grad.argtypes = [vp, vp, vp, i, dp, vp]
    lib.die_te_unet_adam.argtypes = [vp, f, f, f, f, vp]
    lib.die_te_unet_train_step.argtypes = [vp, vp, vp, i, f, dp, vp]
    lib.die_te_unet_pack_inputs.argtypes = [vp, i, vp, vp, i, i, i, vp]
    lib.die_te_unet_pack_targets.argtypes = [vp, vp, vp, i, i, i, vp]
    lib.die_te_warm_start.argtypes = [vp, vp, vp, vp, i, vp]
    lib.die_te_unet_destroy.argtypes = [vp]
    for name in header_symbols():
        if name != "die_te_last_error":
            getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


def header_symbols() -> list[str]:
    """Names of the functions declared in include/*.h."""
    names = set()
    for path in HEADERS:
        with open(path) as f:
            names.update(re.findall(r"^\s*(?:int|const char \*)\s*(die_te_\w+)\s*\(", f.read(), re.M))
    return sorted(names)


def check(code: int, allow_warning: bool = False) -> int:
    if code < 0 or (code > 0 and not allow_warning):
        msg = load().die_te_last_error().decode(errors="replace")
        raise DieTeError(code, msg)
    return code
