"""Python binding of the C ABI, one function per entry point, plus a small
convenience class.  Tensors must be contiguous CUDA (HIP) tensors of the dtype
the entry point expects; the current torch stream is passed to the library."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from ._lib import (DIE_C128, DIE_C64, DieTeGrid, DieTePlan, DieTeSetupOpts, DieTeSolveInfo, DieTeSolveOpts, check,
                   load)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, dtypes, name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} must have dtype in {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _prec(t: torch.Tensor) -> int:
    return DIE_C128 if t.dtype == torch.complex128 else DIE_C64


def _setup_opts(regularize, deflate_k, eigs_tol, eigs_krylov, eigs_max_restarts, seed, fft_variant, deflate_max,
                polarization, magnetic, mu_r):
    mu = None if mu_r is None else _dev(mu_r, (torch.complex128,), "mu_r")
    return DieTeSetupOpts(int(bool(regularize)), int(deflate_k), float(eigs_tol), int(eigs_krylov),
                          int(eigs_max_restarts), int(seed), int(fft_variant) + 1, int(deflate_max),
                          1 if polarization in (1, "tm", "TM") else 0, int(bool(magnetic)), mu)


def die_te_setup(nx: int, ny: int, h: float, eps_r: torch.Tensor, *, k_b: float = 0.0, px: int = 0, py: int = 0,
                 regularize: bool = False, deflate_k: int = 0, eigs_tol: float = 1e-4, eigs_krylov: int = 0,
                 eigs_max_restarts: int = 0, seed: int = 0, fft_variant: int = -1,
                 deflate_max: int = 0, polarization=0, magnetic: bool = False,
                 mu_r: torch.Tensor | None = None) -> ctypes.c_void_p:
    """fft_variant: -1 autotunes the FFT passes, 0..3 forces that variant in every pass.
    deflate_k = -1: automatic deflation size (at most deflate_max, 0 -> 256).
    polarization "tm" (or 1): the scalar TM operator; magnetic: the (E1, E2, H3) TE system
    with relative permeability mu_r (device complex128, same shape as eps_r; None = 1)."""
    lib = load()
    g = DieTeGrid(nx, ny, float(h), float(k_b), px, py)
    o = _setup_opts(regularize, deflate_k, eigs_tol, eigs_krylov, eigs_max_restarts, seed, fft_variant, deflate_max,
                    polarization, magnetic, mu_r)
    ctx = ctypes.c_void_p()
    check(lib.die_te_setup(ctypes.byref(ctx), ctypes.byref(g), _dev(eps_r, (torch.complex128,), "eps_r"),
                           ctypes.byref(o), _stream()))
    return ctx


def die_te_setup_multi(nx: int, ny: int, h: float, nobj: int, eps_r: torch.Tensor, *, k_b: float = 0.0, px: int = 0,
                       py: int = 0, regularize: bool = False, deflate_k: int = 0, eigs_tol: float = 1e-4,
                       eigs_krylov: int = 0, eigs_max_restarts: int = 0, seed: int = 0,
                       fft_variant: int = -1, deflate_max: int = 0, polarization=0, magnetic: bool = False,
                       mu_r: torch.Tensor | None = None) -> ctypes.c_void_p:
    lib = load()
    g = DieTeGrid(nx, ny, float(h), float(k_b), px, py)
    o = _setup_opts(regularize, deflate_k, eigs_tol, eigs_krylov, eigs_max_restarts, seed, fft_variant, deflate_max,
                    polarization, magnetic, mu_r)
    ctx = ctypes.c_void_p()
    check(lib.die_te_setup_multi(ctypes.byref(ctx), ctypes.byref(g), int(nobj),
                                 _dev(eps_r, (torch.complex128,), "eps_r"), ctypes.byref(o), _stream()))
    return ctx


def die_te_matvec(ctx, x: torch.Tensor, y: torch.Tensor, nrhs: int) -> None:
    check(load().die_te_matvec(ctx, _dev(x, (torch.complex128, torch.complex64), "x"),
                               _dev(y, (x.dtype,), "y"), nrhs, _prec(x), _stream()))


def die_te_matvec_noalloc(ctx, x: torch.Tensor, y: torch.Tensor, nrhs: int) -> None:
    check(load().die_te_matvec_noalloc(ctx, _dev(x, (torch.complex128, torch.complex64), "x"),
                                       _dev(y, (x.dtype,), "y"), nrhs, _prec(x), _stream()))


def die_te_regularize(ctx, x: torch.Tensor, y: torch.Tensor, nrhs: int) -> None:
    check(load().die_te_regularize(ctx, _dev(x, (torch.complex128, torch.complex64), "x"),
                                   _dev(y, (x.dtype,), "y"), nrhs, _prec(x), _stream()))


METHODS = {"gmres": 0, "bicgstab": 1, "gcr": 2, "idrs": 3}


def _method(method) -> int:
    if isinstance(method, str):
        if method not in METHODS:
            raise ValueError(f"method must be one of {sorted(METHODS)}")
        return METHODS[method]
    return int(method)


def die_te_solve(ctx, e_in: torch.Tensor, e_tot: torch.Tensor, nrhs: int, *, restart: int = 30,
                 max_iters: int = 100_000, tol: float = 1e-8, mixed: int = 0, x0_given: bool = False,
                 reg_margin: float = 0.0, orth: int = 0, graph: int = 0, block: int = 0,
                 method="gmres") -> tuple[int, list[dict]]:
    """mixed: 0 FP64, 1 (or True) complex64 products and basis, 2 complex64 products with a
    binary16 basis (orth=1).  method: "gmres", "bicgstab", "gcr" (restart = GCR's kept
    directions) or "idrs" (restart = s)."""
    o = DieTeSolveOpts(int(restart), int(max_iters), float(tol), int(mixed), int(bool(x0_given)),
                       float(reg_margin), int(orth), int(bool(graph)), int(block), _method(method))
    info = (DieTeSolveInfo * nrhs)()
    rc = load().die_te_solve(ctx, _dev(e_in, (torch.complex128,), "e_in"), _dev(e_tot, (torch.complex128,), "e_tot"),
                             nrhs, ctypes.byref(o), info, _stream())
    check(rc, allow_warning=True)
    return rc, [info[i].as_dict() for i in range(nrhs)]


def die_te_solve_batch(ctxs, e_ins, e_tots, nrhs, *, restart: int = 30, max_iters: int = 100_000, tol: float = 1e-8,
                       mixed: int = 0, x0_given: bool = False, reg_margin: float = 0.0,
                       orth: int = 0, graph: int = 0, block: int = 0, method="gmres") -> tuple[int, list[list[dict]]]:
    """Several contexts (grid sizes) in one call; returns (code, per-context info lists)."""
    n = len(ctxs)
    if not (len(e_ins) == len(e_tots) == len(nrhs) == n):
        raise ValueError("ctxs, e_ins, e_tots and nrhs must have the same length")
    o = DieTeSolveOpts(int(restart), int(max_iters), float(tol), int(mixed), int(bool(x0_given)),
                       float(reg_margin), int(orth), int(bool(graph)), int(block), _method(method))
    vp = ctypes.c_void_p
    c_arr = (vp * n)(*[vp(c.value if isinstance(c, vp) else c) for c in ctxs])
    i_arr = (vp * n)(*[_dev(t, (torch.complex128,), "e_in") for t in e_ins])
    o_arr = (vp * n)(*[_dev(t, (torch.complex128,), "e_tot") for t in e_tots])
    r_arr = (ctypes.c_int * n)(*[int(r) for r in nrhs])
    infos = [(DieTeSolveInfo * int(r))() for r in nrhs]
    f_arr = (vp * n)(*[ctypes.cast(x, vp) for x in infos])
    rc = load().die_te_solve_batch(c_arr, n, i_arr, o_arr, r_arr, ctypes.byref(o), f_arr, _stream())
    check(rc, allow_warning=True)
    return rc, [[x[k].as_dict() for k in range(int(r))] for x, r in zip(infos, nrhs)]


def die_te_fft_plan(ctx, prec: int, nrhs: int) -> list[int]:
    """The FFT pass variants (row, column + symbol, inverse row) of products of nrhs fields."""
    v = (ctypes.c_int * 3)()
    check(load().die_te_fft_plan(ctx, int(prec), int(nrhs), v, _stream()))
    return [int(x) for x in v]


OPERATORS = {"A": 0, "AR": 1, "ARA": 2, "solved": 3}


def _which(which) -> int:
    if isinstance(which, str):
        if which not in OPERATORS:
            raise ValueError(f"which must be one of {sorted(OPERATORS)}")
        return OPERATORS[which]
    return int(which)


def die_te_operator_dense(ctx, which, obj: int, out: torch.Tensor) -> None:
    """out: device complex128 (nvec, nvec); filled column-major (its transpose, row-major)."""
    check(load().die_te_operator_dense(ctx, _which(which), int(obj), _dev(out, (torch.complex128,), "out"),
                                       _stream()))


def die_te_spectrum(ctx, which, obj: int, nvec: int) -> np.ndarray:
    eig = np.zeros(nvec, dtype=np.complex128)
    check(load().die_te_spectrum(ctx, _which(which), int(obj), ctypes.c_void_p(eig.ctypes.data), _stream()))
    return eig


def die_te_apply_deflation(ctx, x: torch.Tensor, y: torch.Tensor, nrhs: int) -> None:
    check(load().die_te_apply_deflation(ctx, _dev(x, (torch.complex128,), "x"), _dev(y, (torch.complex128,), "y"),
                                        nrhs, _stream()))


def die_te_deflation_info(ctx, nvec: int, device=None, nobj: int = 1):
    """Returns (Ritz values [nobj, r] on CPU, V [nobj, r, nvec] on the device, C [nobj, r, r] on CPU)."""
    lib = load()
    r = ctypes.c_int(0)
    check(lib.die_te_deflation_info(ctx, ctypes.byref(r), None, None, None, _stream()))
    n = r.value
    if n == 0:
        return torch.zeros(nobj, 0, dtype=torch.complex128), None, None
    ritz = torch.zeros(nobj, n, dtype=torch.complex128)
    C = torch.zeros(nobj, n, n, dtype=torch.complex128)
    V = torch.zeros(nobj, n, nvec, dtype=torch.complex128, device=device or "cuda")
    check(lib.die_te_deflation_info(ctx, ctypes.byref(r), ctypes.c_void_p(ritz.data_ptr()),
                                    _dev(V, (torch.complex128,), "V"), ctypes.c_void_p(C.data_ptr()), _stream()))
    return ritz, V, C


def die_te_fft2(data: torch.Tensor, inverse: bool = False) -> None:
    """In-place unnormalised 2-D FFT over the last two axes of a [batch, py, px] tensor."""
    if data.dim() != 3:
        raise ValueError("data must be [batch, py, px]")
    b, py, px = data.shape
    check(load().die_te_fft2(_dev(data, (torch.complex128, torch.complex64), "data"), px, py, b, int(bool(inverse)),
                             _prec(data), _stream()))


def die_te_profile(ctx, every: int) -> None:
    """every >= 1: bracket one launch in `every` of each kind with events; 0: stop."""
    check(load().die_te_profile(ctx, int(every)))


def die_te_profile_read(ctx, kind: int) -> tuple[int, int, float, float]:
    """(bracketed launches, launches seen, total ms and total algorithmic bytes of the
    bracketed launches)."""
    n = ctypes.c_longlong(0)
    seen = ctypes.c_longlong(0)
    ms = ctypes.c_double(0.0)
    nb = ctypes.c_double(0.0)
    check(load().die_te_profile_read(ctx, int(kind), ctypes.byref(n), ctypes.byref(seen), ctypes.byref(ms),
                                     ctypes.byref(nb)))
    return int(n.value), int(seen.value), float(ms.value), float(nb.value)


def die_te_profile_mem(ctx, kind: int) -> float:
    """Total algorithmic HBM bytes of the bracketed launches of `kind` (operand bytes for the
    GEMM kind, whose die_te_profile_read figure is flops)."""
    nb = ctypes.c_double(0.0)
    check(load().die_te_profile_mem(ctx, int(kind), ctypes.byref(nb)))
    return float(nb.value)


def die_te_deflation_radius(eps_r, regularized: bool) -> float:
    """Section 5's deflation radius of an object (eps_r: any array of complex values)."""
    import numpy as np
    e = np.ascontiguousarray(np.asarray(eps_r, dtype=np.complex128).ravel())
    R = ctypes.c_double(0.0)
    check(load().die_te_deflation_radius(ctypes.c_void_p(e.ctypes.data), int(e.size), int(bool(regularized)),
                                         ctypes.byref(R)))
    return float(R.value)


def die_te_plan_memory(mem_bytes: float, beta: float, points_per_wavelength: float, x: float,
                       eps_re_max: float) -> dict:
    """Section 5's memory planner (the paper's 3N system)."""
    p = DieTePlan()
    check(load().die_te_plan_memory(float(mem_bytes), float(beta), float(points_per_wavelength), float(x),
                                    float(eps_re_max), ctypes.byref(p)))
    return p.as_dict()


def die_te_destroy(ctx) -> None:
    if ctx:
        check(load().die_te_destroy(ctx))


def die_te_last_error() -> str:
    return load().die_te_last_error().decode(errors="replace")


class Solver:
    """Scatterers on one grid, owning a library context: eps_r of shape [ny, nx]
    (one object) or [nobj, ny, nx] (nobj objects; batches of fields are then
    grouped object by object, nrhs a multiple of nobj)."""

    def __init__(self, nx: int, ny: int, h: float, eps_r, *, k_b: float = 2.0 * math.pi, px: int = 0, py: int = 0,
                 regularize: bool = False, deflate_k: int = 0, eigs_tol: float = 1e-4, eigs_krylov: int = 0,
                 eigs_max_restarts: int = 0, seed: int = 0, fft_variant: int = -1, deflate_max: int = 0,
                 polarization=0, magnetic: bool = False, mu_r=None, device: str = "cuda"):
        eps = torch.as_tensor(eps_r, dtype=torch.complex128).to(device).contiguous()
        mu = None if mu_r is None else torch.as_tensor(mu_r, dtype=torch.complex128).to(device).contiguous()
        if mu is not None and mu.shape != eps.shape:
            raise ValueError("mu_r must have the shape of eps_r")
        if tuple(eps.shape[-2:]) != (ny, nx) or eps.dim() not in (2, 3):
            raise ValueError(f"eps_r must have shape ({ny}, {nx}) or (nobj, {ny}, {nx})")
        self.nobj = 1 if eps.dim() == 2 else int(eps.shape[0])
        self.nx, self.ny, self.h, self.k_b = nx, ny, h, k_b
        self.ncomp = 1 if polarization in (1, "tm", "TM") else (3 if magnetic else 2)
        self.nvec = self.ncomp * nx * ny
        self.device = device
        self.regularized = bool(regularize)
        kw = dict(k_b=k_b, px=px, py=py, regularize=regularize, deflate_k=deflate_k, eigs_tol=eigs_tol,
                  eigs_krylov=eigs_krylov, eigs_max_restarts=eigs_max_restarts, seed=seed, fft_variant=fft_variant,
                  deflate_max=deflate_max, polarization=polarization, magnetic=magnetic, mu_r=mu)
        if eps.dim() == 2:
            self.ctx = die_te_setup(nx, ny, h, eps, **kw)
        else:
            self.ctx = die_te_setup_multi(nx, ny, h, self.nobj, eps, **kw)

    @classmethod
    def from_grid(cls, grid, eps_r, **kw):
        return cls(grid.nx, grid.ny, grid.h, eps_r, k_b=grid.k, **kw)

    def _shape(self, x: torch.Tensor) -> int:
        if x.shape[-3:] != (self.ncomp, self.ny, self.nx):
            raise ValueError(f"fields must be [..., {self.ncomp}, {self.ny}, {self.nx}]")
        return 1 if x.dim() == 3 else int(x.shape[0])

    def matvec(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        die_te_matvec(self.ctx, x.contiguous(), y, self._shape(x))
        return y

    def regularize(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        die_te_regularize(self.ctx, x.contiguous(), y, self._shape(x))
        return y

    def solve(self, e_in: torch.Tensor, x0: torch.Tensor | None = None, **kw):
        nrhs = self._shape(e_in)
        out = x0.clone().contiguous() if x0 is not None else torch.empty_like(e_in)
        rc, info = die_te_solve(self.ctx, e_in.contiguous(), out, nrhs, x0_given=x0 is not None, **kw)
        return out, rc, info

    @staticmethod
    def solve_batch(solvers, e_ins, x0s=None, inplace=False, **kw):
        """Solvers on different grids in one call: returns [(u, info)] per solver and the code.
        inplace: the solutions overwrite the (contiguous) initial guesses x0s instead of copies."""
        nrhs = [s._shape(e) for s, e in zip(solvers, e_ins)]
        if x0s is not None and any(x0 is None for x0 in x0s):
            raise ValueError("x0s must give an initial guess for every solver (or be None)")
        if inplace and (x0s is None or any(not x0.is_contiguous() for x0 in x0s)):
            raise ValueError("inplace needs contiguous initial guesses")
        outs = [(x0 if inplace else x0.clone().contiguous()) if x0 is not None else torch.empty_like(e)
                for e, x0 in zip(e_ins, x0s or [None] * len(e_ins))]
        rc, infos = die_te_solve_batch([s.ctx for s in solvers], [e.contiguous() for e in e_ins], outs, nrhs,
                                       x0_given=x0s is not None, **kw)
        return [(u, inf) for u, inf in zip(outs, infos)], rc

    def fft_plan(self, nrhs: int, dtype=torch.complex64) -> list[int]:
        return die_te_fft_plan(self.ctx, DIE_C128 if dtype == torch.complex128 else DIE_C64, nrhs)

    def dense_operator(self, which="A", obj: int = 0) -> torch.Tensor:
        """The dense nvec x nvec matrix of an operator ("A", "AR", "ARA" or "solved") for one object."""
        out = torch.empty((self.nvec, self.nvec), dtype=torch.complex128, device=self.device)
        die_te_operator_dense(self.ctx, which, obj, out)
        return out.t()  # the library writes column-major

    def spectrum(self, which="A", obj: int = 0) -> np.ndarray:
        """All eigenvalues of that matrix (nvec <= 4096)."""
        return die_te_spectrum(self.ctx, which, obj, self.nvec)

    def apply_deflation(self, x: torch.Tensor) -> torch.Tensor:
        y = torch.empty_like(x)
        nrhs = x.numel() // self.nvec
        die_te_apply_deflation(self.ctx, x.contiguous(), y, nrhs)
        return y

    def deflation_info(self):
        """(Ritz values, V, C): shapes [r], [r, nvec], [r, r] for one object, with a
        leading [nobj] axis for several."""
        ritz, V, C = die_te_deflation_info(self.ctx, self.nvec, device=self.device, nobj=self.nobj)
        if self.nobj == 1:
            return ritz[0], (None if V is None else V[0]), (None if C is None else C[0])
        return ritz, V, C

    def profile(self, every: int) -> None:
        die_te_profile(self.ctx, every)

    def profile_read(self, kind: int) -> tuple[int, int, float, float]:
        return die_te_profile_read(self.ctx, kind)

    def profile_mem(self, kind: int) -> float:
        return die_te_profile_mem(self.ctx, kind)

    def close(self):
        if self.ctx:
            die_te_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------- learned warm start
def die_te_unet_create(levels: int, base: int, height: int, width: int, max_batch: int, seed: int = 0):
    net = ctypes.c_void_p()
    check(load().die_te_unet_create(ctypes.byref(net), int(levels), int(base), int(height), int(width),
                                    int(max_batch), int(seed), _stream()))
    return net


def die_te_unet_num_params(net) -> int:
    n = ctypes.c_longlong(0)
    check(load().die_te_unet_num_params(net, ctypes.byref(n)))
    return int(n.value)


def _host_f32(t: torch.Tensor, name: str) -> ctypes.c_void_p:
    if t.device.type != "cpu" or t.dtype != torch.float32 or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous CPU float32 tensor")
    return ctypes.c_void_p(t.data_ptr())


def die_te_unet_get_params(net, params: torch.Tensor) -> None:
    check(load().die_te_unet_get_params(net, _host_f32(params, "params"), _stream()))


def die_te_unet_set_params(net, params: torch.Tensor) -> None:
    check(load().die_te_unet_set_params(net, _host_f32(params, "params"), _stream()))


def die_te_unet_get_grads(net, grads: torch.Tensor) -> None:
    check(load().die_te_unet_get_grads(net, _host_f32(grads, "grads"), _stream()))


def die_te_unet_forward(net, x: torch.Tensor, y: torch.Tensor, batch: int) -> None:
    check(load().die_te_unet_forward(net, _dev(x, (torch.float32,), "x"), _dev(y, (torch.float32,), "y"), int(batch),
                                     _stream()))


def die_te_unet_loss_grad(net, x: torch.Tensor, target: torch.Tensor, batch: int) -> float:
    loss = ctypes.c_double(0.0)
    check(load().die_te_unet_loss_grad(net, _dev(x, (torch.float32,), "x"), _dev(target, (torch.float32,), "target"),
                                       int(batch), ctypes.byref(loss), _stream()))
    return float(loss.value)


def die_te_unet_adam(net, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    check(load().die_te_unet_adam(net, float(lr), float(beta1), float(beta2), float(eps), _stream()))


def die_te_unet_train_step(net, x: torch.Tensor, target: torch.Tensor, batch: int, lr: float) -> float:
    loss = ctypes.c_double(0.0)
    check(load().die_te_unet_train_step(net, _dev(x, (torch.float32,), "x"), _dev(target, (torch.float32,), "target"),
                                        int(batch), float(lr), ctypes.byref(loss), _stream()))
    return float(loss.value)


def die_te_unet_pack_inputs(eps_r: torch.Tensor, nobj: int, e_in: torch.Tensor, x: torch.Tensor, batch: int, ny: int,
                            nx: int) -> None:
    check(load().die_te_unet_pack_inputs(_dev(eps_r, (torch.complex128,), "eps_r"), int(nobj),
                                         _dev(e_in, (torch.complex128,), "e_in"), _dev(x, (torch.float32,), "x"),
                                         int(batch), int(ny), int(nx), _stream()))


def die_te_unet_pack_targets(e_tot: torch.Tensor, e_in: torch.Tensor, t: torch.Tensor, batch: int, ny: int,
                             nx: int) -> None:
    check(load().die_te_unet_pack_targets(_dev(e_tot, (torch.complex128,), "e_tot"),
                                          _dev(e_in, (torch.complex128,), "e_in"), _dev(t, (torch.float32,), "t"),
                                          int(batch), int(ny), int(nx), _stream()))


def die_te_warm_start(ctx, net, e_in: torch.Tensor, x0: torch.Tensor, nrhs: int) -> None:
    check(load().die_te_warm_start(ctx, net, _dev(e_in, (torch.complex128,), "e_in"),
                                   _dev(x0, (torch.complex128,), "x0"), int(nrhs), _stream()))


def die_te_unet_destroy(net) -> None:
    if net:
        check(load().die_te_unet_destroy(net))


class UNet:
    """The warm-start network: owns a library network object."""

    def __init__(self, levels: int, base: int, height: int, width: int, max_batch: int, seed: int = 0):
        self.levels, self.base, self.height, self.width, self.max_batch = levels, base, height, width, max_batch
        self.net = die_te_unet_create(levels, base, height, width, max_batch, seed)
        self.n_params = die_te_unet_num_params(self.net)

    def get_params(self) -> torch.Tensor:
        p = torch.empty(self.n_params, dtype=torch.float32)
        die_te_unet_get_params(self.net, p)
        return p

    def set_params(self, p) -> None:
        die_te_unet_set_params(self.net, torch.as_tensor(p, dtype=torch.float32).contiguous())

    def get_grads(self) -> torch.Tensor:
        g = torch.empty(self.n_params, dtype=torch.float32)
        die_te_unet_get_grads(self.net, g)
        return g

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        b = int(x.shape[0])
        y = torch.empty(b, self.height, self.width, 4, dtype=torch.float32, device=x.device)
        die_te_unet_forward(self.net, x.contiguous(), y, b)
        return y

    def loss_grad(self, x: torch.Tensor, target: torch.Tensor) -> float:
        return die_te_unet_loss_grad(self.net, x.contiguous(), target.contiguous(), int(x.shape[0]))

    def adam(self, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
        die_te_unet_adam(self.net, lr, beta1, beta2, eps)

    def train_step(self, x: torch.Tensor, target: torch.Tensor, lr: float) -> float:
        return die_te_unet_train_step(self.net, x.contiguous(), target.contiguous(), int(x.shape[0]), lr)

    @staticmethod
    def pack_inputs(eps_r: torch.Tensor, e_in: torch.Tensor) -> torch.Tensor:
        """eps_r [nobj, ny, nx], e_in [batch, 2, ny, nx] (complex128, device) -> [batch, ny, nx, 8]."""
        b, _, ny, nx = e_in.shape
        eps = eps_r if eps_r.dim() == 3 else eps_r[None]
        x = torch.empty(b, ny, nx, 8, dtype=torch.float32, device=e_in.device)
        die_te_unet_pack_inputs(eps.contiguous(), int(eps.shape[0]), e_in.contiguous(), x, b, ny, nx)
        return x

    @staticmethod
    def pack_targets(e_tot: torch.Tensor, e_in: torch.Tensor) -> torch.Tensor:
        b, _, ny, nx = e_in.shape
        t = torch.empty(b, ny, nx, 4, dtype=torch.float32, device=e_in.device)
        die_te_unet_pack_targets(e_tot.contiguous(), e_in.contiguous(), t, b, ny, nx)
        return t

    def warm_start(self, solver: "Solver", e_in: torch.Tensor) -> torch.Tensor:
        x0 = torch.empty_like(e_in)
        nrhs = 1 if e_in.dim() == 3 else int(e_in.shape[0])
        die_te_warm_start(solver.ctx, self.net, e_in.contiguous(), x0, nrhs)
        return x0

    def close(self):
        if self.net:
            die_te_unet_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
