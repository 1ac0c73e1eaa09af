"""The discretised TE operator A = I - T X, written from its element formulas.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Source: Zouros & Budko, Section 4, the collocation system eq. lin_system with
the element formulas eq. A11 .. A33.  With no magnetic contrast the third
(H3) unknown does not feed back into the electric rows, so the in-plane field
(E1, E2) solves the closed 2N x 2N E-block:

  [A_ll]_nm = -k^2 h^2 chi(x_m) { c_theta(k r) theta_l theta_l + c_delta(k r) },   m != n
  [A_lq]_nm = -k^2 h^2 chi(x_m)   c_theta(k r) theta_l theta_q,                     m != n, l != q
  [A_ll]_nn = 1 + [1 - (i pi k a / 4) H1(k a)] chi(x_n),   a = h / sqrt(pi)
  [A_lq]_nn = 0

  c_theta(z) = i/(2z) H1(z) - i/4 H0(z),   c_delta(z) = i/4 H0(z) - i/(4z) H1(z)

r = |x_n - x_m|, theta = (x_n - x_m)/r, H = Hankel functions of the first
kind (scipy / AMOS here; the GPU library evaluates its own).  Writing
T_lq(d) for the bracketed kernel times k^2 h^2 (and T(0) = [(i pi k a/4) H1(k a) - 1] I)
gives A = I - T X with X = diag(chi).

The contrast is chi = eps/eps_b - 1 (eq. ElectricContrast, eps_b = 1); the
regularizer is the same operator with chi' = eps_b/eps - 1 (eq. InverseSymbol,
eq. Regularization); eps = 0 anywhere violates the existence condition
(eq. ExistenceTE).

Unknown ordering: u = [E1 over cells, E2 over cells], cells in row-major
order n = iy * nx + ix, matching arrays shaped [2, ny, nx].
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg
from scipy.special import hankel1


class SingularContrastError(ValueError):
    """eps = 0 in some cell: the symbol I + chi Q is not invertible there."""


def electric_contrast(eps_r: np.ndarray) -> np.ndarray:
    """chi_e = eps / eps_b - 1 with eps_b = 1 (eq. ElectricContrast)."""
    eps_r = np.asarray(eps_r, dtype=np.complex128)
    if np.any(eps_r == 0):
        raise SingularContrastError("eps_r == 0 in some cell (existence condition)")
    return eps_r - 1.0


def regularizer_contrast(eps_r: np.ndarray) -> np.ndarray:
    """chi'_e = eps_b / eps - 1 (eq. InverseSymbol): contrast of the regularizer A(chi')."""
    eps_r = np.asarray(eps_r, dtype=np.complex128)
    if np.any(eps_r == 0):
        raise SingularContrastError("eps_r == 0 in some cell (existence condition)")
    return 1.0 / eps_r - 1.0


def c_theta(z):
    """Coefficient of theta_l theta_q in the kernel (eq. A11): i/(2z) H1(z) - i/4 H0(z)."""
    return 1j / (2.0 * z) * hankel1(1, z) - 0.25j * hankel1(0, z)


def c_delta(z):
    """Coefficient of delta_lq in the kernel (eq. A11): i/4 H0(z) - i/(4z) H1(z)."""
    return 0.25j * hankel1(0, z) - 1j / (4.0 * z) * hankel1(1, z)


def kernel_offdiag(dx, dy, h: float, k: float):
    """T_11, T_12, T_22 at the separation (dx, dy) (in metres, not zero).

    T_lq = k^2 h^2 [c_theta(k r) theta_l theta_q + c_delta(k r) delta_lq]; the
    matrix element is -T_lq chi(x_m) (eq. A11 and the off-diagonal-block formula).
    """
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    r = np.hypot(dx, dy)
    z = k * r
    t1, t2 = dx / r, dy / r
    ct, cd = c_theta(z), c_delta(z)
    s = k * k * h * h
    return s * (ct * t1 * t1 + cd), s * (ct * t1 * t2), s * (ct * t2 * t2 + cd)


def kernel_self(h: float, k: float) -> complex:
    """T(0) coefficient: the diagonal element is 1 - T(0) chi with
    T(0) = (i pi k a / 4) H1(k a) - 1, a = h / sqrt(pi) (diagonal formula after eq. A11).
    """
    a = h / math.sqrt(math.pi)
    return complex(0.25j * math.pi * k * a * hankel1(1, k * a) - 1.0)


def lag_table(nx: int, ny: int, h: float, k: float) -> np.ndarray:
    """T_lq on every lag (dx, dy) = (ix_n - ix_m, iy_n - iy_m) of an nx x ny grid.

    Returns [3, 2ny-1, 2nx-1] complex128 holding T11, T12, T22, indexed
    [.., dy + ny - 1, dx + nx - 1]; the zero lag holds the self term.
    """
    DX, DY = np.meshgrid(np.arange(-(nx - 1), nx) * h, np.arange(-(ny - 1), ny) * h, indexing="xy")
    zero = (DX == 0) & (DY == 0)
    DXs, DYs = np.where(zero, 1.0, DX), np.where(zero, 0.0, DY)  # placeholder at d = 0
    t11, t12, t22 = kernel_offdiag(DXs, DYs, h, k)
    ts = kernel_self(h, k)
    t11 = np.where(zero, ts, t11)
    t22 = np.where(zero, ts, t22)
    t12 = np.where(zero, 0.0, t12)
    return np.stack([t11, t12, t22]).astype(np.complex128)


def dense_operator(grid, chi: np.ndarray) -> np.ndarray:
    """Assemble the 2N x 2N matrix A element by element (eq. A11 family).

    chi: [ny, nx] contrast (chi_e for A, chi'_e for the regularizer A_R).
    Intended for N up to a few thousand cells.
    """
    nx, ny, h, k = grid.nx, grid.ny, grid.h, grid.k
    N = nx * ny
    ix = np.tile(np.arange(nx), ny)
    iy = np.repeat(np.arange(ny), nx)
    DX = (ix[:, None] - ix[None, :]) * h  # x_n - x_m, rows n, columns m
    DY = (iy[:, None] - iy[None, :]) * h
    diag = np.eye(N, dtype=bool)
    DXs, DYs = np.where(diag, 1.0, DX), np.where(diag, 0.0, DY)
    t11, t12, t22 = kernel_offdiag(DXs, DYs, h, k)
    ts = kernel_self(h, k)
    t11[diag] = ts
    t22[diag] = ts
    t12[diag] = 0.0
    c = np.asarray(chi, dtype=np.complex128).reshape(N)[None, :]  # chi(x_m): column scaling
    A = np.empty((2 * N, 2 * N), dtype=np.complex128)
    A[:N, :N] = -t11 * c
    A[:N, N:] = -t12 * c
    A[N:, :N] = -t12 * c
    A[N:, N:] = -t22 * c
    A[np.arange(2 * N), np.arange(2 * N)] += 1.0
    return A


def apply_operator(grid, chi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Direct O(N^2) product y = A x, summing every source cell for every target.

    x: [2, ny, nx] (or [R, 2, ny, nx]).  The sum over source cells is grouped
    by the source-row/target-row offset dy: for a fixed dy the coupling between
    row iy and row iy - dy is the Toeplitz matrix K_lq(dy)[ix, jx] =
    T_lq(ix - jx, dy) -- the block structure of A itself -- applied with a
    matrix product.  No FFT and no circulant embedding are involved.
    """
    x = np.asarray(x, dtype=np.complex128)
    batched = x.ndim == 4
    X = x if batched else x[None]
    nx, ny = grid.nx, grid.ny
    lag = lag_table(nx, ny, grid.h, grid.k)
    chi = np.asarray(chi, dtype=np.complex128)
    W = X * chi[None, None]  # chi(x_m) x_m
    Y = X.copy()
    toe = np.arange(nx)[:, None] - np.arange(nx)[None, :] + nx - 1  # ix - jx + nx - 1
    pairs = ((0, 0, 0), (0, 1, 1), (1, 0, 1), (1, 1, 2))  # (l, q, index of T_lq in the lag table)
    for dy in range(-(ny - 1), ny):
        row = lag[:, dy + ny - 1, :]
        K = row[:, toe]  # [3, nx(ix), nx(jx)]
        iy0, iy1 = max(0, dy), min(ny, ny + dy)  # target rows with a source row iy - dy in range
        for l, q, t in pairs:
            # Y[:, l, iy, ix] -= sum_jx K[t][ix, jx] W[:, q, iy - dy, jx]
            Y[:, l, iy0:iy1, :] -= W[:, q, iy0 - dy:iy1 - dy, :] @ K[t].T
    return Y if batched else Y[0]


def apply_operator_at(grid, chi: np.ndarray, x: np.ndarray, samples) -> np.ndarray:
    """(A x) at selected outputs only: samples is a list of (component, iy, ix).

    Each output is the explicit sum over all source cells of the element
    formulas -- O(N) per sample -- so it serves for grids too large for
    ``apply_operator``.
    """
    x = np.asarray(x, dtype=np.complex128)
    chi = np.asarray(chi, dtype=np.complex128)
    nx, ny, h, k = grid.nx, grid.ny, grid.h, grid.k
    JX, JY = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    w1, w2 = chi * x[0], chi * x[1]
    out = []
    for comp, iy, ix in samples:
        DX = (ix - JX) * h
        DY = (iy - JY) * h
        self_mask = (DX == 0) & (DY == 0)
        DXs, DYs = np.where(self_mask, 1.0, DX), np.where(self_mask, 0.0, DY)
        t11, t12, t22 = kernel_offdiag(DXs, DYs, h, k)
        ts = kernel_self(h, k)
        t11[self_mask] = ts
        t22[self_mask] = ts
        t12[self_mask] = 0.0
        if comp == 0:
            s = np.sum(t11 * w1) + np.sum(t12 * w2)
        else:
            s = np.sum(t12 * w1) + np.sum(t22 * w2)
        out.append(x[comp, iy, ix] - s)
    return np.array(out, dtype=np.complex128)


def apply_operator_loops(grid, chi: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Pure-Python double loop over target and source cells (tiny grids only)."""
    nx, ny, h, k = grid.nx, grid.ny, grid.h, grid.k
    y = np.array(x, dtype=np.complex128)
    ts = kernel_self(h, k)
    for iy in range(ny):
        for ix in range(nx):
            acc1 = 0j
            acc2 = 0j
            for jy in range(ny):
                for jx in range(nx):
                    w1 = chi[jy, jx] * x[0, jy, jx]
                    w2 = chi[jy, jx] * x[1, jy, jx]
                    if ix == jx and iy == jy:
                        acc1 += ts * w1
                        acc2 += ts * w2
                        continue
                    dx, dy = (ix - jx) * h, (iy - jy) * h
                    r = math.hypot(dx, dy)
                    z = k * r
                    ct = complex(c_theta(z))
                    cd = complex(c_delta(z))
                    t1, t2 = dx / r, dy / r
                    s = k * k * h * h
                    acc1 += s * ((ct * t1 * t1 + cd) * w1 + ct * t1 * t2 * w2)
                    acc2 += s * (ct * t1 * t2 * w1 + (ct * t2 * t2 + cd) * w2)
            y[0, iy, ix] -= acc1
            y[1, iy, ix] -= acc2
    return y


def lu_solver(A: np.ndarray):
    """LU factorisation of the dense matrix; returns a function b -> A^{-1} b."""
    lu = scipy.linalg.lu_factor(A)
    return lambda b: scipy.linalg.lu_solve(lu, b)


def solve_dense(grid, eps_r: np.ndarray, e_in: np.ndarray) -> np.ndarray:
    """Discrete total field u = A^{-1} b by dense LU (b = sampled incident field).

    e_in: [2, ny, nx] or [R, 2, ny, nx]; returns the same shape.
    """
    chi = electric_contrast(eps_r)
    A = dense_operator(grid, chi)
    solve = lu_solver(A)
    b = np.asarray(e_in, dtype=np.complex128)
    batched = b.ndim == 4
    B = b.reshape(-1, 2 * grid.n).T if batched else b.reshape(2 * grid.n)
    U = solve(B)
    return U.T.reshape(b.shape) if batched else U.reshape(b.shape)


def relative_residual(grid, eps_r: np.ndarray, u: np.ndarray, e_in: np.ndarray) -> float:
    """||b - A u||_2 / ||b||_2 with the direct-sum product (per RHS max if batched)."""
    chi = electric_contrast(eps_r)
    r = np.asarray(e_in) - apply_operator(grid, chi, u)
    if np.asarray(u).ndim == 4:
        num = np.linalg.norm(r.reshape(r.shape[0], -1), axis=1)
        den = np.linalg.norm(np.asarray(e_in).reshape(r.shape[0], -1), axis=1)
        return float(np.max(num / den))
    return float(np.linalg.norm(r) / np.linalg.norm(e_in))
