"""The TM operator and the full three-component TE system (E1, E2, H3) with magnetic
contrast, written from their element formulas.

TEST INFRASTRUCTURE ONLY (see the package docstring).

TM (Section 2 eq. MatrixSolutionTM with chi_m = 0): E3_in = E3 - k_b^2 g * (chi_e E3), a
scalar operator of the form identity plus compact (Section 4).  Collocation with the midpoint
rule gives A = I - T X with, for m != n and the self cell (disc of equal area, a = h/sqrt(pi)),

  T(d) = k^2 h^2 (i/4) H0(k r),        T(0) = (i pi k a / 2) H1(k a) - 1,

the formulas the paper prints for its [A33] block (Section 4, the element formulas through
eq. A33) with chi_e in place of chi_m.

Full TE system (Section 4 eq. lin_system, unknowns u = [E1, E2, H3]): A = I - T X with
X = diag(chi_e, chi_e, chi_m) and the symmetric 3 x 3 kernel (eps_b = mu_b = 1, omega = k)

  T11, T12, T22   the E-block of eq. A11 (oracle.operator.kernel_offdiag),
  T13 = (omega mu_b k h^2 / 4) H1(k r) theta_2,   T31 = (omega eps_b k h^2 / 4) H1(k r) theta_2,
  T23 = -(omega mu_b k h^2 / 4) H1(k r) theta_1,  T32 = -(omega eps_b k h^2 / 4) H1(k r) theta_1,
  T33 = k^2 h^2 (i/4) H0(k r),            T33(0) = (i pi k a / 2) H1(k a) - 1,
  T13(0) = T23(0) = 0 (the gradient of g integrates to zero over the centred disc).

T13 and T32 are the paper's printed [A13] and [A32] (times -1/chi).  The printed relations
[A31] = -[A13] and [A23] = -[A32] disagree with the compact kernels K31 and K23 of Section 3
(eqs. KompactKernel31, KompactKernel23) and with the derivation from eq. MatrixSolutionTE;
T31 and T23 above follow those kernels: K31 = -i omega eps_b d2 g and K23 = i omega mu_b d1 g.

Unknown ordering: components in blocks of N cells, cells row-major (arrays [c, ny, nx]).
"""

from __future__ import annotations

import math

import numpy as np
import scipy.linalg
from scipy.special import hankel1

from .operator import kernel_offdiag, kernel_self


def tm_kernel_offdiag(dx, dy, h: float, k: float):
    """T(d) = k^2 h^2 (i/4) H0(k |d|) for d != 0 (the [A33] off-diagonal formula)."""
    r = np.hypot(np.asarray(dx, dtype=np.float64), np.asarray(dy, dtype=np.float64))
    return k * k * h * h * 0.25j * hankel1(0, k * r)


def tm_kernel_self(h: float, k: float) -> complex:
    """T(0) = (i pi k a / 2) H1(k a) - 1, a = h / sqrt(pi) (the [A33] diagonal formula, eq. A33)."""
    a = h / math.sqrt(math.pi)
    return complex(0.5j * math.pi * k * a * hankel1(1, k * a) - 1.0)


def cross_kernels(dx, dy, h: float, k: float, omega: float | None = None, eps_b: float = 1.0, mu_b: float = 1.0):
    """(T13, T23, T31, T32) at the separation (dx, dy) != 0."""
    omega = k if omega is None else omega
    dx = np.asarray(dx, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    r = np.hypot(dx, dy)
    H1 = hankel1(1, k * r)
    t1, t2 = dx / r, dy / r
    c = k * h * h / 4.0 * H1
    return omega * mu_b * c * t2, -omega * mu_b * c * t1, omega * eps_b * c * t2, -omega * eps_b * c * t1


def _lags(grid):
    nx, ny, h = grid.nx, grid.ny, grid.h
    N = nx * ny
    ix = np.tile(np.arange(nx), ny)
    iy = np.repeat(np.arange(ny), nx)
    DX = (ix[:, None] - ix[None, :]) * h  # x_n - x_m: rows n (targets), columns m (sources)
    DY = (iy[:, None] - iy[None, :]) * h
    diag = np.eye(N, dtype=bool)
    return N, np.where(diag, 1.0, DX), np.where(diag, 0.0, DY), diag


def dense_operator_tm(grid, chi: np.ndarray) -> np.ndarray:
    """The N x N TM matrix A = I - T X, element by element."""
    N, DX, DY, diag = _lags(grid)
    T = tm_kernel_offdiag(DX, DY, grid.h, grid.k)
    T[diag] = tm_kernel_self(grid.h, grid.k)
    A = -T * np.asarray(chi, dtype=np.complex128).reshape(N)[None, :]
    A[np.arange(N), np.arange(N)] += 1.0
    return A


def dense_operator_full(grid, chi_e: np.ndarray, chi_m: np.ndarray) -> np.ndarray:
    """The 3N x 3N TE matrix on [E1, E2, H3] with electric and magnetic contrast."""
    N, DX, DY, diag = _lags(grid)
    h, k = grid.h, grid.k
    t11, t12, t22 = kernel_offdiag(DX, DY, h, k)
    ts = kernel_self(h, k)
    t11[diag] = ts
    t22[diag] = ts
    t12[diag] = 0.0
    t13, t23, t31, t32 = cross_kernels(DX, DY, h, k)
    for t in (t13, t23, t31, t32):
        t[diag] = 0.0
    t33 = tm_kernel_offdiag(DX, DY, h, k)
    t33[diag] = tm_kernel_self(h, k)
    ce = np.asarray(chi_e, dtype=np.complex128).reshape(N)[None, :]
    cm = np.asarray(chi_m, dtype=np.complex128).reshape(N)[None, :]
    A = np.empty((3 * N, 3 * N), dtype=np.complex128)
    blocks = [[(t11, ce), (t12, ce), (t13, cm)], [(t12, ce), (t22, ce), (t23, cm)], [(t31, ce), (t32, ce), (t33, cm)]]
    for i in range(3):
        for j in range(3):
            t, c = blocks[i][j]
            A[i * N:(i + 1) * N, j * N:(j + 1) * N] = -t * c
    A[np.arange(3 * N), np.arange(3 * N)] += 1.0
    return A


def apply_operator_full(grid, chi_e, chi_m, x: np.ndarray) -> np.ndarray:
    """Direct O(N^2) product y = A x on x of shape [3, ny, nx]: every source cell summed for
    every target cell with the element formulas (one target row of cells at a time)."""
    nx, ny, h, k = grid.nx, grid.ny, grid.h, grid.k
    x = np.asarray(x, dtype=np.complex128)
    w = np.stack([np.asarray(chi_e) * x[0], np.asarray(chi_e) * x[1], np.asarray(chi_m) * x[2]]).reshape(3, -1)
    JX, JY = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    jx, jy = JX.ravel(), JY.ravel()
    y = x.reshape(3, -1).copy()
    for iy in range(ny):
        for ix in range(nx):
            n = iy * nx + ix
            dx, dy = (ix - jx) * h, (iy - jy) * h
            self_ = (dx == 0) & (dy == 0)
            dxs, dys = np.where(self_, 1.0, dx), np.where(self_, 0.0, dy)
            t11, t12, t22 = kernel_offdiag(dxs, dys, h, k)
            t13, t23, t31, t32 = cross_kernels(dxs, dys, h, k)
            t33 = tm_kernel_offdiag(dxs, dys, h, k)
            for t, v in ((t11, kernel_self(h, k)), (t22, kernel_self(h, k)), (t33, tm_kernel_self(h, k))):
                t[self_] = v
            for t in (t12, t13, t23, t31, t32):
                t[self_] = 0.0
            y[0, n] -= t11 @ w[0] + t12 @ w[1] + t13 @ w[2]
            y[1, n] -= t12 @ w[0] + t22 @ w[1] + t23 @ w[2]
            y[2, n] -= t31 @ w[0] + t32 @ w[1] + t33 @ w[2]
    return y.reshape(3, ny, nx)


def apply_operator_tm(grid, chi, x: np.ndarray) -> np.ndarray:
    """Direct O(N^2) TM product on x of shape [ny, nx] (or [R, ny, nx])."""
    x = np.asarray(x, dtype=np.complex128)
    X = x if x.ndim == 3 else x[None]
    nx, ny, h, k = grid.nx, grid.ny, grid.h, grid.k
    JX, JY = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    jx, jy = JX.ravel(), JY.ravel()
    W = (np.asarray(chi)[None] * X).reshape(X.shape[0], -1)
    Y = X.reshape(X.shape[0], -1).copy()
    ts = tm_kernel_self(h, k)
    for iy in range(ny):
        for ix in range(nx):
            dx, dy = (ix - jx) * h, (iy - jy) * h
            self_ = (dx == 0) & (dy == 0)
            t = tm_kernel_offdiag(np.where(self_, 1.0, dx), np.where(self_, 0.0, dy), h, k)
            t[self_] = ts
            Y[:, iy * nx + ix] -= W @ t
    Y = Y.reshape(X.shape)
    return Y if x.ndim == 3 else Y[0]


def plane_wave_tm(grid, psi: float) -> np.ndarray:
    """Incident E3 = exp(i k (x cos psi + y sin psi)) on the cell centres."""
    x = grid.x0 + (np.arange(grid.nx) + 0.5) * grid.h
    y = grid.y0 + (np.arange(grid.ny) + 0.5) * grid.h
    X, Y = np.meshgrid(x, y, indexing="xy")
    return np.exp(1j * grid.k * (X * math.cos(psi) + Y * math.sin(psi)))


def solve_dense_tm(grid, eps_r, b):
    """u = A^-1 b for the TM system by dense LU; b [ny, nx] or [R, ny, nx]."""
    A = dense_operator_tm(grid, np.asarray(eps_r, dtype=np.complex128) - 1.0)
    b = np.asarray(b, dtype=np.complex128)
    B = b.reshape(-1, grid.n).T
    U = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), B)
    return U.T.reshape(b.shape)


def solve_dense_full(grid, eps_r, mu_r, b):
    """u = A^-1 b for the full TE system by dense LU; b [3, ny, nx] or [R, 3, ny, nx]."""
    A = dense_operator_full(grid, np.asarray(eps_r) - 1.0, np.asarray(mu_r) - 1.0)
    b = np.asarray(b, dtype=np.complex128)
    B = b.reshape(-1, 3 * grid.n).T
    U = scipy.linalg.lu_solve(scipy.linalg.lu_factor(A), B)
    return U.T.reshape(b.shape)
