"""Grids, permittivity maps and incident fields (inputs only).

Conventions (shared by every consumer of these inputs):

* background: eps_b = mu_b = 1, wavelength lambda_b = 1, so k_b = omega = 2*pi;
* a grid has ``nx`` x ``ny`` square cells of side ``h``; cell (ix, iy) has its
  centre at ``(x0 + (ix + 1/2) h, y0 + (iy + 1/2) h)``;
* 2-D arrays are indexed ``[iy, ix]`` (x fastest in memory);
* a curved object is staircased: a cell belongs to it when its centre does
  (boundary ties count as inside).  The paper attributes most of its
  discretisation error for the circular cylinder to exactly this crude
  representation of the boundary (Section 4, grid rule discussion).
"""

from __future__ import annotations

from dataclasses import dataclass
import math

import numpy as np
from scipy.special import ndtr

TWO_PI = 2.0 * math.pi


@dataclass(frozen=True)
class Grid:
    nx: int
    ny: int
    h: float
    x0: float
    y0: float
    k: float = TWO_PI  # background wavenumber k_b (lambda_b = 1)

    @property
    def n(self) -> int:
        return self.nx * self.ny


def centred_grid(nx: int, side: float, ny: int | None = None, k: float = TWO_PI) -> Grid:
    """Grid of ``nx`` cells across a square of side ``side`` centred at the origin."""
    ny = nx if ny is None else ny
    h = side / nx
    return Grid(nx=nx, ny=ny, h=h, x0=-0.5 * nx * h, y0=-0.5 * ny * h, k=k)


def cell_centres(g: Grid) -> tuple[np.ndarray, np.ndarray]:
    """Return (X, Y), each ``[ny, nx]``, the cell-centre coordinates."""
    x = g.x0 + (np.arange(g.nx) + 0.5) * g.h
    y = g.y0 + (np.arange(g.ny) + 0.5) * g.h
    return np.meshgrid(x, y, indexing="xy")


def cylinder(g: Grid, radius: float, eps: complex, centre=(0.0, 0.0)) -> np.ndarray:
    """Homogeneous circular cylinder of relative permittivity ``eps`` in vacuum."""
    X, Y = cell_centres(g)
    inside = (X - centre[0]) ** 2 + (Y - centre[1]) ** 2 <= radius * radius
    out = np.ones((g.ny, g.nx), dtype=np.complex128)
    out[inside] = eps
    return out


def square(g: Grid, side: float, eps: complex, centre=(0.0, 0.0)) -> np.ndarray:
    """Square cross-section of side ``side`` (cells whose centre lies inside)."""
    X, Y = cell_centres(g)
    half = 0.5 * side
    inside = (np.abs(X - centre[0]) <= half + 1e-12) & (np.abs(Y - centre[1]) <= half + 1e-12)
    out = np.ones((g.ny, g.nx), dtype=np.complex128)
    out[inside] = eps
    return out


def layered_square(g: Grid, side: float, eps_outer: complex, eps_core: complex) -> np.ndarray:
    """Square of side ``side`` with a concentric square core of side ``side/2``."""
    out = square(g, side, eps_outer)
    core = square(g, 0.5 * side, eps_core)
    out[core != 1.0] = eps_core
    return out


def ellipse_mask(g: Grid, a: float, b: float, theta: float = 0.0, centre=(0.0, 0.0)) -> np.ndarray:
    X, Y = cell_centres(g)
    dx, dy = X - centre[0], Y - centre[1]
    c, s = math.cos(theta), math.sin(theta)
    u = c * dx + s * dy
    v = -s * dx + c * dy
    return (u / a) ** 2 + (v / b) ** 2 <= 1.0


def plane_wave(g: Grid, psi: float, k: float | None = None) -> np.ndarray:
    """In-plane electric field of a unit TE plane wave travelling at angle ``psi``.

    H3 = exp(i k (x cos psi + y sin psi)); Maxwell's TE equations in the
    background then give E = (-sin psi, cos psi) H3 (with k = omega, eps_b = 1).
    Returned as ``[2, ny, nx]`` complex128 (component 0 = E1 = E_x).
    """
    k = g.k if k is None else k
    X, Y = cell_centres(g)
    phase = np.exp(1j * k * (X * math.cos(psi) + Y * math.sin(psi)))
    return np.stack([-math.sin(psi) * phase, math.cos(psi) * phase]).astype(np.complex128)


def plane_wave_te3(g: Grid, psi: float, k: float | None = None) -> np.ndarray:
    """The TE plane wave with its out-of-plane magnetic field: [E1, E2, H3] ([3, ny, nx])."""
    E = plane_wave(g, psi, k)
    k = g.k if k is None else k
    X, Y = cell_centres(g)
    H3 = np.exp(1j * k * (X * math.cos(psi) + Y * math.sin(psi)))
    return np.concatenate([E, H3[None]]).astype(np.complex128)


def plane_wave_tm(g: Grid, psi: float, k: float | None = None) -> np.ndarray:
    """Electric field E3 of a unit TM plane wave travelling at angle ``psi`` ([1, ny, nx])."""
    k = g.k if k is None else k
    X, Y = cell_centres(g)
    return np.exp(1j * k * (X * math.cos(psi) + Y * math.sin(psi)))[None].astype(np.complex128)


def gaussian_random_field(n: int, h: float, ell: float, seed: int) -> np.ndarray:
    """Unit-variance, zero-mean periodic Gaussian random field on an n x n grid.

    White noise (PCG64, ``seed``) filtered in Fourier space by the square root of
    the spectral density of the covariance exp(-r^2 / (2 ell^2)), then rescaled
    to unit sample variance.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.standard_normal((n, n))
    kx = 2.0 * math.pi * np.fft.fftfreq(n, d=h)
    KX, KY = np.meshgrid(kx, kx, indexing="xy")
    filt = np.exp(-0.25 * ell * ell * (KX * KX + KY * KY))
    z = np.fft.ifft2(np.fft.fft2(w) * filt).real
    z -= z.mean()
    z /= z.std()
    return z


def random_field_object(n: int, seed: int, h: float = 1.0 / 48.0, ell: float = 0.5) -> tuple[Grid, np.ndarray]:
    """Random-field scatterer of the batched workload.

    Re eps = 1 + 9 U, Im eps = 0.5 U2 with U, U2 uniform marginals obtained as
    the normal CDF of two independent Gaussian random fields (correlation
    length ``ell``), masked to a random centred ellipse (semi-axes uniform in
    [0.25, 0.45] L, rotation uniform in [0, pi)); eps = 1 outside.
    """
    g = centred_grid(n, n * h)
    U = ndtr(gaussian_random_field(n, h, ell, seed))
    U2 = ndtr(gaussian_random_field(n, h, ell, seed + 10_000))
    eps = (1.0 + 9.0 * U) + 1j * (0.5 * U2)
    rng = np.random.Generator(np.random.PCG64(seed + 20_000))
    L = n * h
    a, b = rng.uniform(0.25, 0.45, size=2) * L
    theta = rng.uniform(0.0, math.pi)
    mask = ellipse_mask(g, a, b, theta)
    out = np.where(mask, eps, 1.0 + 0j).astype(np.complex128)
    return g, out


def inclusion_object(n: int = 2048, side: float = 25.6, seed: int = 5000, n_incl: int = 40,
                     semi=(12.0, 8.0), eps_host: complex = -3 + 0.1j) -> tuple[Grid, np.ndarray]:
    """Large stress scatterer: an ellipse of negative permittivity with circular inclusions.

    Inclusions: radius ~ U[0.3, 1], centre uniform in the ellipse, rejected unless
    the disc lies inside the ellipse and does not overlap an earlier one;
    eps ~ U[2, 20] + i U[0, 1].  ``semi`` is scaled with the domain when a
    smaller ``side`` is requested so that reduced versions keep the shape.
    """
    g = centred_grid(n, side)
    scale = side / 25.6
    a, b = semi[0] * scale, semi[1] * scale
    out = np.ones((g.ny, g.nx), dtype=np.complex128)
    out[ellipse_mask(g, a, b)] = eps_host
    rng = np.random.Generator(np.random.PCG64(seed))
    X, Y = cell_centres(g)
    placed: list[tuple[float, float, float]] = []
    tries = 0
    while len(placed) < n_incl and tries < 100_000:
        tries += 1
        r = rng.uniform(0.3, 1.0) * scale
        cx, cy = rng.uniform(-a, a), rng.uniform(-b, b)
        if (cx / a) ** 2 + (cy / b) ** 2 > 1.0:
            continue
        # the disc must fit in the ellipse: sample its rim
        t = np.linspace(0.0, 2.0 * math.pi, 64, endpoint=False)
        if np.any(((cx + r * np.cos(t)) / a) ** 2 + ((cy + r * np.sin(t)) / b) ** 2 > 1.0):
            continue
        if any((cx - px) ** 2 + (cy - py) ** 2 < (r + pr) ** 2 for px, py, pr in placed):
            continue
        placed.append((cx, cy, r))
        e = rng.uniform(2.0, 20.0) + 1j * rng.uniform(0.0, 1.0)
        out[(X - cx) ** 2 + (Y - cy) ** 2 <= r * r] = e
    return g, out


def sinusoid_object(n: int, side: float, a: float | None = None) -> tuple[Grid, np.ndarray]:
    """The paper's continuously varying object: eps = 10 + 5 sin(4 pi x/a) sin(4 pi y/a), with
    a the object's side (default: the grid's side)."""
    g = centred_grid(n, side)
    X, Y = cell_centres(g)
    a = side if a is None else a
    eps = 10.0 + 5.0 * np.sin(4.0 * math.pi * X / a) * np.sin(4.0 * math.pi * Y / a)
    return g, eps.astype(np.complex128)
