"""Pins of the TM operator and the full three-component TE system (oracle/systems.py):

* the Green function's normalisation (flux of grad g through a small circle is -1) and the
  TM self term against quadrature of the disc integral of g;
* the coupling kernels against finite differences of g (K13 = -i omega mu_b d2 g,
  K23 = i omega mu_b d1 g, K31 = -i omega eps_b d2 g, K32 = i omega eps_b d1 g, Section 3);
* direct sums against the dense matrices;
* structure: with chi_m = 0 the E-block of the 3N matrix is the 2N operator and H3 follows
  from E by post-processing; with chi_e = 0 the H3 block is the TM operator with chi_m
  (duality); reciprocity (X A^-1 symmetric for TM; D X A^-1 with D = diag(1, 1, -1) for the
  mixed electric-magnetic system);
* the discrete solutions against the series for a homogeneous cylinder (TM; TE with magnetic
  contrast), loose because of the staircased boundary, and decreasing with h;
* the series themselves: interface conditions and the plane wave for eps = mu = 1.
"""
import math

import numpy as np
import pytest
from scipy import integrate
from scipy.special import hankel1

from oracle import mie
from oracle import operator as op
from oracle import systems as sy
from synth import centred_grid, cylinder, cell_centres, plane_wave

K = 2 * math.pi


def test_green_function_flux_normalisation():
    # (Laplacian + k^2) g = -delta: the flux of grad g out of a small circle tends to -1
    r = 1e-7
    dgdr = 0.25j * (-K * hankel1(1, K * r))
    assert abs(2 * math.pi * r * dgdr - (-1.0)) < 1e-6


@pytest.mark.parametrize("h", [0.05, 0.01, 1e-3])
def test_tm_self_term_is_disc_integral(h):
    a = h / math.sqrt(math.pi)
    f = lambda r, part: getattr(2 * math.pi * r * 0.25j * hankel1(0, K * r), part)
    re = integrate.quad(f, 0, a, args=("real",), limit=200)[0]
    im = integrate.quad(f, 0, a, args=("imag",), limit=200, points=[0])[0]
    assert abs(K * K * (re + 1j * im) - sy.tm_kernel_self(h, K)) < 1e-9


def _fd(fun, x, y, s=1e-5):
    return (fun(x + s, y) - fun(x - s, y)) / (2 * s), (fun(x, y + s) - fun(x, y - s)) / (2 * s)


@pytest.mark.parametrize("dx,dy", [(0.13, 0.02), (-0.07, 0.21), (0.3, -0.25), (0.0, 0.11)])
def test_coupling_kernels_against_finite_differences(dx, dy):
    h = 0.02
    g = lambda x, y: 0.25j * hankel1(0, K * np.hypot(x, y))
    d1g, d2g = _fd(g, dx, dy)
    t13, t23, t31, t32 = sy.cross_kernels(dx, dy, h, K)
    # A = I - T X and the matrix element is h^2 K chi: T = -h^2 K
    assert abs(t13 - (-h * h) * (-1j * K * d2g)) < 1e-8 * abs(t13)
    assert abs(t23 - (-h * h) * (1j * K * d1g)) < 1e-8 * max(abs(t23), 1e-30) or abs(t23) < 1e-12
    assert abs(t31 - (-h * h) * (-1j * K * d2g)) < 1e-8 * abs(t31)
    assert abs(t32 - (-h * h) * (1j * K * d1g)) < 1e-8 * max(abs(t32), 1e-30) or abs(t32) < 1e-12
    assert abs(sy.tm_kernel_offdiag(dx, dy, h, K) - K * K * h * h * g(dx, dy)) < 1e-14


def _rand_grid(rng, nx=7, ny=5):
    g = centred_grid(nx, 0.35, ny=ny)
    ce = rng.standard_normal((ny, nx)) + 1j * rng.random((ny, nx))
    cm = rng.standard_normal((ny, nx)) + 1j * rng.random((ny, nx))
    return g, ce, cm


def test_direct_sums_equal_dense_matrices():
    rng = np.random.default_rng(1)
    g, ce, cm = _rand_grid(rng)
    x3 = rng.standard_normal((3, g.ny, g.nx)) + 1j * rng.standard_normal((3, g.ny, g.nx))
    A3 = sy.dense_operator_full(g, ce, cm)
    y = sy.apply_operator_full(g, ce, cm, x3)
    assert np.abs(y.ravel() - A3 @ x3.ravel()).max() <= 1e-13 * np.abs(y).max()
    x1 = x3[0]
    A1 = sy.dense_operator_tm(g, ce)
    assert np.abs(sy.apply_operator_tm(g, ce, x1).ravel() - A1 @ x1.ravel()).max() <= 1e-13 * np.abs(A1 @ x1.ravel()).max()


def test_structure_without_magnetic_contrast_and_duality():
    rng = np.random.default_rng(2)
    g, ce, cm = _rand_grid(rng)
    N = g.n
    A3 = sy.dense_operator_full(g, ce, np.zeros_like(cm))
    A2 = op.dense_operator(g, ce)
    assert np.abs(A3[:2 * N, :2 * N] - A2).max() == 0.0
    # the H3 column blocks are the identity: H3 does not feed back, it is post-processing
    assert np.abs(A3[:, 2 * N:] - np.eye(3 * N)[:, 2 * N:]).max() == 0.0
    # duality: no electric contrast leaves the H3 block as the TM operator with chi_m
    A3m = sy.dense_operator_full(g, np.zeros_like(ce), cm)
    assert np.abs(A3m[2 * N:, 2 * N:] - sy.dense_operator_tm(g, cm)).max() == 0.0


def test_reciprocity_of_both_systems():
    rng = np.random.default_rng(3)
    g, ce, cm = _rand_grid(rng)
    N = g.n
    A3 = sy.dense_operator_full(g, ce, cm)
    X3 = np.diag(np.concatenate([ce.ravel(), ce.ravel(), cm.ravel()]))
    # the coupling kernels are odd in the separation (T13 = -T31^T as matrices), so reciprocity
    # between electric and magnetic sources carries a sign: D X A^-1 is symmetric, D = diag(1, 1, -1)
    D = np.diag(np.concatenate([np.ones(2 * N), -np.ones(N)]))
    S = D @ X3 @ np.linalg.inv(A3)
    assert np.abs(S - S.T).max() <= 1e-12 * np.abs(S).max()
    assert np.abs(X3 @ np.linalg.inv(A3) - (X3 @ np.linalg.inv(A3)).T).max() > 1e-3  # without D it is not
    A1 = sy.dense_operator_tm(g, ce)
    S1 = np.diag(ce.ravel()) @ np.linalg.inv(A1)
    assert np.abs(S1 - S1.T).max() <= 1e-12 * np.abs(S1).max()


def test_series_interface_conditions_and_plane_wave():
    for pol, eps, mu in (("tm", 4.0, 1.0), ("tm", -2.5 + 0.2j, 1.3), ("te", 3.0 + 0.2j, 2.0 + 0.1j)):
        j0, j1 = mie.interface_jumps(K, 0.5, eps, mu, 0.4, pol)
        assert j0 < 1e-4 and j1 < 1e-4, (pol, eps, mu, j0, j1)
    x, y = np.meshgrid(np.linspace(-0.6, 0.6, 7), np.linspace(-0.6, 0.6, 7))
    pw = np.exp(1j * K * (x * math.cos(0.4) + y * math.sin(0.4)))
    assert np.abs(mie.tm_field(x, y, K, 0.3, 1.0, 1.0, 0.4) - pw).max() < 1e-10
    te = mie.te_fields(x, y, K, 0.3, 1.0, 1.0, 0.4)
    assert np.abs(te[2] - pw).max() < 1e-10
    # mu = 1 reproduces the TE electric field of the dielectric series
    assert np.abs(mie.te_fields(x, y, K, 0.3, 4.0, 1.0, 0.4)[:2] - mie.total_field(x, y, K, 0.3, 4.0, 0.4)).max() < 1e-10


def _equal_area_radius(g, obj):
    """Radius of the circle with the area of the staircased object (its cells' total area)."""
    return math.sqrt(float(np.sum(obj)) * g.h * g.h / math.pi)


def _tm_error(n, eps_obj=4.0 + 1.0j, radius=0.4):
    g = centred_grid(n, 1.0)
    eps = cylinder(g, radius, eps_obj)
    u = sy.solve_dense_tm(g, eps, sy.plane_wave_tm(g, 0.3))
    X, Y = cell_centres(g)
    E = mie.tm_field(X, Y, K, _equal_area_radius(g, eps != 1), eps_obj, 1.0, 0.3)
    return np.linalg.norm(u - E) / np.linalg.norm(E)


def test_tm_solution_against_series():
    # staircased lossy cylinder against the series of the cylinder of equal area
    errs = [_tm_error(n) for n in (16, 32, 48)]
    assert errs[2] < 0.02 and errs[0] > 3 * errs[2], errs


def _full_error(n):
    g = centred_grid(n, 1.2)
    eps, mu = cylinder(g, 0.45, 2.5 + 0.1j), cylinder(g, 0.45, 1.8)
    E2 = plane_wave(g, 0.3)
    b = np.stack([E2[0], E2[1], E2[1] / math.cos(0.3)])  # H3_in = E2_in / cos(psi)
    u = sy.solve_dense_full(g, eps, mu, b)
    X, Y = cell_centres(g)
    ref = mie.te_fields(X, Y, K, _equal_area_radius(g, eps != 1), 2.5 + 0.1j, 1.8, 0.3)
    errE = np.linalg.norm(u[:2] - ref[:2]) / np.linalg.norm(ref[:2])
    errH = np.linalg.norm(u[2] - ref[2]) / np.linalg.norm(ref[2])
    return errE, errH, g, eps, mu, b, u


@pytest.mark.slow
def test_full_system_against_series_with_magnetic_contrast():
    e24, h24, *_ = _full_error(24)
    e48, h48, g, eps, mu, b, u = _full_error(48)
    assert e48 < 0.06 and h48 < 0.06 and e24 > e48 and h24 > h48, (e24, h24, e48, h48)
    # without the magnetic contrast the field differs markedly (the H3 coupling is live)
    u0 = sy.solve_dense_full(g, eps, np.ones_like(mu), b)
    assert np.linalg.norm(u0[2] - u[2]) / np.linalg.norm(u[2]) > 0.05


def test_post_processing_of_h3_without_magnetic_contrast():
    g = centred_grid(20, 1.0)
    eps = cylinder(g, 0.35, 4.0 + 0.5j)
    E2 = plane_wave(g, 0.7)
    H3in = E2[1] / math.cos(0.7)
    u3 = sy.solve_dense_full(g, eps, np.ones_like(eps), np.stack([E2[0], E2[1], H3in]))
    u2 = op.solve_dense(g, eps, E2)
    assert np.abs(u3[:2] - u2).max() <= 1e-12 * np.abs(u2).max()
    # H3 = H3_in + row 3 of T applied to chi_e E (one product of the full operator)
    chi = eps - 1.0
    y = sy.apply_operator_full(g, chi, np.zeros_like(chi), np.stack([u2[0], u2[1], np.zeros_like(H3in)]))
    H3 = H3in - y[2]
    assert np.abs(H3 - u3[2]).max() <= 1e-11 * np.abs(H3).max()
