"""Pins of the oracle's dense solution: the Mie series for a circular
cylinder (discretisation-limited), the quasi-static depolarisation limit,
reciprocity and the discrete optical theorem (exact invariants of A = I - T X
with T symmetric)."""
import math

import numpy as np
import pytest

from oracle import operator as op
from oracle import mie
from synth import centred_grid, cylinder, plane_wave, cell_centres, square

K = 2.0 * math.pi


def test_mie_incident_series_is_the_plane_wave():
    X, Y = np.meshgrid(np.linspace(-0.9, 0.7, 9), np.linspace(-0.6, 0.8, 8))
    for psi in (0.0, 0.3, 2.0):
        ref = np.stack([-math.sin(psi), math.cos(psi)])[:, None, None] * np.exp(
            1j * K * (X * math.cos(psi) + Y * math.sin(psi)))
        assert np.abs(mie.incident_field(X, Y, K, psi) - ref).max() < 1e-12


def test_mie_no_contrast_gives_incident_field():
    n, a, c = mie.coefficients(K, 0.5, 1.0 + 0j, 10)
    assert np.abs(a).max() < 1e-14 and np.abs(c - 1).max() < 1e-14


def test_mie_interface_conditions():
    # H3 and (1/eps) dH3/dr continuous: checked through tangential E just inside/outside
    R, eps = 0.5, 4.0 - 0.3j
    th = np.linspace(0, 2 * math.pi, 13)
    eo = mie.total_field((R + 1e-7) * np.cos(th), (R + 1e-7) * np.sin(th), K, R, eps, 0.4)
    ei = mie.total_field((R - 1e-7) * np.cos(th), (R - 1e-7) * np.sin(th), K, R, eps, 0.4)
    et_o = -np.sin(th) * eo[0] + np.cos(th) * eo[1]
    et_i = -np.sin(th) * ei[0] + np.cos(th) * ei[1]
    dn_o = np.cos(th) * eo[0] + np.sin(th) * eo[1]
    dn_i = np.cos(th) * ei[0] + np.sin(th) * ei[1]
    assert np.abs(et_o - et_i).max() < 1e-5
    assert np.abs(dn_o - eps * dn_i).max() < 1e-5  # normal D continuous


@pytest.mark.slow
def test_dense_solution_converges_to_mie_series():
    errs, errs_off = [], []
    for n in (24, 32):
        g = centred_grid(n, 1.2)
        eps = cylinder(g, 0.5, 4.0 + 0j)
        u = op.solve_dense(g, eps, plane_wave(g, 0.0))
        X, Y = cell_centres(g)
        E = mie.total_field(X, Y, K, 0.5, 4.0, 0.0)
        errs.append(np.linalg.norm(u - E) / np.linalg.norm(E))
        band = np.abs(np.hypot(X, Y) - 0.5) > 3 * g.h
        errs_off.append(np.linalg.norm((u - E)[:, band]) / np.linalg.norm(E[:, band]))
    # staircase-limited agreement that improves with refinement
    assert errs[0] < 0.15 and errs[1] < 0.11 and errs[1] < errs[0]
    assert errs_off[0] < 0.10 and errs_off[1] < 0.075 and errs_off[1] < errs_off[0]


def test_quasi_static_limit():
    # a cylinder much smaller than the wavelength sees a uniform interior field 2 E0 / (1 + eps)
    g = centred_grid(16, 0.02)
    eps = cylinder(g, 0.008, 4.0 + 0j)
    u = op.solve_dense(g, eps, plane_wave(g, 0.0))
    X, Y = cell_centres(g)
    inside = np.hypot(X, Y) <= 0.008
    assert abs(u[1][inside].mean() - 2.0 / 5.0) < 0.01
    assert abs(u[0][inside].mean()) < 1e-3  # staircase corners add local E1 that averages out


@pytest.mark.parametrize("eps_obj", [4.0 + 0j, -2.5 + 0.2j, 16.0 + 0j])
def test_reciprocity(eps_obj):
    g = centred_grid(12, 1.0, ny=10)
    eps = square(g, 0.6, eps_obj)
    chi = op.electric_contrast(eps)
    A = op.dense_operator(g, chi)
    solve = op.lu_solver(A)
    b1, b2 = plane_wave(g, 0.2).reshape(-1), plane_wave(g, 1.9).reshape(-1)
    u1, u2 = solve(b1), solve(b2)
    x = np.concatenate([chi.reshape(-1)] * 2)
    lhs, rhs = b1 @ (x * u2), b2 @ (x * u1)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_discrete_optical_theorem_lossless():
    g = centred_grid(10, 0.8)
    eps = cylinder(g, 0.3, 9.0 + 0j)
    chi = op.electric_contrast(eps)
    T = np.eye(2 * g.n) - op.dense_operator(g, np.ones((g.ny, g.nx)))
    b = plane_wave(g, 0.7).reshape(-1)
    u = op.lu_solver(op.dense_operator(g, chi))(b)
    q = np.concatenate([chi.reshape(-1)] * 2) * u
    lhs = -np.imag(np.vdot(q, b))
    rhs = np.real(np.vdot(q, T.imag @ q))
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)
    assert rhs > 0  # extinction is positive: the scatterer only removes power


def test_dense_solution_residual_tiny():
    g = centred_grid(9, 0.5, ny=7)
    eps = cylinder(g, 0.2, -2.5 + 0.2j)
    b = plane_wave(g, 0.5)
    u = op.solve_dense(g, eps, b)
    assert op.relative_residual(g, eps, u, b) < 1e-13
