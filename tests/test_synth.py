"""The seeded input generators: determinism, shapes, value ranges."""
import math

import numpy as np

from synth import (centred_grid, cylinder, plane_wave, random_field_object, inclusion_object,
                   gaussian_random_field, workload, cell_centres)


def test_grid_and_cylinder():
    g = centred_grid(64, 1.2)
    assert abs(g.h - 1.2 / 64) < 1e-15 and abs(g.x0 + 0.6) < 1e-15
    X, Y = cell_centres(g)
    assert abs(X[0, 0] - (-0.6 + 0.5 * g.h)) < 1e-15 and X.shape == (64, 64)
    e = cylinder(g, 0.5, 4.0)
    assert set(np.unique(e)) <= {1.0, 4.0}
    # staircase area close to pi R^2
    assert abs((e == 4).sum() * g.h**2 - math.pi * 0.25) < 0.02


def test_plane_wave_transverse_unit():
    g = centred_grid(8, 1.0)
    for psi in (0.0, 0.7, math.pi / 6):
        b = plane_wave(g, psi)
        assert b.shape == (2, 8, 8) and b.dtype == np.complex128
        kd = np.array([math.cos(psi), math.sin(psi)])
        assert np.abs(kd[0] * b[0] + kd[1] * b[1]).max() < 1e-15  # transverse to propagation
        assert np.allclose(np.abs(b[0]) ** 2 + np.abs(b[1]) ** 2, 1.0)


def test_random_field_deterministic_and_ranges():
    g1, e1 = random_field_object(128, seed=1000)
    g2, e2 = random_field_object(128, seed=1000)
    np.testing.assert_array_equal(e1, e2)
    _, e3 = random_field_object(128, seed=1001)
    assert not np.array_equal(e1, e3)
    inside = e1 != 1.0
    assert 0.1 < inside.mean() < 0.7
    assert e1.real.min() >= 1.0 and e1.real.max() <= 10.0
    assert e1.imag.min() >= 0.0 and e1.imag.max() <= 0.5
    z = gaussian_random_field(64, 1 / 48, 0.5, 3)
    assert abs(z.std() - 1) < 1e-12 and abs(z.mean()) < 1e-12


def test_inclusion_object_small():
    g, e = inclusion_object(n=256, side=25.6 / 4, n_incl=10)
    assert e.shape == (256, 256)
    host = np.isclose(e, -3 + 0.1j)
    assert host.sum() > 0 and np.any((e.real >= 2) & (e.real <= 20))


def test_workloads_build():
    w = workload("cyl_small")
    assert w["grids"][0].nx == 64 and w["restart"] == 20
    w = workload("cyl_hard")
    assert abs(w["psi"][0] - math.pi / 6) < 1e-15 and w["deflate_k"] == 20
