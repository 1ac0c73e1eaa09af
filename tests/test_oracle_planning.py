"""Pins of the oracle's deflation-size and memory-planning steps (Section 5):

* the paper's worked example of the systematic application: M = 4 GB (2^32 bytes),
  beta = 0.0011, 15 points per wavelength, restart = 8 r and eps = 10 + 5 sin sin give
  [a/lambda]_max = 4 (4.006 before rounding), 3N = 162867 unknowns (233^2 nodes), r = 180 and
  restarts 1440 (preconditioned) and 1620 (unpreconditioned, fair memory);
* the memory identity the planner solves: M_A + M_prec at N_max equals M;
* the deflation radius of a lossless segment against the closed form the paper states for it,
  1 + (1 - eps)^2 / (4 eps), and of a background cell (eps = 1) against 1;
* the deflation radius against brute force: the largest |lam'| of the mapped dense
  spectrum of a homogeneous object's A lies within the radius (up to discretisation), and
  the radius of an inhomogeneous object is the largest of its segments'.
"""
import math

import numpy as np
import pytest

from oracle import operator as op
from oracle import planning as pl
from oracle import spectral as sp
from synth import centred_grid, cylinder


def test_worked_example_of_section5():
    p = pl.plan_memory(float(2 ** 32), 0.0011, 15.0, 8.0, 15.0)
    assert abs(p["a_over_lambda_max"] - 4.006) < 5e-4
    assert round(p["a_over_lambda_max"]) == 4
    assert p["nodes"] == 233
    assert p["unknowns"] == 162867
    assert p["r"] == 180
    assert p["restart"] == 1440
    assert p["restart_unpreconditioned"] == 1620


def test_planner_solves_the_memory_budget():
    M, beta, x = 3.0e9, 0.002, 4.0
    p = pl.plan_memory(M, beta, 15.0, x, 12.0)
    n = p["n_max"]
    r = 3 * n * beta
    total = 720.0 * n + 16 * r * r + 48 * n * r + 48 * n * x * r
    assert abs(total - M) <= 1e-9 * M


def test_fair_memory_rule_matches_table2():
    # Table 2: restart + r = 40 for every system
    for r, restart in ((6, 34), (14, 26), (7, 33), (30, 10), (3, 37)):
        assert pl.fair_restart(restart, r) == 40


@pytest.mark.parametrize("eps", [4.0, 10.0, 16.0, 20.0])
def test_lossless_segment_radius_closed_form(eps):
    R = pl.segment_image_radius(eps, samples=20001)
    assert abs(R - (1.0 + (1.0 - eps) ** 2 / (4.0 * eps))) <= 1e-7 * R
    assert abs(R - sp.lossless_segment_image(eps)[1]) <= 1e-7 * R


def test_background_cell_radius_is_one():
    assert pl.segment_image_radius(1.0 + 0j) == 1.0


def test_radius_of_inhomogeneous_object_is_largest_segment():
    cells = np.array([1.0, 4.0, -16 + 1.5j, 2.5 + 20j, 16.0])
    R = pl.deflation_radius(cells)
    assert R == max(pl.segment_image_radius(e) for e in cells)
    assert R == pl.segment_image_radius(2.5 + 20j)


@pytest.mark.parametrize("eps", [16.0, -16 + 1.5j])
def test_mapped_dense_spectrum_inside_radius(eps):
    # homogeneous object: the eigenvalues of A_R A are the images of those of A (exact), and
    # those of A cluster along [1, eps]; the dense cluster of A_R A lies inside R while
    # outliers (discrete eigenvalues off the segment) may lie outside -- they are what gets
    # deflated.  Most eigenvalues (the dense cluster) must be within R.
    g = centred_grid(8, 0.8)
    e = np.full((8, 8), eps, dtype=complex)
    A = op.dense_operator(g, op.electric_contrast(e))
    lam = np.linalg.eigvals(A)
    lam_r = sp.homogeneous_map(lam, eps)
    R = pl.deflation_radius(e)
    inside = np.mean(np.abs(lam_r) <= R * 1.05)
    assert inside >= 0.8
    # and R is attained by the image of the segment itself
    t = np.linspace(0, 1, 4001)
    img = sp.homogeneous_map(1 + t * (eps - 1), eps)
    assert abs(np.abs(img).max() - R) <= 1e-12 * R
