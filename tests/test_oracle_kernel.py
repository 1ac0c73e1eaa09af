"""Pins of the oracle's Green-tensor kernel against its defining operator.

The matrix elements of Section 4 (eq. A11 family) must be the midpoint-rule
sample of h^2 (k^2 I + grad grad) g, g = (i/4) H0(k|x|) (eq. MatrixSolutionTE,
eq. GreenFunction), and the self term must be the integral of that tensor
(with its delta part) over the disc of equal area, tending to the free term
-1/2 (eq. FreeTerms, s = 1 + chi/2).  These tests check the oracle's closed
forms against finite differences and quadrature of g alone.
"""
import math

import numpy as np
import pytest
from scipy.integrate import quad
from scipy.special import hankel1

from oracle import operator as op

K = 2.0 * math.pi


def g(x, y):
    return 0.25j * hankel1(0, K * np.hypot(x, y))


@pytest.mark.parametrize("x,y", [(0.13, 0.07), (0.4, -0.3), (-0.05, 0.21), (-0.9, -1.3), (0.02, 0.0)])
def test_offdiag_kernel_matches_finite_differences(x, y):
    h = 0.03
    d = 1e-4 if math.hypot(x, y) > 0.05 else 2e-5
    gxx = (g(x + d, y) - 2 * g(x, y) + g(x - d, y)) / d**2
    gyy = (g(x, y + d) - 2 * g(x, y) + g(x, y - d)) / d**2
    gxy = (g(x + d, y + d) - g(x + d, y - d) - g(x - d, y + d) + g(x - d, y - d)) / (4 * d * d)
    ref = np.array([K * K * g(x, y) + gxx, gxy, K * K * g(x, y) + gyy]) * h * h
    got = np.array(op.kernel_offdiag(x, y, h, K))
    assert np.all(np.abs(got - ref) <= 2e-6 * np.abs(ref).max())


def test_offdiag_kernel_symmetries():
    h = 0.02
    for x, y in [(0.1, 0.3), (-0.7, 0.2)]:
        a = np.array(op.kernel_offdiag(x, y, h, K))
        b = np.array(op.kernel_offdiag(-x, -y, h, K))
        c = np.array(op.kernel_offdiag(-x, y, h, K))
        np.testing.assert_allclose(a, b, rtol=1e-15)  # T(-d) = T(d)
        np.testing.assert_allclose(c, a * np.array([1, -1, 1]), rtol=1e-14)  # T12 odd in x
        s = np.array(op.kernel_offdiag(y, x, h, K))
        np.testing.assert_allclose(s, a[::-1], rtol=1e-14)  # swapping axes swaps T11/T22


@pytest.mark.parametrize("h", [0.3, 0.05, 1.2 / 64, 1e-3])
def test_self_term_is_disc_integral_of_green_tensor(h):
    """T(0) = k^2 int_disc g + oint_{|x|=a} n_b d_a g ds (divergence theorem gives the
    distributional grad-grad part, delta included), a = h / sqrt(pi)."""
    a = h / math.sqrt(math.pi)
    re = quad(lambda r: (0.25j * hankel1(0, K * r) * 2 * math.pi * r).real, 0, a, limit=200)[0]
    im = quad(lambda r: (0.25j * hankel1(0, K * r) * 2 * math.pi * r).imag, 0, a, limit=200)[0]
    vol = K * K * (re + 1j * im)
    # boundary term for the (1,1) entry: oint n_1 d_1 g ds, d_1 g by central differences
    d = 1e-6 * a
    nt = 256
    th = (np.arange(nt) + 0.5) * 2 * math.pi / nt
    px, py = a * np.cos(th), a * np.sin(th)
    d1g = (g(px + d, py) - g(px - d, py)) / (2 * d)
    bnd = np.sum(np.cos(th) * d1g) * a * 2 * math.pi / nt
    assert abs(op.kernel_self(h, K) - (vol + bnd)) < 1e-7


def test_self_term_free_term_limit():
    # diagonal element 1 - T(0) chi -> 1 + chi/2 as h -> 0
    for h, tol in [(1e-3, 1e-4), (1e-5, 1e-8)]:
        assert abs(op.kernel_self(h, K) + 0.5) < tol


def test_lag_table_layout():
    nx, ny, h = 5, 3, 0.07
    lag = op.lag_table(nx, ny, h, K)
    assert lag.shape == (3, 2 * ny - 1, 2 * nx - 1)
    assert lag[0, ny - 1, nx - 1] == op.kernel_self(h, K)
    assert lag[1, ny - 1, nx - 1] == 0
    t = op.kernel_offdiag(2 * h, -1 * h, h, K)
    for i in range(3):
        assert lag[i, -1 + ny - 1, 2 + nx - 1] == t[i]
