"""The oracle's three forms of y = A x agree: pure loops over cells (brute
force), the dense element-by-element matrix, the block-Toeplitz direct sum,
and the per-output sampled sum -- on non-square, odd and degenerate grids."""
import math

import numpy as np
import pytest

from oracle import operator as op
from synth import centred_grid, Grid


def rand_c(rng, shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


@pytest.mark.parametrize("nx,ny", [(4, 3), (1, 1), (1, 5), (6, 1), (3, 7)])
def test_all_forms_agree(nx, ny):
    rng = np.random.default_rng(nx * 10 + ny)
    g = centred_grid(nx, 0.05 * nx, ny=ny)
    chi = rand_c(rng, (ny, nx))
    x = rand_c(rng, (2, ny, nx))
    y_loop = op.apply_operator_loops(g, chi, x)
    y_dense = (op.dense_operator(g, chi) @ x.reshape(-1)).reshape(x.shape)
    y_sum = op.apply_operator(g, chi, x)
    scale = np.abs(y_loop).max()
    assert np.abs(y_dense - y_loop).max() <= 1e-13 * scale
    assert np.abs(y_sum - y_loop).max() <= 1e-13 * scale
    samples = [(c, iy, ix) for c in range(2) for iy in range(ny) for ix in range(nx)]
    y_at = op.apply_operator_at(g, chi, x, samples)
    assert np.abs(y_at - y_loop.reshape(-1)).max() <= 1e-13 * scale


def test_direct_sum_batched_and_larger():
    rng = np.random.default_rng(7)
    g = centred_grid(13, 0.4, ny=9)
    chi = rand_c(rng, (9, 13))
    X = rand_c(rng, (3, 2, 9, 13))
    A = op.dense_operator(g, chi)
    Y = op.apply_operator(g, chi, X)
    for r in range(3):
        ref = (A @ X[r].reshape(-1)).reshape(2, 9, 13)
        assert np.abs(Y[r] - ref).max() <= 1e-13 * np.abs(ref).max()


def test_zero_contrast_is_identity():
    g = centred_grid(5, 0.3)
    x = rand_c(np.random.default_rng(1), (2, 5, 5))
    np.testing.assert_array_equal(op.apply_operator(g, np.zeros((5, 5)), x), x)


def test_existence_condition():
    eps = np.ones((3, 3), dtype=complex)
    eps[1, 2] = 0
    with pytest.raises(op.SingularContrastError):
        op.electric_contrast(eps)
    with pytest.raises(op.SingularContrastError):
        op.regularizer_contrast(eps)


def test_contrasts():
    eps = np.array([[4.0, -2.5 + 0.2j]])
    np.testing.assert_allclose(op.electric_contrast(eps), [[3.0, -3.5 + 0.2j]])
    np.testing.assert_allclose(op.regularizer_contrast(eps), 1 / eps - 1)
    # the symbol of A(chi') inverts that of A(chi): (1 + chi q)(1 + chi' q) = 1 on the range of the projector
    chi, chir = op.electric_contrast(eps), op.regularizer_contrast(eps)
    np.testing.assert_allclose((1 + chi) * (1 + chir), 1.0, rtol=1e-15)
