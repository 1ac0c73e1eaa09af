"""Pins of the oracle's spectral pieces: the exact homogeneous-object identity
behind eq. EigenvaluesArA, the lossless segment image, the essential-spectrum
segment, and the deflation properties of eq. DeflatingPrecondtioner."""
import math

import numpy as np
import pytest

from oracle import operator as op
from oracle import spectral as sp
from synth import centred_grid, square


def homogeneous(n, eps):
    g = centred_grid(n, 0.9)
    e = np.full((n, n), eps, dtype=complex)
    return g, op.dense_operator(g, op.electric_contrast(e)), op.dense_operator(g, op.regularizer_contrast(e))


@pytest.mark.parametrize("eps", [4.0, 16.0, -16 + 1.5j, -2.5 + 0.2j])
def test_homogeneous_regularized_matrix_identity(eps):
    # A = I - chi T, A_R = I - chi' T with chi' = -chi/eps  =>  A_R A = A + (1/eps)(I - A) A
    g, A, AR = homogeneous(6, eps)
    I = np.eye(A.shape[0])
    lhs = AR @ A
    rhs = A + (I - A) @ A / eps
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(lhs).max()


@pytest.mark.parametrize("eps", [4.0, -16 + 1.5j])
def test_homogeneous_eigenvalue_map(eps):
    g, A, AR = homogeneous(7, eps)
    lam = np.linalg.eigvals(A)
    mapped = sp.homogeneous_map(lam, eps)
    lam_r = np.linalg.eigvals(AR @ A)
    # every eigenvalue of A_R A is the image of one of A (matched greedily)
    d = np.abs(lam_r[:, None] - mapped[None, :]).min(axis=1)
    assert d.max() <= 1e-10 * np.abs(lam_r).max()


@pytest.mark.parametrize("eps", [4.0, 16.0, 2.0])
def test_lossless_segment_image(eps):
    t = np.linspace(1.0, eps, 200001)
    f = sp.homogeneous_map(t, eps).real
    lo, hi = sp.lossless_segment_image(eps)
    assert abs(f.max() - hi) < 1e-8 * hi and abs(f.min() - lo) < 1e-12


def test_segment_distance():
    assert abs(sp.segment_distance_to_origin(1, 4) - 1.0) < 1e-15
    assert abs(sp.segment_distance_to_origin(1, -1) - 0.0) < 1e-15
    # -2.5+0.2i: distance |Im eps| / |eps - 1| from the line through 1
    e = -2.5 + 0.2j
    assert abs(sp.segment_distance_to_origin(1, e) - 0.2 / abs(e - 1)) < 1e-15


@pytest.mark.parametrize("eps", [-2.5 + 0.2j, -16 + 1.5j])
def test_essential_spectrum_segment(eps):
    g, A, AR = homogeneous(20, eps)
    lam = np.linalg.eigvals(A)
    a, b = sp.essential_segment(eps)
    d = b - a
    t = np.clip((np.conj(d) * (lam - a)).real / abs(d) ** 2, 0, 1)
    dist = np.abs(lam - (a + t * d))
    assert np.mean(dist < 0.05 * abs(d)) > 0.85
    # negative permittivity: the segment passes near 0 and so does the spectrum of A and A_R
    d0 = sp.segment_distance_to_origin(1, eps)
    assert abs(np.abs(lam).min() / d0 - 1) < 0.15
    d0r = sp.segment_distance_to_origin(1, 1 / eps)
    assert abs(np.abs(np.linalg.eigvals(AR)).min() / d0r - 1) < 0.05


def test_deflation_moves_r_eigenvalues_to_one():
    g = centred_grid(8, 0.8)
    eps = square(g, 0.5, -16 + 1.5j)
    A = op.dense_operator(g, op.electric_contrast(eps))
    r = 6
    lam, X = sp.largest_eigvecs(A, r)
    V = sp.modified_gram_schmidt(X)
    assert np.abs(V.conj().T @ V - np.eye(r)).max() < 1e-12
    Pinv = sp.deflation_preconditioner(A, V)
    mu = np.linalg.eigvals(A @ Pinv)
    all_lam = np.linalg.eigvals(A)
    keep = np.argsort(-np.abs(all_lam))[r:]
    # r eigenvalues at 1, the rest unchanged
    n_one = np.sum(np.abs(mu - 1) < 1e-8)
    assert n_one >= r
    rest = all_lam[keep]
    dist = np.abs(rest[:, None] - mu[None, :]).min(axis=1)
    assert dist.max() < 1e-8 * np.abs(all_lam).max()


def test_deflation_invariant_to_basis():
    g = centred_grid(6, 0.6)
    eps = square(g, 0.4, 9.0 + 0j)
    A = op.dense_operator(g, op.electric_contrast(eps))
    lam, X = sp.largest_eigvecs(A, 4)
    V = sp.modified_gram_schmidt(X)
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
    P1 = sp.deflation_preconditioner(A, V)
    P2 = sp.deflation_preconditioner(A, V @ Q)
    assert np.abs(P1 - P2).max() < 1e-10
    x = rng.standard_normal(A.shape[0]) + 0j
    C = sp.deflation_terms(A, V)
    np.testing.assert_allclose(sp.apply_deflation(V, C, x), P1 @ x, rtol=1e-12, atol=1e-12)
