"""GPU eigensolver and deflation projector against dense eigenvectors (oracle)."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, rand_c, say
from oracle import operator as op
from oracle import spectral as sp
from synth import centred_grid, square, cylinder

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")


@pytest.mark.parametrize("reg,eps_obj,r", [(False, -16 + 1.5j, 6), (True, -16 + 1.5j, 8), (True, 16.0 + 0j, 5)])
def test_deflation_basis_and_projector(reg, eps_obj, r):
    say(f"deflation reg={reg} eps={eps_obj} r={r}")
    g = centred_grid(10, 0.9, ny=8)
    eps = square(g, 0.6, eps_obj)
    A = op.dense_operator(g, op.electric_contrast(eps))
    M = op.dense_operator(g, op.regularizer_contrast(eps)) @ A if reg else A
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=r, eigs_tol=1e-10, seed=7)
    ritz, V, C = s.deflation_info()
    assert len(ritz) == r
    lam = np.linalg.eigvals(M)
    top = lam[np.argsort(-np.abs(lam))[:r]]
    for t in ritz.numpy():
        assert np.min(np.abs(top - t)) <= 1e-7 * abs(t)
    Vh = host(V).T  # columns
    assert np.abs(Vh.conj().T @ Vh - np.eye(r)).max() < 1e-12
    # invariant subspace: M V = V T to the eigensolver tolerance
    T = Vh.conj().T @ M @ Vh
    assert np.linalg.norm(M @ Vh - Vh @ T) <= 1e-8 * np.linalg.norm(M)
    np.testing.assert_allclose(C.numpy(), sp.deflation_terms(M, Vh), rtol=0, atol=1e-9 * np.abs(C.numpy()).max())
    # projector apply
    x = rand_c(np.random.default_rng(1), (2, 2 * g.n))
    got = host(s.apply_deflation(dev(x)))
    ref = sp.apply_deflation(Vh, C.numpy(), x.T).T
    assert rel(got, ref) < 1e-13
    # deflation moves r eigenvalues of M P^-1 to 1
    P = sp.deflation_preconditioner(M, Vh)
    mu = np.linalg.eigvals(M @ P)
    assert np.sum(np.abs(mu - 1) < 1e-6) >= r


def test_default_tolerance_ritz_values():
    g = centred_grid(16, 1.0)
    eps = cylinder(g, 0.4, -16 + 1.5j)
    r = 10
    s = api.Solver.from_grid(g, eps, regularize=True, deflate_k=r, seed=1)
    ritz, V, C = s.deflation_info()
    A = op.dense_operator(g, op.electric_contrast(eps))
    M = op.dense_operator(g, op.regularizer_contrast(eps)) @ A
    lam = np.linalg.eigvals(M)
    top = lam[np.argsort(-np.abs(lam))[:r]]
    for t in ritz.numpy():
        assert np.min(np.abs(top - t)) <= 1e-3 * abs(t)
