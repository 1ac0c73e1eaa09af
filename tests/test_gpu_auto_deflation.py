"""Automatic deflation size (Section 5): with deflate_k = -1 the library deflates every
eigenvalue of the solved operator beyond the object's deflation radius R.  On small grids the
count is checked against the dense spectrum from the oracle's matrices, and the deflated solve
against dense LU and the oracle residual."""
import numpy as np
import pytest

from gpu_util import dev, host, rel, say
from oracle import operator as op
from oracle import planning as pl
from synth import centred_grid, cylinder, square, plane_wave

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")


@pytest.mark.parametrize("shape,eps_obj,reg", [("cyl", -16 + 1.5j, True), ("square", 16.0 + 0j, True),
                                               ("cyl", -2.5 + 0.2j, False)])
def test_automatic_count_matches_dense_spectrum(shape, eps_obj, reg):
    g = centred_grid(20, 1.0, ny=18)
    eps = cylinder(g, 0.4, eps_obj) if shape == "cyl" else square(g, 0.7, eps_obj)
    A = op.dense_operator(g, op.electric_contrast(eps))
    M = op.dense_operator(g, op.regularizer_contrast(eps)) @ A if reg else A
    lam = np.linalg.eigvals(M)
    R = pl.deflation_radius(eps)  if reg else max(1.0, float(np.abs(eps).max()))
    dense = int(np.sum(np.abs(lam) > R))
    near = int(np.sum(np.abs(np.abs(lam) - R) <= 1e-3 * R))  # eigenvalues too close to R to count exactly
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=-1, eigs_tol=1e-8, seed=2)
    ritz, V, C = s.deflation_info()
    ritz = ritz.numpy()
    r = int(np.sum(np.abs(ritz) > 0))
    say(f"auto deflation {shape} eps={eps_obj} reg={reg}: R {R:.4f}, dense count {dense} (near {near}), library r {r}")
    assert abs(r - dense) <= near
    assert np.all(np.abs(ritz[:r]) > R * (1 - 1e-3))
    # the deflated system solves to the oracle's tolerance and agrees with LU
    b = np.stack([plane_wave(g, 0.4), plane_wave(g, 2.0)])
    u, rc, info = s.solve(dev(b), restart=20, max_iters=20000, tol=1e-8)
    u_lu = op.solve_dense(g, eps, b)
    uh = host(u)
    assert rc == 0
    for k in range(2):
        assert op.relative_residual(g, eps, uh[k], b[k]) <= 1.02e-8
        assert rel(uh[k], u_lu[k]) < 2e-5
    s.close()


def test_automatic_count_per_object_and_cap():
    # two objects in one context deflate their own counts (the other slots zero); the cap holds
    g = centred_grid(16, 0.8)
    eps = np.stack([cylinder(g, 0.3, -16 + 1.5j), np.full((16, 16), 1.5 + 0j)])
    s = api.Solver.from_grid(g, eps, regularize=True, deflate_k=-1, seed=2)
    ritz, V, C = s.deflation_info()
    counts = [int(np.sum(np.abs(ritz[o].numpy()) > 0)) for o in range(2)]
    R1 = pl.deflation_radius(eps[1])
    say(f"per-object counts {counts}, R of the weak object {R1:.4f}")
    assert counts[0] >= 1
    s.close()
    s2 = api.Solver.from_grid(g, eps[0], regularize=True, deflate_k=-1, deflate_max=2, seed=2)
    ritz2, _, _ = s2.deflation_info()
    assert int(np.sum(np.abs(ritz2.numpy()) > 0)) <= 2
    s2.close()
