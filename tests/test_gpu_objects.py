"""Contexts holding several objects on one grid (each object the collocation system
of Section 4; solving many of them in the same launches is the library's batching,
not the paper's): every product, projector and solve of a multi-object context must
equal the same call on one-object contexts, and the products must equal the
oracle's direct sum."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, rand_c, say
from oracle import operator as op
from synth import centred_grid, cylinder, square, plane_wave

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")
from paper_1104_4263_amd._lib import DieTeError  # noqa: E402


def objects(g):
    """Three different scatterers on one grid: a dielectric cylinder, a plasmonic
    cylinder and a lossy square."""
    return np.stack([cylinder(g, 0.35, 4.0 + 0j), cylinder(g, 0.3, -2.5 + 0.2j), square(g, 0.5, 6.0 + 1.0j)])


def fields(g, psis):
    return np.stack([plane_wave(g, p) for p in psis])


@pytest.mark.parametrize("nx,ny", [(24, 20), (37, 11)])
@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_products_match_single_object_and_oracle(nx, ny, dtype):
    say(f"multi-object products {nx}x{ny} {dtype}")
    g = centred_grid(nx, 1.0, ny=ny)
    eps = objects(g)
    nobj, per = eps.shape[0], 3
    rng = np.random.default_rng(7)
    x = rand_c(rng, (nobj * per, 2, ny, nx))
    multi = api.Solver.from_grid(g, eps)
    xd = dev(x, dtype)
    ym, yrm = host(multi.matvec(xd)), host(multi.regularize(xd))
    tol = 1e-12 if dtype == torch.complex128 else 2e-6
    for o in range(nobj):
        one = api.Solver.from_grid(g, eps[o])
        sl = slice(o * per, (o + 1) * per)
        ys, yrs = host(one.matvec(dev(x[sl], dtype))), host(one.regularize(dev(x[sl], dtype)))
        assert np.array_equal(ym[sl], ys) and np.array_equal(yrm[sl], yrs)
        for r in range(per):
            xr = x[o * per + r].astype(np.complex64).astype(np.complex128) if dtype == torch.complex64 else x[o * per + r]
            ref = op.apply_operator(g, op.electric_contrast(eps[o]), xr)
            refr = op.apply_operator(g, op.regularizer_contrast(eps[o]), xr)
            assert rel(ym[o * per + r], ref) < tol
            assert rel(yrm[o * per + r], refr) < tol


def test_nrhs_must_be_a_multiple_of_nobj():
    g = centred_grid(12, 1.0)
    multi = api.Solver.from_grid(g, objects(g))
    with pytest.raises(DieTeError):
        multi.matvec(dev(np.zeros((4, 2, 12, 12), np.complex128)))
    with pytest.raises(DieTeError):
        multi.solve(dev(np.zeros((2, 2, 12, 12), np.complex128)))


@pytest.mark.parametrize("reg,defl,mixed", [(False, 0, False), (True, 6, False), (False, 8, True)])
def test_solve_matches_single_object_and_lu(reg, defl, mixed):
    say(f"multi-object solve reg={reg} defl={defl} mixed={mixed}")
    g = centred_grid(22, 1.0, ny=18)
    eps = objects(g)
    nobj, psis = eps.shape[0], [0.2, 1.7]
    per = len(psis)
    b1 = fields(g, psis)
    B = np.concatenate([b1] * nobj)
    multi = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=5)
    U, rc, info = multi.solve(dev(B), restart=20, max_iters=20000, tol=1e-8, mixed=mixed)
    assert rc == 0
    Uh = host(U)
    for o in range(nobj):
        one = api.Solver.from_grid(g, eps[o], regularize=reg, deflate_k=defl, seed=5)
        u1, rc1, info1 = one.solve(dev(b1), restart=20, max_iters=20000, tol=1e-8, mixed=mixed)
        assert rc1 == 0
        u_lu = op.solve_dense(g, eps[o], b1)
        for r in range(per):
            i = o * per + r
            assert info[i]["status"] == 0 and info[i]["rel_res_true"] <= 1e-8
            # the same arithmetic on the same operands, batched differently: equal iteration counts
            assert info[i]["iters"] == info1[r]["iters"]
            assert rel(Uh[i], host(u1)[r]) < 1e-9
            assert op.relative_residual(g, eps[o], Uh[i], b1[r]) <= 1.02e-8
            assert rel(Uh[i], u_lu[r]) < 2e-5
        say(f"  object {o}: iters {[info[o * per + r]['iters'] for r in range(per)]}")


def test_deflation_per_object():
    g = centred_grid(16, 1.0)
    eps = objects(g)
    nobj, r = eps.shape[0], 5
    multi = api.Solver.from_grid(g, eps, regularize=True, deflate_k=r, seed=2)
    ritz, V, C = multi.deflation_info()
    assert ritz.shape == (nobj, r) and V.shape == (nobj, r, multi.nvec) and C.shape == (nobj, r, r)
    rng = np.random.default_rng(3)
    x = rand_c(rng, (nobj * 2, 2, 16, 16))
    ym = host(multi.apply_deflation(dev(x)))
    for o in range(nobj):
        one = api.Solver.from_grid(g, eps[o], regularize=True, deflate_k=r, seed=2)
        ritz1, V1, C1 = one.deflation_info()
        assert np.allclose(ritz[o].numpy(), ritz1.numpy(), rtol=1e-10, atol=0)
        assert torch.allclose(C[o], C1, rtol=1e-9, atol=1e-12)
        ys = host(one.apply_deflation(dev(x[2 * o:2 * o + 2])))
        assert rel(ym[2 * o:2 * o + 2], ys) < 1e-12
