"""The TM operator and the full (E1, E2, H3) TE system with magnetic contrast on the GPU
against the oracle (oracle/systems.py): products against the direct sums (FP64 1e-12,
FP32 2e-6 relative) on odd, ragged and degenerate grids; solves against dense LU and the
oracle's residual, plain, deflated (automatic size: the unit circle for TM), regularized
(full system), mixed precision and the block solver."""
import math

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, rand_c, say
from oracle import operator as op
from oracle import systems as sy
from synth import centred_grid, cylinder, square, layered_square, plane_wave

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")

GRIDS = [(1, 1), (1, 7), (6, 1), (13, 9), (24, 20), (33, 17)]


@pytest.mark.parametrize("nx,ny", GRIDS)
def test_tm_products_vs_direct_sum(nx, ny):
    rng = np.random.default_rng(nx * 100 + ny)
    g = centred_grid(nx, 0.04 * nx, ny=ny)
    eps = 1.0 + 6.0 * rng.random((ny, nx)) - 3.0 * (rng.random((ny, nx)) < 0.3) * 3.0 + 0.5j * rng.random((ny, nx))
    x = rand_c(rng, (3, 1, ny, nx))
    s = api.Solver.from_grid(g, eps, polarization="tm")
    ref = np.stack([sy.apply_operator_tm(g, eps - 1.0, x[r, 0]) for r in range(3)])[:, None]
    y64 = host(s.matvec(dev(x)))
    y32 = host(s.matvec(dev(x, torch.complex64)))
    e64, e32 = rel(y64, ref), rel(y32, ref)
    say(f"TM product {nx}x{ny}: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 2e-6
    s.close()


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 7), (9, 5), (16, 12), (21, 19)])
def test_full_system_products_vs_direct_sum(nx, ny):
    rng = np.random.default_rng(nx * 31 + ny)
    g = centred_grid(nx, 0.05 * nx, ny=ny)
    eps = 2.0 + 8.0 * rng.random((ny, nx)) + 1j * rng.random((ny, nx))
    mu = 1.0 + 3.0 * rng.random((ny, nx)) + 0.3j * rng.random((ny, nx))
    x = rand_c(rng, (2, 3, ny, nx))
    s = api.Solver.from_grid(g, eps, magnetic=True, mu_r=mu)
    ref = np.stack([sy.apply_operator_full(g, eps - 1.0, mu - 1.0, x[r]) for r in range(2)])
    y64 = host(s.matvec(dev(x)))
    y32 = host(s.matvec(dev(x, torch.complex64)))
    e64, e32 = rel(y64, ref), rel(y32, ref)
    say(f"full TE product {nx}x{ny}: fp64 {e64:.2e} fp32 {e32:.2e}")
    assert e64 <= 1e-12 and e32 <= 2e-6
    # the regularizer: the same operator with chi' = 1/eps - 1 and chi_m' = 1/mu - 1
    rr = np.stack([sy.apply_operator_full(g, 1.0 / eps - 1.0, 1.0 / mu - 1.0, x[r]) for r in range(2)])
    assert rel(host(s.regularize(dev(x))), rr) <= 1e-12
    s.close()


def test_full_system_without_mu_matches_te_block_and_post_processes_h3():
    rng = np.random.default_rng(4)
    g = centred_grid(20, 1.0, ny=16)
    eps = cylinder(g, 0.35, 4.0 + 0.5j)
    s3 = api.Solver.from_grid(g, eps, magnetic=True)
    s2 = api.Solver.from_grid(g, eps)
    x = rand_c(rng, (1, 3, g.ny, g.nx))
    y3 = host(s3.matvec(dev(x)))
    y2 = host(s2.matvec(dev(x[:, :2].copy())))
    assert rel(y3[:, :2], y2) <= 1e-13
    s2.close()
    s3.close()


def _tm_case(n=24):
    g = centred_grid(n, 1.0, ny=n - 4)
    eps = cylinder(g, 0.35, -16 + 1.5j)
    b = np.stack([sy.plane_wave_tm(g, 0.3), sy.plane_wave_tm(g, 2.1)])[:, None]
    return g, eps, b


@pytest.mark.parametrize("defl,mixed,block", [(0, 0, 0), (8, 0, 0), (-1, 1, 0), (0, 1, 2), (6, 0, 1)])
def test_tm_solves_vs_lu(defl, mixed, block):
    g, eps, b = _tm_case()
    s = api.Solver.from_grid(g, eps, polarization="tm", deflate_k=defl, seed=3)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=20000, tol=1e-8, mixed=mixed, block=block,
                          orth=1 if block == 1 else 0)
    uh = host(u)
    u_lu = sy.solve_dense_tm(g, eps, b[:, 0])
    for r in range(2):
        res = np.linalg.norm(b[r, 0] - sy.apply_operator_tm(g, eps - 1.0, uh[r, 0])) / np.linalg.norm(b[r, 0])
        say(f"TM solve defl={defl} mixed={mixed} block={block} rhs {r}: iters {info[r]['iters']} "
            f"oracle res {res:.2e} |u-u_lu| {rel(uh[r, 0], u_lu[r]):.2e}")
        assert info[r]["status"] == 0 and res <= 1.02e-8 and rel(uh[r, 0], u_lu[r]) < 2e-5
    assert rc == 0
    if defl == -1:
        ritz, _, _ = s.deflation_info()
        k = int((ritz.abs() > 0).sum())
        assert k >= 1 and bool((ritz[:k].abs() > 1.0 - 1e-6).all())
    s.close()


@pytest.mark.parametrize("reg,defl,mixed", [(False, 0, 0), (True, 0, 0), (True, 6, 1), (False, 0, 1)])
def test_full_system_solves_vs_lu(reg, defl, mixed):
    g = centred_grid(18, 0.9, ny=16)
    eps = cylinder(g, 0.3, 2.5 + 0.2j)
    mu = cylinder(g, 0.3, 1.8 + 0.05j)
    E = np.stack([plane_wave(g, 0.4), plane_wave(g, 1.9)])
    H3 = np.stack([E[0, 1] / math.cos(0.4), E[1, 1] / math.cos(1.9)])
    b = np.concatenate([E, H3[:, None]], axis=1)
    s = api.Solver.from_grid(g, eps, magnetic=True, mu_r=mu, regularize=reg, deflate_k=defl, seed=2)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=20000, tol=1e-8, mixed=mixed)
    uh = host(u)
    u_lu = sy.solve_dense_full(g, eps, mu, b)
    for r in range(2):
        res = np.linalg.norm(b[r] - sy.apply_operator_full(g, eps - 1.0, mu - 1.0, uh[r])) / np.linalg.norm(b[r])
        say(f"full solve reg={reg} defl={defl} mixed={mixed} rhs {r}: iters {info[r]['iters']} res {res:.2e}")
        assert info[r]["status"] == 0 and res <= 1.02e-8 and rel(uh[r], u_lu[r]) < 2e-5
    assert rc == 0
    s.close()


def test_option_validation():
    g = centred_grid(8, 0.3)
    eps = np.full((8, 8), 2.0 + 0j)
    with pytest.raises(api._lib.DieTeError):
        api.Solver.from_grid(g, eps, polarization="tm", regularize=True)
    with pytest.raises(api._lib.DieTeError):
        api.Solver.from_grid(g, eps, polarization="tm", magnetic=True)
    mu = np.full((8, 8), 1.5 + 0j)
    mu[2, 2] = 0.0
    with pytest.raises(api._lib.DieTeError) as ei:
        api.Solver.from_grid(g, eps, magnetic=True, mu_r=mu)
    assert ei.value.code == -2
