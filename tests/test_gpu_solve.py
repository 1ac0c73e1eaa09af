"""GPU solves against the oracle: dense LU on small grids, the direct-sum true
residual, the Mie series on the small cylinder; regularized, deflated, mixed
precision and batched variants; error and warning paths."""
import math

import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, rand_c, say
from oracle import operator as op
from oracle import mie
from synth import centred_grid, cylinder, square, layered_square, plane_wave, cell_centres, workload

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")


def lu_case(n, eps_obj, shape="cyl"):
    g = centred_grid(n, 1.0, ny=n - 4)
    if shape == "cyl":
        eps = cylinder(g, 0.35, eps_obj)
    elif shape == "layer":
        eps = layered_square(g, 0.7, 16.0, 2.5 + 20j)
    else:
        eps = square(g, 0.6, eps_obj)
    b = np.stack([plane_wave(g, 0.3), plane_wave(g, 2.1)])
    u_lu = op.solve_dense(g, eps, b)
    return g, eps, b, u_lu


@pytest.mark.parametrize("eps_obj,reg,defl,mixed", [
    (4.0 + 0j, False, 0, False),
    (4.0 + 0j, False, 0, True),
    (-2.5 + 0.2j, True, 0, False),
    (-2.5 + 0.2j, True, 8, False),
    (-16 + 1.5j, True, 10, True),
    (16.0 + 0j, False, 6, False),
])
def test_solve_matches_lu(eps_obj, reg, defl, mixed):
    say(f"solve vs LU eps={eps_obj} reg={reg} defl={defl} mixed={mixed}")
    g, eps, b, u_lu = lu_case(24, eps_obj)
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=3)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=20000, tol=1e-8, mixed=mixed)
    uh = host(u)
    for r in range(2):
        assert info[r]["status"] == 0 and info[r]["rel_res_true"] <= 1e-8
        res = op.relative_residual(g, eps, uh[r], b[r])
        say(f"  rhs {r}: iters {info[r]['iters']} cycles {info[r]['cycles']} gpu res {info[r]['rel_res_true']:.2e} "
            f"oracle res {res:.2e} |u-u_lu|/|u_lu| {rel(uh[r], u_lu[r]):.2e}")
        assert res <= 1.02e-8
        assert rel(uh[r], u_lu[r]) < 2e-5
    assert rc == 0


def test_cyl_small_plain_vs_mie_and_oracle():
    w = workload("cyl_small")
    g, eps = w["grids"][0], w["eps"][0]
    b = plane_wave(g, 0.0)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=5000, tol=1e-8)
    uh = host(u)
    assert rc == 0 and info[0]["rel_res_true"] <= 1e-8
    assert op.relative_residual(g, eps, uh, b) <= 1.02e-8
    X, Y = cell_centres(g)
    E = mie.total_field(X, Y, g.k, 0.5, 4.0, 0.0)
    err = rel(uh, E)
    say(f"cyl_small iters {info[0]['iters']} mie rel err {err:.3f}")
    assert err < 0.08


def test_batched_equals_separate():
    g, eps, b, u_lu = lu_case(20, 4.0 + 0j, shape="square")
    psis = [0.0, 0.7, 1.9, 3.0, 4.4]
    B = np.stack([plane_wave(g, p) for p in psis])
    s = api.Solver.from_grid(g, eps)
    U, rc, info = s.solve(dev(B), restart=15, max_iters=5000)
    assert rc == 0
    for r, p in enumerate(psis):
        u1, rc1, i1 = s.solve(dev(B[r]), restart=15, max_iters=5000)
        assert rc1 == 0
        assert i1[0]["iters"] == info[r]["iters"]
        assert rel(host(U[r]), host(u1)) < 1e-12
        assert op.relative_residual(g, eps, host(U[r]), B[r]) <= 1.02e-8


def test_initial_guess_resume():
    g, eps, b, u_lu = lu_case(20, -2.5 + 0.2j)
    s = api.Solver.from_grid(g, eps)
    u1, rc1, i1 = s.solve(dev(b), restart=10, max_iters=25)
    assert rc1 == 1 and all(i["status"] == 1 for i in i1)
    # resume from the returned best iterate: reaches the tolerance
    u2, rc2, i2 = s.solve(dev(b), x0=u1, restart=10, max_iters=20000)
    assert rc2 == 0
    assert op.relative_residual(g, eps, host(u2[0]), b[0]) <= 1.02e-8
    # the warning path returned a residual the oracle agrees with
    res1 = op.relative_residual(g, eps, host(u1[0]), b[0])
    assert abs(res1 - i1[0]["rel_res_true"]) <= 1e-6 * res1


def test_exact_initial_guess_takes_no_iteration():
    g, eps, b, u_lu = lu_case(16, 4.0 + 0j)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b[0]), x0=dev(u_lu[0]), restart=10, max_iters=100)
    assert rc == 0 and info[0]["iters"] == 0


def test_zero_incident_field():
    g = centred_grid(8, 0.3)
    s = api.Solver.from_grid(g, cylinder(g, 0.1, 4.0))
    u, rc, info = s.solve(torch.zeros(2, 8, 8, dtype=torch.complex128, device="cuda"))
    assert rc == 0 and float(u.abs().max()) == 0.0


def test_singular_and_invalid_inputs():
    g = centred_grid(8, 0.3)
    eps = cylinder(g, 0.1, 4.0)
    eps[3, 3] = 0.0
    with pytest.raises(api._lib.DieTeError) as ei:
        api.Solver.from_grid(g, eps)
    assert ei.value.code == -2
    with pytest.raises(api._lib.DieTeError) as ei:
        api.Solver(8, 8, 0.01, np.ones((8, 8)), px=8)  # px < 2 nx - 1
    assert ei.value.code == -1
    with pytest.raises(api._lib.DieTeError) as ei:
        api.Solver(8, 8, -0.01, np.ones((8, 8)))
    assert ei.value.code == -1
    s = api.Solver.from_grid(g, np.ones((8, 8)) * 2)
    with pytest.raises(api._lib.DieTeError) as ei:
        s.solve(dev(plane_wave(g, 0.0)), restart=0)
    assert ei.value.code == -1
