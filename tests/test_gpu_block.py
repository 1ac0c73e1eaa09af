"""Block GMRES (solve option block=1, and block=2 with its Gram-Schmidt GEMMs in binary16):
all right-hand sides of an object share one block Krylov space.  Solutions against dense LU
and against the per-rhs solver, the regularized and deflated variants, a rank-deficient set
of incident fields, and the product savings."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import operator as op
from synth import centred_grid, cylinder, plane_wave, random_field_object

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")
from paper_1104_4263_amd._lib import DIE_PROF_GEMM, DieTeError  # noqa: E402


@pytest.mark.parametrize("orth", [0, 1])
@pytest.mark.parametrize("eps_obj,reg,defl,mixed", [
    (4.0 + 0j, False, 0, 0), (4.0 + 0j, False, 0, 1), (-2.5 + 0.2j, True, 0, 0),
    (-2.5 + 0.2j, True, 8, 0), (16.0 + 0j, False, 6, 1), (-16 + 1.5j, True, 10, 1),
])
def test_block_matches_lu(eps_obj, reg, defl, mixed, orth):
    say(f"block GMRES eps={eps_obj} reg={reg} defl={defl} mixed={mixed} orth={orth}")
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, eps_obj)
    b = np.stack([plane_wave(g, p) for p in (0.3, 1.2, 2.1, 4.0)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=3)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=4000, tol=1e-8, mixed=mixed, block=1, orth=orth)
    assert rc == 0
    uh = host(u)
    for r in range(b.shape[0]):
        assert info[r]["rel_res_true"] <= 1e-8
        assert op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8
        assert rel(uh[r], u_lu[r]) < 2e-5
    say(f"  block steps {[x['iters'] for x in info]}, cycles {[x['cycles'] for x in info]}, "
        f"products per rhs {[x['products_A'] for x in info]}")


def test_block_multi_object_agrees_with_per_rhs_solver():
    objs = [random_field_object(32, seed=7000 + i) for i in range(3)]
    g = objs[0][0]
    eps = np.stack([e for _, e in objs])
    psis = [2 * np.pi * j / 8 for j in range(8)]
    b = np.concatenate([np.stack([plane_wave(g, p) for p in psis])] * 3)
    s = api.Solver.from_grid(g, eps)
    ub, rcb, ib = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, mixed=1, block=1, orth=1)
    up, rcp, ip = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, mixed=1)
    assert rcb == 0 and rcp == 0
    assert rel(host(ub), host(up)) < 1e-6
    for r in range(b.shape[0]):
        assert op.relative_residual(g, eps[r // 8], host(ub)[r], b[r]) <= 1.02e-8
    pb = sum(x["products_A"] for x in ib)
    pp = sum(x["products_A"] for x in ip)
    say(f"  products block {pb} vs per-rhs {pp}")
    assert pb < pp


def test_block_rank_deficient_fields_and_warm_start():
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, 4.0 + 0j)
    b0 = plane_wave(g, 0.7)
    b = np.stack([b0, plane_wave(g, 2.0), b0, 2.0 * b0])  # three fields along one direction
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=4000, tol=1e-8, block=1)
    assert rc == 0
    uh = host(u)
    assert rel(uh[2], uh[0]) < 1e-10 and rel(uh[3], 2.0 * uh[0]) < 1e-10
    u_lu = op.solve_dense(g, eps, b)
    assert rel(uh, u_lu) < 2e-5
    # started at the solution: no block step
    u2, rc2, info2 = s.solve(dev(b), x0=u, restart=20, max_iters=4000, tol=1e-8, block=1)
    assert rc2 == 0 and all(x["iters"] == 0 for x in info2)


@pytest.mark.parametrize("orth", [0, 1])
@pytest.mark.parametrize("eps_obj,reg,defl", [
    (4.0 + 0j, False, 0), (-2.5 + 0.2j, True, 8), (16.0 + 0j, False, 6), (-16 + 1.5j, True, 10),
])
def test_block_half_gemm_matches_lu(eps_obj, reg, defl, orth):
    """block=2: the projections and updates on binary16 planar copies; the FP64 restarts still
    take every right-hand side to the same true residual and LU solution as block=1."""
    say(f"block GMRES binary16 GEMMs eps={eps_obj} reg={reg} defl={defl} orth={orth}")
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, eps_obj)
    b = np.stack([plane_wave(g, p) for p in (0.3, 1.2, 2.1, 4.0)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=3)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=4000, tol=1e-8, mixed=1, block=2, orth=orth)
    assert rc == 0
    uh = host(u)
    for r in range(b.shape[0]):
        assert info[r]["rel_res_true"] <= 1e-8
        assert op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8
        assert rel(uh[r], u_lu[r]) < 2e-5
    say(f"  block steps {[x['iters'] for x in info]}, cycles {[x['cycles'] for x in info]}")


@pytest.mark.parametrize("block,mixed", [(1, 0), (1, 1), (2, 1)])
@pytest.mark.parametrize("nx,ny", [(3, 3), (5, 4)])
def test_block_krylov_space_filled_within_a_cycle(block, mixed, nx, ny):
    """18 and 40 unknowns, four right-hand sides, GMRES(10): the block Krylov space fills the
    whole space after a few block steps, so a new block is numerically dependent and the cycle
    ends before it (the device CholQR factor's rank test, which the host reads one step later,
    after the next step is already queued); the solutions still match dense LU."""
    g = centred_grid(nx, 1.0, ny=ny)
    eps = cylinder(g, 0.35, 4.0 + 0j)
    b = np.stack([plane_wave(g, 0.3 + 1.1 * q) for q in range(4)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=10, max_iters=2000, tol=1e-8, mixed=mixed, block=block, orth=0)
    say(f"  {nx}x{ny} block={block} mixed={mixed}: block steps {[x['iters'] for x in info]}")
    assert rc == 0
    uh = host(u)
    for r in range(b.shape[0]):
        assert info[r]["rel_res_true"] <= 1e-8
        assert op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8
        assert rel(uh[r], u_lu[r]) < 2e-5


@pytest.mark.parametrize("block", [1, 2])
def test_block_more_than_64_rhs_per_object(block):
    """70 incidence angles on one object: the block solver runs them in two groups (64 and 6
    right-hand sides) that reuse the same per-step flags, events and buffers one after another."""
    g = centred_grid(16, 1.0)
    eps = cylinder(g, 0.35, 4.0 + 0j)
    b = np.stack([plane_wave(g, 2.0 * np.pi * q / 70) for q in range(70)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=4000, tol=1e-8, mixed=1, block=block, orth=0)
    say(f"  block={block}: block steps {sorted({x['iters'] for x in info})}")
    assert rc == 0
    uh = host(u)
    for r in range(b.shape[0]):
        assert info[r]["rel_res_true"] <= 1e-8
        assert rel(uh[r], u_lu[r]) < 2e-5
    for r in (0, 37, 64, 69):
        assert op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8


@pytest.mark.parametrize("nang", [1, 3])
def test_block_half_gemm_small_blocks(nang):
    """block=2 with one and with three right-hand sides per object (blocks of width 1 and 3)."""
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, 4.0 + 0j)
    b = np.stack([plane_wave(g, 0.4 + 1.9 * q) for q in range(nang)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=4000, tol=1e-8, mixed=1, block=2, orth=0)
    assert rc == 0
    for r in range(nang):
        assert info[r]["rel_res_true"] <= 1e-8
        assert rel(host(u)[r], u_lu[r]) < 2e-5


def test_block_half_gemm_rank_deficient_and_warm_start():
    """block=2 on fields where three of four lie along one direction: the duplicates get the same
    solution (and the doubled field twice it), and a start at the solution takes no block step."""
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, 4.0 + 0j)
    b0 = plane_wave(g, 0.7)
    b = np.stack([b0, plane_wave(g, 2.0), b0, 2.0 * b0])
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=20, max_iters=4000, tol=1e-8, mixed=1, block=2, orth=0)
    assert rc == 0
    uh = host(u)
    assert rel(uh[2], uh[0]) < 1e-12 and rel(uh[3], 2.0 * uh[0]) < 1e-12
    assert rel(uh, op.solve_dense(g, eps, b)) < 2e-5
    u2, rc2, info2 = s.solve(dev(b), x0=u, restart=20, max_iters=4000, tol=1e-8, mixed=1, block=2, orth=0)
    assert rc2 == 0 and all(x["iters"] == 0 for x in info2)


def test_block_half_gemm_odd_grid():
    """block=2 on a 15 x 13 grid: a vector length (390) that is even but not a multiple of 4."""
    g = centred_grid(15, 1.0, ny=13)
    eps = cylinder(g, 0.3, 4.0 + 0.5j)
    b = np.stack([plane_wave(g, p) for p in (0.1, 1.7, 3.3)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=12, max_iters=2000, tol=1e-8, mixed=1, block=2, orth=0)
    assert rc == 0
    assert rel(host(u), u_lu) < 2e-5


@pytest.mark.parametrize("n_side,nobj,nang", [(32, 3, 8), (64, 2, 16)])
def test_block_half_gemm_multi_object_agrees(n_side, nobj, nang):
    """block=2 on random-field objects with the projection split into several K chunks
    (vector lengths 2048 and 8192): same solutions as the per-rhs solver, to the tolerance."""
    objs = [random_field_object(n_side, seed=7100 + i) for i in range(nobj)]
    g = objs[0][0]
    eps = np.stack([e for _, e in objs])
    psis = [2 * np.pi * j / nang for j in range(nang)]
    b = np.concatenate([np.stack([plane_wave(g, p) for p in psis])] * nobj)
    s = api.Solver.from_grid(g, eps)
    say(f"block=2 {n_side}^2 x {nobj} objects x {nang} angles")
    ub, rcb, ib = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, mixed=1, block=2, orth=1)
    up, rcp, ip = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, mixed=1)
    assert rcb == 0 and rcp == 0
    uh = host(ub)
    for r in range(b.shape[0]):
        assert ib[r]["rel_res_true"] <= 1e-8
        assert op.relative_residual(g, eps[r // nang], uh[r], b[r]) <= 1.02e-8
    assert rel(uh, host(up)) < 1e-6
    say(f"  block steps {sorted(set(x['iters'] for x in ib))}, cycles {sorted(set(x['cycles'] for x in ib))}")


def test_block_contexts_in_one_batch_call_with_profiling():
    """Two single-object contexts solved together by die_te_solve_batch (a thread and a stream
    each) with block=2: the same fields as solving them one by one, and the HIP-event timing
    recorded on the call's own streams can still be read after the call returns."""
    objs = [random_field_object(32, seed=7200 + i) for i in range(2)]
    g = objs[0][0]
    b = np.stack([plane_wave(g, 2 * np.pi * j / 8) for j in range(8)])
    kw = dict(restart=30, max_iters=20000, tol=1e-8, mixed=1, block=2, orth=0)
    singles = [api.Solver.from_grid(g, e) for _, e in objs]
    for sv in singles:
        sv.profile(1)
    res, rc = api.Solver.solve_batch(singles, [dev(b)] * 2, **kw)
    assert rc == 0
    for sv in singles:
        n, seen, ms, flops = sv.profile_read(DIE_PROF_GEMM)
        assert n > 0 and seen == n and ms > 0.0 and flops > 0.0
        assert sv.profile_mem(DIE_PROF_GEMM) > 0.0
        sv.profile(0)
    for (u, info), sv, (_, e) in zip(res, singles, objs):
        u1, rc1, _ = sv.solve(dev(b), **kw)
        assert rc1 == 0
        assert rel(host(u), host(u1)) < 1e-6
        for r in range(b.shape[0]):
            assert info[r]["rel_res_true"] <= 1e-8
            assert op.relative_residual(g, e, host(u)[r], b[r]) <= 1.02e-8


def test_block_context_reused_across_precisions():
    """The block solver keeps its work buffers in the context: complex64, then complex128, then
    complex64 solves on one context give the same fields as fresh contexts."""
    g = centred_grid(32, 1.0, ny=28)
    eps = cylinder(g, 0.35, 4.0 + 0.3j)
    b = np.stack([plane_wave(g, p) for p in (0.2, 1.1, 2.6, 3.9, 5.0)])
    s = api.Solver.from_grid(g, eps)
    outs = []
    for mixed, block in ((1, 2), (0, 1), (1, 1)):
        u, rc, info = s.solve(dev(b), restart=15, max_iters=4000, tol=1e-8, mixed=mixed, block=block,
                              orth=0 if block == 2 else 1)
        assert rc == 0
        fresh = api.Solver.from_grid(g, eps)
        uf, rcf, _ = fresh.solve(dev(b), restart=15, max_iters=4000, tol=1e-8, mixed=mixed, block=block,
                                 orth=0 if block == 2 else 1)
        assert rcf == 0
        assert rel(host(u), host(uf)) < 1e-6
        for r in range(b.shape[0]):
            assert op.relative_residual(g, eps, host(u)[r], b[r]) <= 1.02e-8
        outs.append(host(u))
    assert rel(outs[0], outs[1]) < 2e-6 and rel(outs[2], outs[1]) < 2e-6


def test_block_option_validation():
    g = centred_grid(16, 1.0)
    s = api.Solver.from_grid(g, cylinder(g, 0.3, 4.0))
    b = dev(plane_wave(g, 0.0))
    with pytest.raises(DieTeError):
        s.solve(b, block=1, mixed=2, orth=1)
    with pytest.raises(DieTeError):
        s.solve(b, block=2, mixed=0)
    with pytest.raises(DieTeError):
        s.solve(b, block=3, mixed=1)


@pytest.mark.parametrize("block", [1, 2])
def test_mixed_block_fp64_finish_of_stalled_rhs(block):
    """Restarted GMRES(6) on an eps = 9 cylinder: an early cycle gains under 10% (restart
    stagnation, in any precision), so the complex64 block cycles hand the right-hand side to the
    FP64 finish, which converges (about 1200 steps, as the FP64 solvers alone); the result
    matches dense LU."""
    say(f"FP64 finish of a stalled complex64 block solve, block={block}")
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, 9.0 + 0j)
    b = plane_wave(g, 0.3)[None]
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps)
    u, rc, info = s.solve(dev(b), restart=6, max_iters=6000, tol=1e-8, mixed=1, block=block,
                          orth=0 if block == 2 else 1)
    say(f"  iters {info[0]['iters']}, FP64 finish {info[0]['finish_iters']}, cycles {info[0]['cycles']}")
    assert rc == 0 and info[0]["status"] == 0
    assert 0 < info[0]["finish_iters"] < info[0]["iters"]
    assert info[0]["rel_res_true"] <= 1e-8
    assert op.relative_residual(g, eps, host(u)[0], b[0]) <= 1.02e-8
    assert rel(host(u)[0], u_lu[0]) < 2e-5
    # a solve that converges without stalling reports no FP64 finish
    _, rc2, info2 = s.solve(dev(b), restart=30, max_iters=6000, tol=1e-8, mixed=1, block=block,
                            orth=0 if block == 2 else 1)
    assert rc2 == 0 and info2[0]["finish_iters"] == 0
