"""The one-reduction Arnoldi (orth=1: CGS2 with the second projection delayed by one step)
against dense LU and against the two-projection CGS2 (orth=0): same solutions, comparable
iteration counts, all solver variants."""
import numpy as np
import pytest

from gpu_util import dev, host, rel, say
from oracle import operator as op
from synth import centred_grid, cylinder, square, plane_wave, random_field_object

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")


@pytest.mark.parametrize("eps_obj,reg,defl,mixed", [
    (4.0 + 0j, False, 0, False),
    (4.0 + 0j, False, 0, True),
    (-2.5 + 0.2j, True, 0, False),
    (-2.5 + 0.2j, True, 8, False),
    (-16 + 1.5j, True, 10, True),
    (16.0 + 0j, False, 6, False),
])
def test_one_reduction_matches_lu_and_cgs2(eps_obj, reg, defl, mixed):
    say(f"orth=1 vs LU eps={eps_obj} reg={reg} defl={defl} mixed={mixed}")
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, eps_obj)
    b = np.stack([plane_wave(g, 0.3), plane_wave(g, 2.1)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=3)
    u1, rc1, info1 = s.solve(dev(b), restart=20, max_iters=20000, tol=1e-8, mixed=mixed, orth=1)
    u0, rc0, info0 = s.solve(dev(b), restart=20, max_iters=20000, tol=1e-8, mixed=mixed, orth=0)
    assert rc1 == 0 and rc0 == 0
    uh = host(u1)
    for r in range(2):
        assert info1[r]["rel_res_true"] <= 1e-8
        assert op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8
        assert rel(uh[r], u_lu[r]) < 2e-5
        say(f"  rhs {r}: iters orth1 {info1[r]['iters']} orth0 {info0[r]['iters']}, products "
            f"{info1[r]['products_A']} / {info0[r]['products_A']}")
        # Near stagnation (the eps = 16 cylinder needs thousands of restarted iterations)
        # the counts of both variants move by several per cent under any change of
        # rounding order (an FFT summation order moved them from 3594 / 3378 to
        # 3888 / 3308), so the bound widens there.
        slack = 1.1 if info0[r]["iters"] < 1000 else 1.25
        assert info1[r]["iters"] <= slack * info0[r]["iters"] + 3


def test_one_reduction_batched_random_fields():
    """A batch of small random-field objects with several angles each: same iteration
    counts (to a few per cent) and the same solutions as CGS2, batch-invariant results."""
    objs = [random_field_object(48, seed=7000 + i) for i in range(4)]
    g = objs[0][0]
    eps = np.stack([e for _, e in objs])
    psis = [0.0, 1.3, 2.6]
    b = np.concatenate([np.stack([plane_wave(g, p) for p in psis])] * len(objs))
    s = api.Solver.from_grid(g, eps)
    for mixed in (0, 1, 2):
        u1, rc1, i1 = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, mixed=mixed, orth=1)
        u0, rc0, i0 = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, mixed=min(mixed, 1), orth=0)
        assert rc1 == 0 and rc0 == 0
        it1 = np.array([x["iters"] for x in i1])
        it0 = np.array([x["iters"] for x in i0])
        say(f"  mixed={mixed}: iters orth1 {it1.tolist()} orth0 {it0.tolist()}")
        assert it1.sum() <= (1.05 if mixed < 2 else 1.3) * it0.sum() + 5
        assert rel(host(u1), host(u0)) < 1e-6
        for o in range(len(objs)):
            sl = slice(3 * o, 3 * o + 3)
            assert all(op.relative_residual(g, eps[o], host(u1)[k], b[k]) <= 1.02e-8 for k in range(sl.start, sl.stop))
    # the same right-hand side alone gives the same iteration count (results do not depend on the batch)
    one = api.Solver.from_grid(g, eps[0])
    u, rc, info = one.solve(dev(b[1]), restart=30, max_iters=20000, tol=1e-8, orth=1)
    _, _, ib = s.solve(dev(b), restart=30, max_iters=20000, tol=1e-8, orth=1)
    assert info[0]["iters"] == ib[1]["iters"]


@pytest.mark.parametrize("eps_obj,reg,defl", [(4.0 + 0j, False, 0), (-2.5 + 0.2j, True, 8), (16.0 + 0j, False, 6)])
def test_binary16_basis_matches_lu(eps_obj, reg, defl):
    """mixed=2 stores the Krylov basis as complex binary16: the FP64 refinement still
    brings every solution to 1e-8; the iteration count may grow a little."""
    say(f"binary16 basis eps={eps_obj} reg={reg} defl={defl}")
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, eps_obj)
    b = np.stack([plane_wave(g, 0.3), plane_wave(g, 2.1)])
    u_lu = op.solve_dense(g, eps, b)
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=3)
    u2, rc2, i2 = s.solve(dev(b), restart=20, max_iters=40000, tol=1e-8, mixed=2, orth=1)
    _, rc1, i1 = s.solve(dev(b), restart=20, max_iters=40000, tol=1e-8, mixed=1, orth=1)
    assert rc2 == 0 and rc1 == 0
    uh = host(u2)
    for r in range(2):
        assert i2[r]["rel_res_true"] <= 1e-8
        assert op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8
        assert rel(uh[r], u_lu[r]) < 2e-5
        say(f"  rhs {r}: iters binary16 {i2[r]['iters']} complex64 {i1[r]['iters']}")


def test_binary16_basis_needs_one_reduction():
    g = centred_grid(16, 1.0)
    s = api.Solver.from_grid(g, cylinder(g, 0.3, 4.0 + 0j))
    with pytest.raises(Exception):
        s.solve(dev(plane_wave(g, 0.0)), mixed=2, orth=0)
