"""Objects on grids of different sizes in one call (die_te_solve_batch): the same results,
bit for bit, as one die_te_solve call per grid, every solution at the FP64 true-residual
tolerance against the oracle's direct-sum operator, and errors reported per context."""
import math

import numpy as np
import pytest
import torch

from gpu_util import dev, host, say
from oracle import operator as op
from synth import random_field_object, plane_wave

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")
from paper_1104_4263_amd._lib import DieTeError  # noqa: E402


def _classes(sizes, per, seed0):
    """One context per grid size, `per` random-field objects each, 3 angles per object."""
    out = []
    for k, n in enumerate(sizes):
        objs = [random_field_object(n, seed=seed0 + 10 * k + i) for i in range(per)]
        g = objs[0][0]
        eps = np.stack([e for _, e in objs])
        b = np.concatenate([np.stack([plane_wave(g, p) for p in (0.0, 2.1, 4.2)]) for _ in range(per)])
        out.append((g, eps, b))
    return out


@pytest.mark.parametrize("mixed,orth", [(0, 0), (2, 1)])
def test_batch_equals_separate_calls(mixed, orth):
    say(f"solve_batch mixed={mixed} orth={orth}")
    cls = _classes([16, 32, 24], 2, 4200)
    solvers = [api.Solver.from_grid(g, eps) for g, eps, _ in cls]
    B = [dev(b) for _, _, b in cls]
    kw = dict(restart=20, max_iters=4000, tol=1e-8, mixed=mixed, orth=orth)
    sep = [s.solve(b, **kw) for s, b in zip(solvers, B)]
    res, rc = api.Solver.solve_batch(solvers, B, **kw)
    assert rc == 0
    for k, ((u, info), (u1, rc1, info1)) in enumerate(zip(res, sep)):
        assert rc1 == 0
        assert torch.equal(u, u1), k  # fixed-order sums: concurrency does not change a bit
        assert [x["iters"] for x in info] == [x["iters"] for x in info1]
        g, eps, b = cls[k]
        uh = host(u)
        for r in range(b.shape[0]):
            assert info[r]["rel_res_true"] <= 1e-8
            assert op.relative_residual(g, eps[r // 3], uh[r], b[r]) <= 1.02e-8
        say(f"  {g.nx}x{g.ny}: iters {[x['iters'] for x in info]}")


def test_batch_with_initial_guesses_and_one_context():
    cls = _classes([16], 2, 4300)
    g, eps, b = cls[0]
    s = api.Solver.from_grid(g, eps)
    B = dev(b)
    u0, rc0, _ = s.solve(B, restart=20, max_iters=4000, tol=1e-8)
    res, rc = api.Solver.solve_batch([s], [B], x0s=[u0], restart=20, max_iters=4000, tol=1e-8)
    assert rc == 0
    u, info = res[0]
    assert all(x["iters"] == 0 for x in info)  # started at a converged solution
    assert torch.equal(u, u0)


def test_batch_reports_the_failing_context():
    cls = _classes([16, 24], 2, 4400)
    solvers = [api.Solver.from_grid(g, eps) for g, eps, _ in cls]
    B = [dev(b) for _, _, b in cls]
    bad = B[1][:5].contiguous()  # 5 fields for 2 objects: not a multiple of the object count
    with pytest.raises(DieTeError, match="context 1"):
        api.Solver.solve_batch(solvers, [B[0], bad], restart=20, max_iters=100, tol=1e-8)
    with pytest.raises(ValueError):
        api.Solver.solve_batch(solvers, B, x0s=[B[0], None])
