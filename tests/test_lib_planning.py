"""The library's host-side planning entry points against the oracle (CPU only, no GPU call):
the memory planner of Section 5 against the oracle's planner (both reproduce the paper's
worked example, pinned in test_oracle_planning.py) over a range of inputs, and the closed-form
deflation radius against the oracle's densely sampled segment images."""
import numpy as np
import pytest

from oracle import planning as pl
from paper_1104_4263_amd import api
from paper_1104_4263_amd._lib import DieTeError


@pytest.mark.parametrize("M,beta,ppw,x,emax", [
    (2.0 ** 32, 0.0011, 15.0, 8.0, 15.0),   # the paper's worked example
    (8.0e9, 0.002, 15.0, 2.0, 16.0),
    (1.0e9, 0.0005, 20.0, 10.0, 4.0),
    (6.4e10, 0.003, 10.0, 0.5, 20.0),
])
def test_planner_matches_oracle(M, beta, ppw, x, emax):
    lib = api.die_te_plan_memory(M, beta, ppw, x, emax)
    ref = pl.plan_memory(M, beta, ppw, x, emax)
    for k in ("alpha", "n_max", "a_over_lambda_max"):
        assert abs(lib[k] - ref[k]) <= 1e-12 * abs(ref[k])
    assert lib["nodes"] == ref["nodes"] and lib["n"] == ref["N"] and lib["unknowns"] == ref["unknowns"]
    assert lib["r"] == ref["r"] and lib["restart"] == ref["restart"]
    assert lib["restart_unpreconditioned"] == ref["restart_unpreconditioned"]
    assert abs(lib["mem_system"] - ref["M_A"]) <= 1e-9 * ref["M_A"]
    assert abs(lib["mem_preconditioner"] - ref["M_prec"]) <= 1e-9 * ref["M_prec"]


def test_planner_rejects_bad_inputs():
    with pytest.raises(DieTeError):
        api.die_te_plan_memory(-1.0, 0.001, 15, 8, 15)
    with pytest.raises(DieTeError):
        api.die_te_plan_memory(1e9, 0.0, 15, 8, 15)


def test_radius_closed_form_matches_sampled_images():
    rng = np.random.default_rng(5)
    eps = np.concatenate([1 + 19 * rng.random(40) + 1j * rng.random(40),
                          -20 * rng.random(20) + 1j * rng.random(20) * 2,
                          [16.0, -16 + 1.5j, 2.5 + 20j, -2.5 + 0.2j, -3 + 0.1j, 1.0]])
    for e in eps:
        lib = api.die_te_deflation_radius([e], True)
        ref = pl.segment_image_radius(e, samples=40001)
        assert abs(lib - ref) <= 2e-7 * ref, (e, lib, ref)
    # inhomogeneous: the largest over the cells
    assert abs(api.die_te_deflation_radius(eps, True) - pl.deflation_radius(eps, samples=40001)) <= 2e-7 * 40
    # without the regularizer the segments themselves: max |eps|, at least 1
    assert api.die_te_deflation_radius(eps, False) == max(1.0, float(np.abs(eps).max()))


def test_radius_rejects_zero_permittivity():
    with pytest.raises(DieTeError) as ei:
        api.die_te_deflation_radius([2.0, 0.0], True)
    assert ei.value.code == -2
