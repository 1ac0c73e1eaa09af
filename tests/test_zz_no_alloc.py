"""The product entry point that allocates nothing (die_te_matvec_noalloc): its FFT
intermediate lives in a static per-device scratch array.  It must equal die_te_matvec
on the same inputs (same pass variants, so bit for bit), on two calls in a row with the
second smaller than the first (the array keeps the first call's contents), in both
precisions, for a multi-object context, and reject an intermediate beyond the array."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, rand_c, say
from oracle import operator as op
from synth import centred_grid, cylinder

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")


def _pair(s, x):
    """(die_te_matvec, die_te_matvec_noalloc) of x on solver s."""
    nrhs = x.shape[0]
    y_ref = torch.empty_like(x)
    api.die_te_matvec(s.ctx, x, y_ref, nrhs)
    y_na = torch.full_like(x, float("nan"))
    api.die_te_matvec_noalloc(s.ctx, x, y_na, nrhs)
    torch.cuda.synchronize()
    return host(y_ref), host(y_na)


@pytest.mark.parametrize("dtype", [torch.complex128, torch.complex64])
def test_noalloc_equals_matvec_two_calls_second_smaller(dtype):
    rng = np.random.default_rng(7)
    g = centred_grid(200, 3.0, ny=180)  # px = 512, py = 512: tuned pass variants, ragged tiles
    eps = cylinder(g, 1.2, -2.5 + 0.2j)
    s = api.Solver.from_grid(g, eps)
    for nrhs in (6, 2):  # the second call smaller than the first
        say(f"noalloc vs matvec: {dtype} nrhs={nrhs} grid {g.ny}x{g.nx}")
        x = dev(rand_c(rng, (nrhs, 2, g.ny, g.nx)), dtype)
        y_ref, y_na = _pair(s, x)
        assert np.isfinite(y_na).all()
        assert np.array_equal(y_na, y_ref), rel(y_na, y_ref)
    # and against the oracle on one field (the 1e-12 bar in FP64, 2e-6 in FP32)
    x1 = rand_c(rng, (1, 2, g.ny, g.nx))
    y1 = torch.empty(1, 2, g.ny, g.nx, dtype=dtype, device="cuda")
    api.die_te_matvec_noalloc(s.ctx, dev(x1, dtype), y1, 1)
    ref = op.apply_operator(g, op.electric_contrast(eps), x1[0])
    err = rel(host(y1)[0], ref)
    say(f"  vs oracle: {err:.2e}")
    assert err <= (1e-12 if dtype == torch.complex128 else 2e-6)
    s.close()


def test_noalloc_multi_object_and_first_use_before_matvec():
    # a fresh context whose first product is the no-allocation one (no tuned variants yet for
    # this batch class), then the regular product: equal to the FP64 bar
    rng = np.random.default_rng(11)
    g = centred_grid(40, 1.0, ny=36)
    eps = np.stack([cylinder(g, 0.3, 4.0), cylinder(g, 0.4, -16 + 1.5j)])
    s = api.Solver.from_grid(g, eps)
    x = dev(rand_c(rng, (4, 2, g.ny, g.nx)))
    y_na = torch.empty_like(x)
    api.die_te_matvec_noalloc(s.ctx, x, y_na, 4)
    y_ref = torch.empty_like(x)
    api.die_te_matvec(s.ctx, x, y_ref, 4)
    torch.cuda.synchronize()
    assert rel(host(y_na), host(y_ref)) <= 1e-12
    s.close()


def test_noalloc_rejects_intermediate_beyond_scratch():
    g = centred_grid(256, 4.4)  # 2 * 512 * 256 complex128 = 4 MiB per field: 17 fields exceed 64 MiB
    s = api.Solver.from_grid(g, np.full((256, 256), 2.0 + 0j))
    x = torch.zeros(17, 2, 256, 256, dtype=torch.complex128, device="cuda")
    y = torch.empty_like(x)
    with pytest.raises(api._lib.DieTeError) as ei:
        api.die_te_matvec_noalloc(s.ctx, x, y, 17)
    assert ei.value.code == -1 and "scratch" in str(ei.value)
    # the largest accepted batch works
    x16 = torch.zeros(16, 2, 256, 256, dtype=torch.complex128, device="cuda")
    y16 = torch.empty_like(x16)
    api.die_te_matvec_noalloc(s.ctx, x16, y16, 16)
    torch.cuda.synchronize()
    assert float(y16.abs().max()) == 0.0
    s.close()
