"""Bi-CGSTAB, restarted GCR and IDR(s) on the GPU (the paper's Conclusions name them as
alternatives on the preconditioned system A_R A P^-1 v = A_R b) against dense LU and the
oracle's direct-sum residual, plain, regularized, deflated and both; their iteration counts
beside the oracle's own solvers on the same dense system; the TM and full systems; the guess
fallback; and the option checks."""
import numpy as np
import pytest
import torch

from gpu_util import dev, host, rel, say
from oracle import krylov
from oracle import operator as op
from oracle import systems as sy
from synth import centred_grid, cylinder, plane_wave

pytestmark = pytest.mark.gpu

api = pytest.importorskip("paper_1104_4263_amd.api")


def _case():
    g = centred_grid(24, 1.0, ny=20)
    eps = cylinder(g, 0.35, 4.0 + 0.5j)
    b = np.stack([plane_wave(g, 0.3), plane_wave(g, 1.7)])
    return g, eps, b


RESTART = {"bicgstab": 20, "gcr": 20, "idrs": 4}


@pytest.mark.parametrize("method", ["bicgstab", "gcr", "idrs"])
@pytest.mark.parametrize("reg,defl", [(False, 0), (True, 0), (False, 6), (True, 6)])
def test_alt_solvers_vs_lu(method, reg, defl):
    g, eps, b = _case()
    s = api.Solver.from_grid(g, eps, regularize=reg, deflate_k=defl, seed=2)
    u, rc, info = s.solve(dev(b), restart=RESTART[method], max_iters=20000, tol=1e-8, method=method)
    uh = host(u)
    u_lu = op.solve_dense(g, eps, b)
    # the oracle's solver on the same dense system (the GPU deflation basis for P^-1)
    A = op.dense_operator(g, op.electric_contrast(eps))
    AR = op.dense_operator(g, op.regularizer_contrast(eps))
    M = AR @ A if reg else A
    prec = None
    if defl:
        _, V, C = s.deflation_info()
        V, C = host(V), host(C)
        Pinv = np.eye(A.shape[0]) + V.T @ C @ V.conj()
        prec = lambda x: Pinv @ x  # noqa: E731
    for r in range(2):
        bb = b[r].ravel()
        res = op.relative_residual(g, eps, uh[r], b[r])
        rhs = AR @ bb if reg else bb
        fn = {"bicgstab": krylov.bicgstab, "gcr": krylov.gcr, "idrs": krylov.idrs}[method]
        kw = {"bicgstab": {}, "gcr": {"restart": 20}, "idrs": {"s": 4}}[method]
        _, hist, apps = fn(M, rhs, tol=1e-8 * 0.1, maxiter=20000, prec=prec, **kw)
        say(f"{method} reg={reg} defl={defl} rhs {r}: iters {info[r]['iters']} (oracle {apps}) "
            f"checks {info[r]['cycles']} res {res:.2e} |u - u_lu| {rel(uh[r], u_lu[r]):.2e}")
        assert info[r]["status"] == 0 and res <= 1.02e-8 and rel(uh[r], u_lu[r]) < 2e-5
        assert info[r]["iters"] <= 2 * apps + 40
    assert rc == 0
    s.close()


@pytest.mark.parametrize("method", ["bicgstab", "gcr", "idrs"])
def test_alt_solvers_tm_and_full_system(method):
    g = centred_grid(20, 0.9, ny=18)
    eps = cylinder(g, 0.3, -6.0 + 1.0j)
    btm = np.stack([sy.plane_wave_tm(g, 0.3)])[:, None]
    s = api.Solver.from_grid(g, eps, polarization="tm")
    u, rc, info = s.solve(dev(btm), restart=15 if method != "idrs" else 4, max_iters=20000, tol=1e-8, method=method)
    res = np.linalg.norm(btm[0, 0] - sy.apply_operator_tm(g, eps - 1.0, host(u)[0, 0])) / np.linalg.norm(btm[0, 0])
    say(f"{method} TM: iters {info[0]['iters']} res {res:.2e}")
    assert rc == 0 and res <= 1.02e-8
    s.close()
    mu = cylinder(g, 0.3, 1.5 + 0.1j)
    eps2 = cylinder(g, 0.3, 3.0 + 0.3j)
    E = plane_wave(g, 0.4)
    b3 = np.concatenate([E, (E[1] / np.cos(0.4))[None]], axis=0)[None]
    s3 = api.Solver.from_grid(g, eps2, magnetic=True, mu_r=mu, regularize=True)
    u3, rc3, info3 = s3.solve(dev(b3), restart=15 if method != "idrs" else 4, max_iters=20000, tol=1e-8,
                              method=method)
    res3 = np.linalg.norm(b3[0] - sy.apply_operator_full(g, eps2 - 1.0, mu - 1.0, host(u3)[0])) / np.linalg.norm(b3[0])
    say(f"{method} full system: iters {info3[0]['iters']} res {res3:.2e}")
    assert rc3 == 0 and res3 <= 1.02e-8
    s3.close()


@pytest.mark.parametrize("method", ["bicgstab", "idrs"])
def test_alt_solver_replaces_a_bad_guess(method):
    g, eps, b = _case()
    s = api.Solver.from_grid(g, eps)
    x0 = np.full_like(b, np.nan)
    x0[1] = 10.0 * b[1]
    u, rc, info = s.solve(dev(b), x0=dev(x0), restart=4, max_iters=20000, tol=1e-8, method=method)
    uh = host(u)
    for r in range(2):
        assert info[r]["status"] == 0 and op.relative_residual(g, eps, uh[r], b[r]) <= 1.02e-8
    s.close()


def test_alt_solver_option_checks():
    g, eps, b = _case()
    s = api.Solver.from_grid(g, eps)
    with pytest.raises(api._lib.DieTeError):
        s.solve(dev(b), method="bicgstab", mixed=1)
    with pytest.raises(api._lib.DieTeError):
        s.solve(dev(b), method="gcr", block=1)
    with pytest.raises(api._lib.DieTeError):
        s.solve(dev(b), method="idrs", restart=65)
    with pytest.raises(ValueError):
        s.solve(dev(b), method="qmr")
    s.close()
