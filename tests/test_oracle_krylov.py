"""Pins of the oracle's Bi-CGSTAB, GCR and IDR(s) (oracle/krylov.py), which the GPU solvers are
checked against: SciPy's Bi-CGSTAB (the same algorithm) produces the same iterates; finite
termination on a matrix with few distinct eigenvalues; GCR with every direction kept has full
GMRES's minimal residuals; restarted GCR never increases the residual; IDR(s) terminates within
n + n/s operator applications (the IDR theorem); right preconditioning solves the original
system."""
import numpy as np
import pytest

from oracle import krylov

scipy_sparse = pytest.importorskip("scipy.sparse.linalg")


def _matrix(n=60, seed=0, shift=4.0):
    rng = np.random.default_rng(seed)
    A = (rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))) / np.sqrt(n)
    return A + shift * np.eye(n), rng.standard_normal(n) + 1j * rng.standard_normal(n)


def test_bicgstab_iterates_match_scipy():
    A, b = _matrix()
    xs = []
    scipy_sparse.bicgstab(A, b, rtol=1e-14, atol=0.0, maxiter=8, callback=lambda xk: xs.append(xk.copy()))
    for k in range(1, 6):
        x, hist, apps = krylov.bicgstab(A, b, tol=0.0, maxiter=k)
        assert apps == 2 * k
        assert np.linalg.norm(x - xs[k - 1]) <= 1e-10 * np.linalg.norm(xs[k - 1])


@pytest.mark.parametrize("solver", ["bicgstab", "gcr"])
def test_finite_termination_on_four_distinct_eigenvalues(solver):
    rng = np.random.default_rng(1)
    d = np.repeat([1.0, 2.0 + 1j, -3.0, 0.5j], 10)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40)))
    A = Q @ np.diag(d) @ Q.conj().T  # normal, four distinct eigenvalues
    b = rng.standard_normal(40) + 1j * rng.standard_normal(40)
    x, hist, apps = getattr(krylov, solver)(A, b, tol=1e-12, maxiter=10)
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
    assert len(hist) - 1 <= 4  # iterations


def test_gcr_full_memory_has_gmres_residuals():
    A, b = _matrix(seed=2, shift=1.5)
    _, hist, _ = krylov.gcr(A, b, tol=0.0, maxiter=25)
    ref = krylov.gmres_residuals(A, b, 25)
    assert np.allclose(hist, ref[: len(hist)], rtol=1e-8, atol=1e-12 * ref[0])


def test_restarted_gcr_is_monotone_and_converges():
    A, b = _matrix(seed=3, shift=2.0)
    x, hist, _ = krylov.gcr(A, b, tol=1e-10, maxiter=500, restart=5)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    assert np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)


@pytest.mark.parametrize("solver", ["bicgstab", "gcr"])
def test_right_preconditioning_solves_the_original_system(solver):
    A, b = _matrix(seed=4, shift=3.0)
    rng = np.random.default_rng(5)
    Pinv = np.eye(60) + 0.1 * (rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))) / np.sqrt(60)
    x, _, _ = getattr(krylov, solver)(A, b, tol=1e-12, maxiter=400, prec=lambda v: Pinv @ v)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("s", [2, 3, 4, 6])
def test_idrs_terminates_within_n_plus_n_over_s(s):
    # the IDR theorem (Sonneveld and van Gijzen): the residual spaces shrink by s dimensions every
    # s + 1 steps, so in exact arithmetic IDR(s) reaches the zero residual within n + n / s
    # applications of the operator; on a well-conditioned matrix rounding does not delay it
    rng = np.random.default_rng(12 * 10 + s)
    n = 12
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 6.0 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    x, hist, apps = krylov.idrs(A, b, s=s, tol=0.0, maxiter=n + n // s)
    assert apps == n + n // s
    assert hist[-1] <= 1e-9 * np.linalg.norm(b) and np.linalg.norm(A @ x - b) <= 1e-9 * np.linalg.norm(b)
    assert hist[n // 2] > 1e-6 * np.linalg.norm(b)  # and not by accident much earlier


def test_idrs_converges_with_a_right_preconditioner():
    A, b = _matrix(seed=7, shift=3.0)
    rng = np.random.default_rng(8)
    Pinv = np.eye(60) + 0.1 * (rng.standard_normal((60, 60)) + 1j * rng.standard_normal((60, 60))) / np.sqrt(60)
    x, hist, apps = krylov.idrs(A, b, s=4, tol=1e-12, maxiter=400, prec=lambda v: Pinv @ v)
    assert np.linalg.norm(A @ x - b) <= 1e-10 * np.linalg.norm(b)
