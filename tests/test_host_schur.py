"""Host Schur decomposition of the eigensolver (dense.hpp), compiled with g++ and checked against
LAPACK through numpy and against its own backward error (A = Z T Z*, Z unitary, T triangular):
a random matrix, the bordered triangular pattern a Krylov-Schur restart produces, and columns
whose subdiagonal entries are so small that an unscaled Householder step overflows (1e-158 made
NaN before the column scaling); and eigenvectors of a triangular matrix through a tight cluster
of eigenvalues, whose back-substitution overflowed before the partial vector was rescaled."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_1104_4263_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <complex>
#include "dense.hpp"
using namespace die::la;
int main() {
  int n, mode;
  if (std::scanf("%d %d", &n, &mode) != 2) return 1;
  Mat A(n, n);
  for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) { double re, im; if (std::scanf("%lf %lf", &re, &im) != 2) return 1; A(i, j) = cd(re, im); }
  if (mode == 0) {
    Mat Z = Mat::eye(n);
    hessenberg(A, Z);
    const bool ok = schur(A, Z);
    std::printf("%d\n", ok ? 1 : 0);
    for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", A(i, j).real(), A(i, j).imag());
    for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", Z(i, j).real(), Z(i, j).imag());
  } else {
    Mat Y = tri_eigvecs(A);
    std::printf("1\n");
    for (int j = 0; j < n; ++j) for (int i = 0; i < n; ++i) std::printf("%.17g %.17g\n", Y(i, j).real(), Y(i, j).imag());
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("schur")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def _run(driver, A, mode):
    n = A.shape[0]
    inp = f"{n} {mode}\n" + "\n".join(f"{A[i, j].real:.17g} {A[i, j].imag:.17g}" for j in range(n) for i in range(n))
    out = subprocess.run([driver], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    ok = out[0].strip() == "1"
    vals = np.array([complex(*map(float, l.split())) for l in out[1:] if l.strip()])
    return ok, vals


def _match(a, b):
    # greedy matching of two multisets of eigenvalues
    b = list(b)
    worst = 0.0
    for x in a:
        k = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[k]))
        b.pop(k)
    return worst


def _schur(driver, A):
    n = A.shape[0]
    ok, v = _run(driver, A, 0)
    T = v[: n * n].reshape(n, n).T
    Z = v[n * n:].reshape(n, n).T
    return ok, T, Z


def _check_schur(A, T, Z):
    """A = Z T Z* with Z unitary and T upper triangular, to a small multiple of rounding."""
    n = A.shape[0]
    nrm = np.linalg.norm(A)
    assert np.all(np.isfinite(T)) and np.all(np.isfinite(Z))
    assert np.linalg.norm(Z.conj().T @ Z - np.eye(n)) <= 1e-13 * n
    assert np.linalg.norm(A - Z @ T @ Z.conj().T) <= 1e-14 * n * nrm
    assert np.linalg.norm(np.tril(T, -1)) <= 1e-15 * n * nrm


def test_schur_random(driver):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 40)) + 1j * rng.standard_normal((40, 40))
    ok, T, Z = _schur(driver, A)
    assert ok
    _check_schur(A, T, Z)
    assert _match(np.diag(T), np.linalg.eigvals(A)) <= 1e-10 * np.abs(A).max()


def test_schur_restart_pattern_with_tiny_border(driver):
    rng = np.random.default_rng(1)
    k, m = 60, 90
    A = np.zeros((m, m), complex)
    T = np.triu(rng.standard_normal((k, k)) + 1j * rng.standard_normal((k, k))) * 0.1
    T[np.arange(k), np.arange(k)] = 1.0 + 0.01 * (rng.standard_normal(k) + 1j * rng.standard_normal(k))
    T[:5, :5] += np.diag([30.0, 25.0, 20.0, 15.0, 10.0])
    A[:k, :k] = T
    A[k, :k] = 10.0 ** rng.uniform(-220, -1, k) * np.exp(2j * np.pi * rng.random(k))  # the bordering row
    B = rng.standard_normal((m, m - k)) + 1j * rng.standard_normal((m, m - k))
    A[:, k:] = np.triu(B, -(k)) * 0.3  # Arnoldi columns after the restart (Hessenberg below)
    for j in range(k, m):
        A[j + 2:, j] = 0.0
    ok, T, Z = _schur(driver, A)
    assert ok
    _check_schur(A, T, Z)
    # the clustered eigenvalues near 1 belong to a far-from-normal block and are ill-conditioned;
    # the five isolated ones are well conditioned and must agree with LAPACK's
    d = np.diag(T)
    for lam in (30.0, 25.0, 20.0, 15.0, 10.0):
        ref = np.linalg.eigvals(A)
        assert abs(d[np.argmin(abs(d - lam))] - ref[np.argmin(abs(ref - lam))]) <= 1e-10 * lam


@pytest.mark.parametrize("tiny", [1e-158, 1e-200, 1e-300])
def test_schur_column_of_tiny_entries(driver, tiny):
    # a first column whose subdiagonal part is ~1e-158 squares into the subnormal range, and
    # 2 / |v|^2 of an unscaled Householder vector then overflows
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 30)) + 1j * rng.standard_normal((30, 30))
    A[1:, 0] = tiny * (rng.standard_normal(29) + 1j * rng.standard_normal(29))
    ok, T, Z = _schur(driver, A)
    assert ok
    _check_schur(A, T, Z)
    d, ref = np.diag(T), np.linalg.eigvals(A)
    assert _match(d, ref) <= 1e-10 * np.abs(A).max()


def test_triangular_eigenvectors_through_a_cluster(driver):
    rng = np.random.default_rng(2)
    n = 120
    T = np.triu(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)), 1)
    lam = 1.0 + 1e-9 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))  # a tight cluster
    lam[:4] = [5.0, 4.0, 3.0, 2.0]
    T[np.arange(n), np.arange(n)] = lam
    ok, y = _run(driver, T, 1)
    Y = y.reshape(n, n).T
    assert np.all(np.isfinite(Y))
    # each column is a unit vector (the eigenvectors of a tight cluster are ill-conditioned, so
    # only the well-separated ones are checked for the eigen-relation)
    assert np.allclose(np.linalg.norm(Y, axis=0), 1.0)
    for k in range(4):
        assert np.linalg.norm(T @ Y[:, k] - lam[k] * Y[:, k]) <= 1e-10 * np.abs(T).max()
