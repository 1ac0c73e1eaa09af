"""Host dense algebra of the block solver (dense.hpp), compiled with g++ and checked against
numpy: rank-revealing pivoted Cholesky of a Gram matrix, the scaled Cholesky QR factor with its
smallest scaled pivot, the upper triangular inverse and the product of upper triangular matrices."""
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
int main(int argc, char** argv) {
  int k; double tau2;
  if (std::scanf("%d %lf", &k, &tau2) != 2) return 1;
  Mat G(k, k);
  for (int j = 0; j < k; ++j) for (int i = 0; i < k; ++i) { double re, im; std::scanf("%lf %lf", &re, &im); G(i, j) = cd(re, im); }
  Mat L; std::vector<int> perm;
  const int p = pivoted_cholesky(G, tau2, L, perm);
  std::printf("%d\n", p);
  for (int i = 0; i < k; ++i) std::printf("%d ", perm[i]);
  std::printf("\n");
  for (int j = 0; j < k; ++j) for (int i = 0; i < k; ++i) std::printf("%.17g %.17g\n", L(i, j).real(), L(i, j).imag());
  Mat R;
  const bool ok = chol_upper_scaled(G, 1e-13, R);
  std::printf("%d\n", ok ? 1 : 0);
  if (ok) {
    Mat X = upper_inverse(R);
    for (int j = 0; j < k; ++j) for (int i = 0; i < k; ++i) std::printf("%.17g %.17g\n", R(i, j).real(), R(i, j).imag());
    for (int j = 0; j < k; ++j) for (int i = 0; i < k; ++i) std::printf("%.17g %.17g\n", X(i, j).real(), X(i, j).imag());
    Mat R2; double mp = -1.0;
    chol_upper_scaled(G, 1e-13, R2, &mp);
    std::printf("%.17g\n", mp);
    Mat P = upper_product(R, R);
    for (int j = 0; j < k; ++j) for (int i = 0; i < k; ++i) std::printf("%.17g %.17g\n", P(i, j).real(), P(i, j).imag());
  }
  return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    d = tmp_path_factory.mktemp("dense")
    src = d / "drv.cpp"
    src.write_text(DRIVER)
    exe = d / "drv"
    subprocess.run(["g++", "-O1", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


def run(exe, G, tau2):
    k = G.shape[0]
    lines = [f"{k} {float(tau2)!r}"] + [f"{float(G[i, j].real)!r} {float(G[i, j].imag)!r}" for j in range(k) for i in range(k)]
    out = subprocess.run([exe], input="\n".join(lines), capture_output=True, text=True, check=True).stdout.split("\n")
    p = int(out[0])
    perm = [int(v) for v in out[1].split()]
    vals = [complex(*map(float, ln.split())) for ln in out[2:2 + k * k]]
    L = np.array(vals).reshape(k, k).T
    ok = out[2 + k * k] == "1"
    R = X = None
    run.extra = None
    if ok:
        base = 3 + k * k
        R = np.array([complex(*map(float, ln.split())) for ln in out[base:base + k * k]]).reshape(k, k).T
        X = np.array([complex(*map(float, ln.split())) for ln in out[base + k * k:base + 2 * k * k]]).reshape(k, k).T
        mp = float(out[base + 2 * k * k])
        P = np.array([complex(*map(float, ln.split())) for ln in out[base + 2 * k * k + 1:base + 3 * k * k + 1]])
        run.extra = (mp, P.reshape(k, k).T)
    return p, perm, L, ok, R, X


def test_full_rank_gram(driver):
    rng = np.random.default_rng(0)
    A = rng.standard_normal((40, 6)) + 1j * rng.standard_normal((40, 6))
    A[:, 2] *= 1e-3  # a short column: the scaled factorisation must not mind
    G = A.conj().T @ A
    p, perm, L, ok, R, X = run(driver, G, 1e-30)
    assert p == 6 and sorted(perm) == list(range(6))
    Gp = G[np.ix_(perm, perm)]
    assert np.allclose(L @ L.conj().T, Gp, rtol=0, atol=1e-12 * np.abs(G).max())
    assert ok
    assert np.allclose(np.triu(R), R)
    assert np.allclose(R.conj().T @ R, G, rtol=0, atol=1e-12 * np.abs(G).max())
    assert np.allclose(X @ R, np.eye(6), atol=1e-10)
    # smallest pivot of the unit-diagonal Gram's Cholesky, and the triangular product R R
    mp, P = run.extra
    d = 1.0 / np.sqrt(np.diag(G).real)
    S = G * d[:, None] * d[None, :]
    piv = np.diag(np.linalg.cholesky(S)).real ** 2
    assert abs(mp - piv.min()) <= 1e-12
    assert np.allclose(P, R @ R, rtol=0, atol=1e-12 * np.abs(R @ R).max())
    assert np.allclose(np.tril(P, -1), 0)


def test_rank_deficient_gram_selects_independent_columns(driver):
    rng = np.random.default_rng(1)
    B = rng.standard_normal((50, 3)) + 1j * rng.standard_normal((50, 3))
    A = np.column_stack([B[:, 0], B[:, 1], B[:, 0] + 2 * B[:, 1], B[:, 2], 3j * B[:, 2]])
    A /= np.linalg.norm(A, axis=0)
    G = A.conj().T @ A
    p, perm, L, ok, _, _ = run(driver, G, 1e-12)
    assert p == 3  # rank 3
    sel = perm[:3]
    assert np.linalg.matrix_rank(A[:, sel]) == 3
    # every column's projection onto the selected span is reproduced: G[perm][perm] = L L^H
    Gp = G[np.ix_(perm, perm)]
    Lp = L[:, :p]
    assert np.allclose(Lp @ Lp.conj().T, Gp, atol=1e-10)
    assert not ok  # the plain factorisation reports the rank deficiency
