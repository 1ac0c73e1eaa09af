// Small dense complex linear algebra on the host (FP64) for the offline
// eigensolver: Householder reduction to Hessenberg form, the shifted QR
// algorithm to complex Schur form, reordering of the Schur form, eigenvectors
// of a triangular matrix, and an LU inverse.  Matrices are column-major.
#pragma once
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

namespace die {
namespace la {

using cd = std::complex<double>;

struct Mat {
  int n = 0, m = 0;  // rows, cols
  std::vector<cd> a;
  Mat() = default;
  Mat(int rows, int cols) : n(rows), m(cols), a((size_t)rows * cols, cd(0.0, 0.0)) {}
  cd& operator()(int i, int j) { return a[(size_t)j * n + i]; }
  const cd& operator()(int i, int j) const { return a[(size_t)j * n + i]; }
  static Mat eye(int k) {
    Mat e(k, k);
    for (int i = 0; i < k; ++i) e(i, i) = 1.0;
    return e;
  }
};

// Rotation G = [[c, s], [-conj(s), c]] with G [a; b] = [r; 0].
inline void givens(cd a, cd b, double* c, cd* s, cd* r) {
  const double aa = std::abs(a), bb = std::abs(b);
  if (bb == 0.0) { *c = 1.0; *s = 0.0; *r = a; return; }
  if (aa == 0.0) { *c = 0.0; *s = std::conj(b) / bb; *r = bb; return; }
  const double rho = std::hypot(aa, bb);
  *c = aa / rho;
  *s = (a / aa) * std::conj(b) / rho;
  *r = (a / aa) * rho;
}

// rows k, k+1 of H (columns j0..j1-1) <- G rows
inline void rot_rows(Mat& H, int k, double c, cd s, int j0, int j1) {
  for (int j = j0; j < j1; ++j) {
    const cd t1 = H(k, j), t2 = H(k + 1, j);
    H(k, j) = c * t1 + s * t2;
    H(k + 1, j) = -std::conj(s) * t1 + c * t2;
  }
}
// columns k, k+1 of H (rows i0..i1-1) <- times G^H
inline void rot_cols(Mat& H, int k, double c, cd s, int i0, int i1) {
  for (int i = i0; i < i1; ++i) {
    const cd t1 = H(i, k), t2 = H(i, k + 1);
    H(i, k) = c * t1 + std::conj(s) * t2;
    H(i, k + 1) = -s * t1 + c * t2;
  }
}

// A (n x n) -> Q H Q^H with H upper Hessenberg (Householder); Q accumulated into Z (Z <- Z Q).
inline void hessenberg(Mat& A, Mat& Z) {
  const int n = A.n;
  std::vector<cd> v(n);
  for (int k = 0; k + 2 < n + 0 && k < n - 2; ++k) {
    // the column is scaled by its largest entry before any squaring: entries as small as the
    // ones a Krylov-Schur restart leaves for converged directions (1e-200 and below) would
    // otherwise underflow in |x|^2 and overflow in 2 / |v|^2
    double scale = 0.0;
    for (int i = k + 1; i < n; ++i) scale = std::max(scale, std::abs(A(i, k)));
    if (scale == 0.0) continue;
    double alpha2 = 0.0;
    for (int i = k + 1; i < n; ++i) alpha2 += std::norm(A(i, k) / scale);
    const double anorm = std::sqrt(alpha2);  // |x| / scale
    const cd x0 = A(k + 1, k);
    const cd ph = std::abs(x0) > 0 ? x0 / std::abs(x0) : cd(1.0, 0.0);
    // v = x / scale + ph |x / scale| e1, H = I - 2 v v^H / (v^H v) (independent of the scale)
    for (int i = 0; i < n; ++i) v[i] = 0.0;
    for (int i = k + 1; i < n; ++i) v[i] = A(i, k) / scale;
    v[k + 1] += ph * anorm;
    double vn = 0.0;
    for (int i = k + 1; i < n; ++i) vn += std::norm(v[i]);
    if (vn == 0.0) continue;
    const double tau = 2.0 / vn;
    // A <- H A
    for (int j = 0; j < n; ++j) {
      cd s = 0.0;
      for (int i = k + 1; i < n; ++i) s += std::conj(v[i]) * A(i, j);
      s *= tau;
      for (int i = k + 1; i < n; ++i) A(i, j) -= v[i] * s;
    }
    // A <- A H, Z <- Z H
    for (int i = 0; i < n; ++i) {
      cd s = 0.0;
      for (int j = k + 1; j < n; ++j) s += A(i, j) * v[j];
      s *= tau;
      for (int j = k + 1; j < n; ++j) A(i, j) -= s * std::conj(v[j]);
    }
    for (int i = 0; i < Z.n; ++i) {
      cd s = 0.0;
      for (int j = k + 1; j < n; ++j) s += Z(i, j) * v[j];
      s *= tau;
      for (int j = k + 1; j < n; ++j) Z(i, j) -= s * std::conj(v[j]);
    }
    for (int i = k + 2; i < n; ++i) A(i, k) = 0.0;
  }
}

// Hessenberg H -> upper triangular T = Z^H H Z by single-shift QR with Wilkinson
// shifts (and an exceptional shift when a block stalls).  Z <- Z * (rotations).
// Returns false if it did not converge within 60 n sweeps.
inline bool schur(Mat& H, Mat& Z) {
  const int n = H.n;
  const double eps = 2.220446049250313e-16;
  int hi = n - 1;
  int iter = 0, since = 0;
  const int maxit = 60 * std::max(n, 1);
  while (hi > 0) {
    if (iter++ > maxit) return false;
    int l = hi;
    while (l > 0) {
      const double s = std::abs(H(l, l)) + std::abs(H(l - 1, l - 1));
      if (std::abs(H(l, l - 1)) <= eps * (s > 0 ? s : 1.0)) { H(l, l - 1) = 0.0; break; }
      --l;
    }
    if (l == hi) { --hi; since = 0; continue; }
    ++since;
    cd mu;
    if (since % 11 == 10) {
      mu = H(hi, hi) + 0.75 * std::abs(H(hi, hi - 1));
    } else {
      const cd a = H(hi - 1, hi - 1), b = H(hi - 1, hi), c = H(hi, hi - 1), d = H(hi, hi);
      const cd tr = a + d, det = a * d - b * c;
      const cd disc = std::sqrt(tr * tr / 4.0 - det);
      const cd e1 = tr / 2.0 + disc, e2 = tr / 2.0 - disc;
      mu = std::abs(e1 - d) < std::abs(e2 - d) ? e1 : e2;
    }
    cd x = H(l, l) - mu, y = H(l + 1, l);
    for (int k = l; k < hi; ++k) {
      double c; cd s, r;
      givens(x, y, &c, &s, &r);
      rot_rows(H, k, c, s, k > l ? k - 1 : l, n);
      rot_cols(H, k, c, s, 0, std::min(k + 3, hi + 1));
      rot_cols(Z, k, c, s, 0, Z.n);
      if (k > l) H(k + 1, k - 1) = 0.0;
      if (k + 1 < hi) { x = H(k + 1, k); y = H(k + 2, k); }
    }
  }
  for (int j = 0; j < n; ++j)
    for (int i = j + 1; i < n; ++i) H(i, j) = 0.0;
  return true;
}

// Swap the adjacent diagonal entries T(i,i), T(i+1,i+1) of the upper triangular T.
inline void schur_swap(Mat& T, Mat& Z, int i) {
  const int n = T.n;
  const cd a = T(i, i), b = T(i + 1, i + 1), t = T(i, i + 1);
  double c; cd s, r;
  givens(t, b - a, &c, &s, &r);  // G [t; b - a] = [r; 0]: the eigenvector of b goes first
  rot_rows(T, i, c, s, i, n);
  rot_cols(T, i, c, s, 0, i + 2);
  rot_cols(Z, i, c, s, 0, Z.n);
  T(i + 1, i) = 0.0;
  T(i, i) = b;
  T(i + 1, i + 1) = a;
}

// Move the entries flagged in `want` (by current diagonal position) to the leading
// positions, keeping their relative order.
inline void reorder(Mat& T, Mat& Z, std::vector<char> want) {
  int dest = 0;
  for (int k = 0; k < T.n; ++k) {
    if (!want[k]) continue;
    for (int p = k; p > dest; --p) {
      schur_swap(T, Z, p - 1);
      std::swap(want[p], want[p - 1]);
    }
    ++dest;
  }
}

// Eigenvector y_k of upper triangular T for T(k,k): y_k(k) = 1, zero below k; columns of Y.
inline Mat tri_eigvecs(const Mat& T) {
  const int n = T.n;
  Mat Y(n, n);
  double tn = 0.0;
  for (auto& v : T.a) tn = std::max(tn, std::abs(v));
  const double small = 1e-14 * (tn > 0 ? tn : 1.0);
  for (int k = 0; k < n; ++k) {
    const cd lam = T(k, k);
    Y(k, k) = 1.0;
    for (int i = k - 1; i >= 0; --i) {
      cd s = 0.0;
      for (int j = i + 1; j <= k; ++j) s += T(i, j) * Y(j, k);
      cd d = T(i, i) - lam;
      if (std::abs(d) < small) d = small;
      Y(i, k) = -s / d;
      // through a cluster of close eigenvalues the entries grow by |T(i, j) / d| per step: the
      // partial vector is rescaled before it can overflow (the normalisation below removes it)
      const double a = std::abs(Y(i, k));
      if (a > 1e100)
        for (int j = i; j <= k; ++j) Y(j, k) /= a;
    }
    double nrm = 0.0;
    for (int i = 0; i <= k; ++i) nrm += std::norm(Y(i, k));
    nrm = std::sqrt(nrm);
    for (int i = 0; i <= k; ++i) Y(i, k) /= nrm;
  }
  return Y;
}

// Cholesky G = L L^H of a Hermitian matrix (lower triangle of G read); false when a pivot is
// not above rel_tol times the largest diagonal entry (numerically rank deficient).
inline bool cholesky(const Mat& G, Mat& L, double rel_tol, double* min_pivot = nullptr) {
  const int k = G.n;
  double dmax = 0.0;
  for (int i = 0; i < k; ++i) dmax = std::max(dmax, G(i, i).real());
  if (!(dmax > 0.0)) return false;
  // row-major working copy, so that every inner product below runs over contiguous memory;
  // the complex multiply-adds are written out (finite values only)
  std::vector<cd> Lr((size_t)k * k, cd(0.0, 0.0));
  double dmin = 1.0;
  for (int j = 0; j < k; ++j) {
    const cd* lj = &Lr[(size_t)j * k];
    double d = G(j, j).real();
    for (int q = 0; q < j; ++q) d -= lj[q].real() * lj[q].real() + lj[q].imag() * lj[q].imag();
    if (!(d > rel_tol * dmax)) return false;
    dmin = std::min(dmin, d / dmax);
    const double ljj = std::sqrt(d);
    Lr[(size_t)j * k + j] = ljj;
    for (int i = j + 1; i < k; ++i) {
      const cd* li = &Lr[(size_t)i * k];
      double sr = G(i, j).real(), si = G(i, j).imag();
      for (int q = 0; q < j; ++q) {  // s -= L(i, q) conj(L(j, q))
        sr -= li[q].real() * lj[q].real() + li[q].imag() * lj[q].imag();
        si -= li[q].imag() * lj[q].real() - li[q].real() * lj[q].imag();
      }
      Lr[(size_t)i * k + j] = cd(sr / ljj, si / ljj);
    }
  }
  L = Mat(k, k);
  for (int j = 0; j < k; ++j)
    for (int i = j; i < k; ++i) L(i, j) = Lr[(size_t)i * k + j];
  if (min_pivot) *min_pivot = dmin;
  return true;
}

// Pivoted Cholesky of a Hermitian positive semidefinite G: with rows of L in pivot order,
// G(perm[i], perm[j]) = sum_q L(i, q) conj(L(j, q)) for the leading p pivots, L (k x k, lower
// trapezoidal in its first p columns).  Stops when the largest remaining diagonal entry is
// not above tau2; returns the rank p.
inline int pivoted_cholesky(const Mat& G, double tau2, Mat& L, std::vector<int>& perm) {
  const int k = G.n;
  L = Mat(k, k);
  perm.resize(k);
  for (int i = 0; i < k; ++i) perm[i] = i;
  std::vector<double> d(k);
  for (int i = 0; i < k; ++i) d[i] = G(i, i).real();
  int p = 0;
  for (; p < k; ++p) {
    int q = p;
    for (int i = p + 1; i < k; ++i)
      if (d[perm[i]] > d[perm[q]]) q = i;
    if (!(d[perm[q]] > tau2)) break;
    if (q != p) {
      std::swap(perm[p], perm[q]);
      for (int c = 0; c < p; ++c) std::swap(L(p, c), L(q, c));
    }
    const int jp = perm[p];
    const double ljj = std::sqrt(d[jp]);
    L(p, p) = ljj;
    for (int i = p + 1; i < k; ++i) {
      const int ji = perm[i];
      cd s = G(ji, jp);
      for (int c = 0; c < p; ++c) s -= L(i, c) * std::conj(L(p, c));
      L(i, p) = s / ljj;
      d[ji] -= std::norm(L(i, p));
    }
  }
  return p;
}

// Inverse of the upper triangular R (non-zero diagonal).
inline Mat upper_inverse(const Mat& R) {
  const int k = R.n;
  // rows of R contiguous, columns of X contiguous: each entry is one contiguous inner product
  std::vector<cd> Rr((size_t)k * k), rd(k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j; ++i) Rr[(size_t)i * k + j] = R(i, j);
  for (int i = 0; i < k; ++i) {
    const cd r = R(i, i);
    const double m = r.real() * r.real() + r.imag() * r.imag();
    rd[i] = cd(r.real() / m, -r.imag() / m);  // 1 / R(i, i)
  }
  Mat X(k, k);
  for (int j = 0; j < k; ++j) {
    cd* xj = &X.a[(size_t)j * k];
    xj[j] = rd[j];
    for (int i = j - 1; i >= 0; --i) {
      const cd* ri = &Rr[(size_t)i * k];
      double sr = 0.0, si = 0.0;
      for (int q = i + 1; q <= j; ++q) {
        sr += ri[q].real() * xj[q].real() - ri[q].imag() * xj[q].imag();
        si += ri[q].real() * xj[q].imag() + ri[q].imag() * xj[q].real();
      }
      // X(i, j) = -s / R(i, i)
      xj[i] = cd(-(sr * rd[i].real() - si * rd[i].imag()), -(sr * rd[i].imag() + si * rd[i].real()));
    }
  }
  return X;
}

// Product of two upper triangular matrices (k x k): C = A B, upper triangular.
inline Mat upper_product(const Mat& A, const Mat& B) {
  const int k = A.n;
  std::vector<cd> Ar((size_t)k * k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j; ++i) Ar[(size_t)i * k + j] = A(i, j);
  Mat C(k, k);
  for (int j = 0; j < k; ++j) {
    const cd* bj = &B.a[(size_t)j * k];
    for (int i = 0; i <= j; ++i) {
      const cd* ai = &Ar[(size_t)i * k];
      double sr = 0.0, si = 0.0;
      for (int q = i; q <= j; ++q) {
        sr += ai[q].real() * bj[q].real() - ai[q].imag() * bj[q].imag();
        si += ai[q].real() * bj[q].imag() + ai[q].imag() * bj[q].real();
      }
      C(i, j) = cd(sr, si);
    }
  }
  return C;
}

// G = R^H R with R upper triangular, from the Cholesky factor of the unit-diagonal scaling
// D G D (D = diag(G)^-1/2), so that the rank test rel_tol is relative to each column's own
// norm; false when a column vanishes or the scaled matrix is numerically rank deficient.
inline bool chol_upper_scaled(const Mat& G, double rel_tol, Mat& R, double* min_pivot = nullptr) {
  const int k = G.n;
  std::vector<double> dinv(k);
  for (int i = 0; i < k; ++i) {
    const double d = G(i, i).real();
    if (!(d > 0.0) || !std::isfinite(d)) return false;
    dinv[i] = 1.0 / std::sqrt(d);
  }
  Mat S(k, k);
  for (int j = 0; j < k; ++j)
    for (int i = 0; i < k; ++i) S(i, j) = G(i, j) * dinv[i] * dinv[j];
  Mat L;
  if (!cholesky(S, L, rel_tol, min_pivot)) return false;
  R = Mat(k, k);  // R = L^H D^-1
  for (int j = 0; j < k; ++j)
    for (int i = 0; i <= j; ++i) R(i, j) = std::conj(L(j, i)) / dinv[j];
  return true;
}

// Inverse by LU with partial pivoting; false if singular.
inline bool inverse(const Mat& A, Mat& Ainv) {
  const int n = A.n;
  Mat L = A;
  std::vector<int> piv(n);
  for (int k = 0; k < n; ++k) {
    int p = k;
    double best = std::abs(L(k, k));
    for (int i = k + 1; i < n; ++i)
      if (std::abs(L(i, k)) > best) { best = std::abs(L(i, k)); p = i; }
    if (best == 0.0) return false;
    piv[k] = p;
    if (p != k)
      for (int j = 0; j < n; ++j) std::swap(L(k, j), L(p, j));
    for (int i = k + 1; i < n; ++i) {
      L(i, k) /= L(k, k);
      for (int j = k + 1; j < n; ++j) L(i, j) -= L(i, k) * L(k, j);
    }
  }
  Ainv = Mat::eye(n);
  for (int k = 0; k < n; ++k)
    if (piv[k] != k)
      for (int j = 0; j < n; ++j) std::swap(Ainv(k, j), Ainv(piv[k], j));
  for (int j = 0; j < n; ++j) {
    for (int i = 0; i < n; ++i)
      for (int l = 0; l < i; ++l) Ainv(i, j) -= L(i, l) * Ainv(l, j);
    for (int i = n - 1; i >= 0; --i) {
      for (int l = i + 1; l < n; ++l) Ainv(i, j) -= L(i, l) * Ainv(l, j);
      Ainv(i, j) /= L(i, i);
    }
  }
  return true;
}

}  // namespace la
}  // namespace die
