// Host FP64 evaluation of the discretised Green tensor of the 2-D operators.
//
// TE electric block.  For a cell separation d = (dx, dy) h != 0, r = |d|, theta = d / r, z = k r,
//   T_lq(d) = k^2 h^2 [ c_theta(z) theta_l theta_q + c_delta(z) delta_lq ],
//   c_theta(z) = i/(2z) H1(z) - i/4 H0(z),   c_delta(z) = i/4 H0(z) - i/(4z) H1(z),
// and for the self cell (the disc of equal area, radius a = h / sqrt(pi))
//   T(0) = [(i pi k a / 4) H1(k a) - 1] I,
// so that the matrix of the collocation system is A = I - T diag(chi)
// (Section 4, eq. A11 and the element formulas that follow it).
// Scalar kernel (TM, and the H3-H3 block of the full TE system; the [A33] formulas):
//   T33(d) = k^2 h^2 (i/4) H0(k r),   T33(0) = (i pi k a / 2) H1(k a) - 1.
// Coupling of E and H3 (eps_b = mu_b = 1, omega = k; Section 3, the compact kernels K13..K32):
//   T13(d) = T31(d) = (k^2 h^2 / 4) H1(k r) theta_2,   T23(d) = T32(d) = -(k^2 h^2 / 4) H1(k r) theta_1,
// zero on the self cell.  The symbol is therefore symmetric at every frequency.
// Hankel functions of the first kind are formed from the C library's double-precision
// Bessel functions: H_n = J_n + i Y_n.
#pragma once
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

namespace die {
namespace green {

using cd = std::complex<double>;

inline void hankel01(double z, cd* h0, cd* h1) {
  *h0 = cd(::j0(z), ::y0(z));
  *h1 = cd(::j1(z), ::y1(z));
}

// T11, T12, T22 at separation (dx, dy) in cell units (not both zero).
inline void tensor(int dx, int dy, double h, double k, cd* t11, cd* t12, cd* t22) {
  const double ex = (double)dx, ey = (double)dy;
  const double rc = std::sqrt(ex * ex + ey * ey);  // in cells
  const double th1 = ex / rc, th2 = ey / rc;
  const double z = k * h * rc;
  cd H0, H1;
  hankel01(z, &H0, &H1);
  const cd I(0.0, 1.0);
  const cd ct = I / (2.0 * z) * H1 - 0.25 * I * H0;
  const cd cdl = 0.25 * I * H0 - I / (4.0 * z) * H1;
  const double s = k * k * h * h;
  *t11 = s * (ct * th1 * th1 + cdl);
  *t12 = s * (ct * th1 * th2);
  *t22 = s * (ct * th2 * th2 + cdl);
}

inline cd self_term(double h, double k) {
  const double a = h / std::sqrt(M_PI);
  cd H0, H1;
  hankel01(k * a, &H0, &H1);
  return cd(0.0, 0.25 * M_PI * k * a) * H1 - 1.0;
}

// The scalar kernel's self term and, at (dx, dy) != 0, the scalar and coupling kernels.
inline cd scalar_self_term(double h, double k) {
  const double a = h / std::sqrt(M_PI);
  cd H0, H1;
  hankel01(k * a, &H0, &H1);
  return cd(0.0, 0.5 * M_PI * k * a) * H1 - 1.0;
}
inline void scalar_and_coupling(int dx, int dy, double h, double k, cd* t33, cd* t13, cd* t23) {
  const double ex = (double)dx, ey = (double)dy;
  const double rc = std::sqrt(ex * ex + ey * ey);
  const double z = k * h * rc;
  cd H0, H1;
  hankel01(z, &H0, &H1);
  const double s = k * k * h * h;
  *t33 = s * cd(0.0, 0.25) * H0;
  *t13 = 0.25 * s * H1 * (ey / rc);
  *t23 = -0.25 * s * H1 * (ex / rc);
}

// Circulant embedding of the kernel planes for ncomp field components in a px x py grid:
// E_c[iy][ix] = T_c(dx(ix), dy(iy)) with dx(ix) = ix for ix < nx, ix - px for
// ix > px - nx, and 0 for the unused wrap-around gap (same for y).  Row-major
// [planes][py][px], interleaved complex; planes: T33 (ncomp 1, TM); T11, T12, T22 (2);
// T11, T12, T22, T13, T23, T33 (3).  Each kernel is evaluated once per non-negative
// separation and reflected: T11, T22, T33 are even in dx and in dy, T12 is odd in each,
// T13 odd in dy, T23 odd in dx.
inline void embed(int nx, int ny, int px, int py, double h, double k, int ncomp, std::vector<cd>& out) {
  const int npl = ncomp == 1 ? 1 : (ncomp == 2 ? 3 : 6);
  out.assign((size_t)npl * px * py, cd(0.0, 0.0));
  const size_t plane = (size_t)px * py;
  const cd ts = self_term(h, k), ts33 = scalar_self_term(h, k);
  unsigned nth = std::thread::hardware_concurrency();
  if (nth == 0) nth = 1;
  if (nth > 32) nth = 32;
  if ((size_t)nx * ny < 4096) nth = 1;
  auto work = [&](int dy0, int dy1) {
    for (int dy = dy0; dy < dy1; ++dy) {
      for (int dx = 0; dx < nx; ++dx) {
        cd t11 = 0.0, t12 = 0.0, t22 = 0.0, t13 = 0.0, t23 = 0.0, t33 = 0.0;
        if (dx == 0 && dy == 0) {
          t11 = ts; t22 = ts; t33 = ts33;
        } else {
          if (ncomp >= 2) tensor(dx, dy, h, k, &t11, &t12, &t22);
          if (ncomp != 2) scalar_and_coupling(dx, dy, h, k, &t33, &t13, &t23);
        }
        for (int sy = 0; sy < 2; ++sy) {
          if (sy == 1 && dy == 0) continue;
          const int iy = sy == 0 ? dy : py - dy;
          for (int sx = 0; sx < 2; ++sx) {
            if (sx == 1 && dx == 0) continue;
            const int ix = sx == 0 ? dx : px - dx;
            const double sgn = (sx ^ sy) ? -1.0 : 1.0;
            const size_t o = (size_t)iy * px + ix;
            if (ncomp == 1) {
              out[o] = t33;
              continue;
            }
            out[o] = t11;
            out[plane + o] = sgn * t12;
            out[2 * plane + o] = t22;
            if (ncomp == 3) {
              out[3 * plane + o] = (sy ? -1.0 : 1.0) * t13;
              out[4 * plane + o] = (sx ? -1.0 : 1.0) * t23;
              out[5 * plane + o] = t33;
            }
          }
        }
      }
    }
  };
  if (nth == 1) {
    work(0, ny);
  } else {
    std::vector<std::thread> ths;
    const int chunk = (ny + (int)nth - 1) / (int)nth;
    for (unsigned t = 0; t < nth; ++t) {
      const int a = (int)t * chunk, b = std::min(ny, a + chunk);
      if (a < b) ths.emplace_back(work, a, b);
    }
    for (auto& th : ths) th.join();
  }
}

}  // namespace green
}  // namespace die
