// Deflation size and memory planning of Section 5 (host only).
//
// Deflation radius.  The dense line segments of the spectrum of A run from 1 to eps(x)/eps_b
// (Section 3, eq. EssentialSpectrum); the regularizer maps an eigenvalue lam of a homogeneous
// object to lam' = [1 + (1 - lam)/eps] lam (Section 5, eq. EigenvaluesArA), and the paper takes
// the largest |lam'| over the images of all segments [1, eps(x)] as the radius beyond which
// eigenvalues are deflated.  On the segment lam = 1 + t (eps - 1), t in [0, 1], the image is
// lam' = 1 + a t (1 - t) with a = (eps - 1)^2 / eps; |1 + a s|^2 is a convex quadratic in
// s = t (1 - t) in [0, 1/4], so its largest value is at an end: R(eps) = max(1, |1 + a / 4|)
// (for a lossless eps > 0 this is (1 + eps)^2 / (4 eps), the paper's lossless image).  Without
// the regularizer the segments themselves bound the dense spectrum: R(eps) = max(1, |eps|).
#include <algorithm>
#include <cmath>
#include <complex>

#include "die_te.h"
#include "host.hpp"

namespace die_host {

double deflation_radius(const double2* eps, size_t ncells, bool regularized) {
  double R = 1.0;
  for (size_t e = 0; e < ncells; ++e) {
    const std::complex<double> ep(eps[e].x, eps[e].y);
    const double Re = regularized ? std::abs(1.0 + (ep - 1.0) * (ep - 1.0) / (4.0 * ep)) : std::abs(ep);
    R = std::max(R, Re);
  }
  return R;
}

}  // namespace die_host

extern "C" {

int die_te_deflation_radius(const void* eps_r, long long ncells, int regularized, double* radius) {
  die_host::last_error().clear();
  if (!eps_r || !radius || ncells < 1) return die_host::fail(DIE_E_INVALID, "null argument or ncells < 1");
  const double2* e = static_cast<const double2*>(eps_r);
  for (long long i = 0; i < ncells; ++i)
    if (e[i].x == 0.0 && e[i].y == 0.0)
      return die_host::fail(DIE_E_SINGULAR, "eps_r == 0 at cell " + std::to_string(i));
  *radius = die_host::deflation_radius(e, (size_t)ncells, regularized != 0);
  return DIE_OK;
}

int die_te_plan_memory(double mem_bytes, double beta, double points_per_wavelength, double x, double eps_re_max,
                       die_te_plan* plan) {
  die_host::last_error().clear();
  if (!plan) return die_host::fail(DIE_E_INVALID, "null plan");
  if (!(mem_bytes > 0) || !(beta > 0) || !(points_per_wavelength > 0) || !(x > 0) || !(eps_re_max > 0) ||
      !std::isfinite(mem_bytes) || !std::isfinite(beta) || !std::isfinite(x) || !std::isfinite(eps_re_max))
    return die_host::fail(DIE_E_INVALID, "every planning input must be positive and finite");
  die_te_plan p{};
  p.alpha = points_per_wavelength * std::sqrt(eps_re_max);
  // M_A + M_prec = 720 N + 144 (beta^2 + beta + x beta) N^2 = M, solved for N
  const double s = beta * beta + beta + x * beta;
  p.n_max = (std::sqrt(900.0 + mem_bytes * s) - 30.0) / (12.0 * s);
  p.a_over_lambda_max = (std::sqrt(p.n_max) - 1.0) / p.alpha;
  if (!(p.a_over_lambda_max > 0)) return die_host::fail(DIE_E_INVALID, "the budget does not hold a single cell");
  p.nodes = (long long)std::floor(std::sqrt(p.n_max) + 1e-9);  // alpha a/lambda + 1 nodes per side
  p.n = p.nodes * p.nodes;
  p.unknowns = 3 * p.n;
  p.r = (int)std::ceil(3.0 * (double)p.n * beta - 1e-9);
  p.restart = (int)std::llround(x * p.r);
  p.restart_unpreconditioned = p.restart + p.r;  // the same memory without deflation
  p.mem_system = 720.0 * (double)p.n;
  p.mem_preconditioner = 16.0 * p.r * (double)p.r + 48.0 * (double)p.n * p.r + 48.0 * (double)p.n * p.restart;
  *plan = p;
  return DIE_OK;
}

}  // extern "C"
