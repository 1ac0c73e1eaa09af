// Least squares of the block GMRES cycle on the GPU: min || B - H Y || for the block upper
// Hessenberg H of block Arnoldi with block size p (at most p sub-diagonals), by Householder
// QR one p-column panel at a time: the panel's rows span at most 2p (its own block row and
// the triangular sub-diagonal block below it), so each panel is factored in LDS by one
// workgroup, and its reflectors are then applied to the trailing columns and to B in
// parallel, one wavefront per column.  A triangular solve with R finishes it (the caller).
// Complex FP64 throughout; H is column-major with leading dimension ld.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ops.hpp"

namespace die {
namespace {

constexpr int kPanelThreads = 1024;
constexpr int kPanelWaves = kPanelThreads / 64;
// A 16-lane row of a wave holds one column, 8 rows a lane (row i at lane i % 16, slot i / 16):
// a column's inner product is 8 local multiply-adds and a 4-step DPP butterfly in the row.
constexpr int kRowsPerLane = kPanelMaxRows / 16;
static_assert(kPanelMaxCols == 4 * kPanelWaves && kPanelMaxRows % 16 == 0, "panel tiling");

// DPP move of a double within each row of 16 lanes (CTRL: a DPP16 row or quad permutation).
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b & 0xffffffffu), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((unsigned long long)(unsigned)hi << 32) | (unsigned)lo);
}
// Sum over the 16 lanes of each row, left in all of them: row mirror (i <-> 15 - i), half-row
// mirror (i <-> 7 - i), then the quad permutations [2,3,0,1] and [1,0,3,2].
__device__ __forceinline__ double sum16(double v) {
  v += dpp_f64<0x140>(v);
  v += dpp_f64<0x141>(v);
  v += dpp_f64<0x4e>(v);
  v += dpp_f64<0xb1>(v);
  return v;
}

__device__ __forceinline__ double2 cfma_conj(double2 a, double2 b, double2 acc) {  // acc + conj(a) b
  acc.x = fma(a.x, b.x, acc.x);
  acc.x = fma(a.y, b.y, acc.x);
  acc.y = fma(a.x, b.y, acc.y);
  acc.y = fma(-a.y, b.x, acc.y);
  return acc;
}

// Factor the panel H[r0 : r0 + rows, c0 : c0 + pc] (rows <= kPanelMaxRows, pc <= kPanelMaxCols)
// in place: R on and above the diagonal; the reflectors u_q (q < pc; u_q[i] = 0 for i < q) go to
// U (rows x pc, column-major, leading dimension kPanelMaxRows) with scales s[q] = 2 / (u_q^H u_q)
// (0 for a zero column).  The reflector P_q = I - s_q u_q u_q^H maps column q to -e^{i arg a} |x| e_q.
// The panel lives in registers: column j in row j / 16 of wave j % 16.  Per reflector the row
// holding column q (which already carries P_0 .. P_{q-1}) forms u_q and publishes it in its own
// LDS slot; after one barrier every row applies it to its column if that lies right of q.  The
// wave holding column q + 1 forms u_{q+1} right after applying u_q, in the same interval, at raised
// issue priority.  U and s are written once, after the last reflector.
__global__ void __launch_bounds__(kPanelThreads)
k_panel_qr(double2* __restrict__ H, int ld, int r0, int c0, int rows, int pc, double2* __restrict__ U,
           double* __restrict__ s) {
  // every reflector stays in LDS until the end: global stores inside the loop would make each
  // reflector's barrier wait for them
  __shared__ double2 ush[kPanelMaxCols][kPanelMaxRows];
  __shared__ double ssh[kPanelMaxCols];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int j = w + kPanelWaves * g;  // this row's column
  double2 x[kRowsPerLane];
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int i = l16 + 16 * t;
    x[t] = (j < pc && i < rows) ? H[(size_t)(c0 + j) * ld + r0 + i] : make_double2(0.0, 0.0);
  }
  // the wave holding column q forms u_q (wave-uniform call; its row q / 16 writes it to LDS) and
  // turns column q into R's
  auto form = [&](int q) {
    const bool own = g == q / kPanelWaves;
    double sq = 0.0;
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) {
      const int i = l16 + 16 * t;
      if (i >= q && i < rows) sq = fma(x[t].x, x[t].x, fma(x[t].y, x[t].y, sq));
    }
    const double nrm = sqrt(sum16(sq));  // the norm of this row's column below q
    double2 aq = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t)
      if (q / 16 == t) aq = x[t];
    const int src = (q / kPanelWaves) * 16 + (q & 15);  // the lane holding row q of column q
    const unsigned long long ax = __builtin_bit_cast(unsigned long long, aq.x);
    const unsigned long long ay = __builtin_bit_cast(unsigned long long, aq.y);
    const double2 a = make_double2(
        __builtin_bit_cast(double, ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(ax >> 32), src)
                                    << 32) |
                                       (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(ax & 0xffffffffu), src)),
        __builtin_bit_cast(double, ((unsigned long long)(unsigned)__builtin_amdgcn_readlane((int)(ay >> 32), src)
                                    << 32) |
                                       (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(ay & 0xffffffffu), src)));
    const double aa = sqrt(a.x * a.x + a.y * a.y);
    const double2 ph = aa > 0.0 ? make_double2(a.x / aa, a.y / aa) : make_double2(1.0, 0.0);
    // u = x[q:] + e^{i arg a} |x| e_q;  u^H u = 2 |x| (|x| + |a|)
    const double uu = 2.0 * nrm * (nrm + aa);
    const double sc = uu > 0.0 ? 2.0 / uu : 0.0;
    if (own) {
#pragma unroll
      for (int t = 0; t < kRowsPerLane; ++t) {
        const int i = l16 + 16 * t;
        double2 u = make_double2(0.0, 0.0);
        if (i == q) u = make_double2(a.x + ph.x * nrm, a.y + ph.y * nrm);
        else if (i > q && i < rows) u = x[t];
        ush[q][i] = u;
        // column q becomes R's: -e^{i arg a} |x| on the diagonal, zeros below
        if (i == q) x[t] = make_double2(-ph.x * nrm, -ph.y * nrm);
        else if (i > q) x[t] = make_double2(0.0, 0.0);
      }
      if (l16 == 0) ssh[q] = sc;
    }
  };
  if (w == 0) form(0);
  lds_sync();
  for (int q = 0; q < pc; ++q) {
    // the wave that forms u_{q+1} applies u_q first at raised issue priority, so that forming
    // u_{q+1} (norm, square roots, divisions: a serial chain) overlaps the other waves' updates
    const bool next = q + 1 < pc && w == (q + 1) % kPanelWaves;
    if (next) __builtin_amdgcn_s_setprio(3);
    const double sc = ssh[q];
    double2 u[kRowsPerLane];
    double2 d = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) {
      u[t] = ush[q][l16 + 16 * t];
      d = cfma_conj(u[t], x[t], d);
    }
    d.x = sum16(d.x);
    d.y = sum16(d.y);
    if (j > q && j < pc) {  // y -= sc u (u^H y)
      const double2 f = make_double2(sc * d.x, sc * d.y);
#pragma unroll
      for (int t = 0; t < kRowsPerLane; ++t) {
        x[t].x -= u[t].x * f.x - u[t].y * f.y;
        x[t].y -= u[t].x * f.y + u[t].y * f.x;
      }
    }
    if (next) {
      form(q + 1);
      __builtin_amdgcn_s_setprio(0);
    }
    lds_sync();
  }
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int i = l16 + 16 * t;
    if (j < pc && i < rows) H[(size_t)(c0 + j) * ld + r0 + i] = x[t];
  }
  // the reflectors (rows < rows) and their scales, for the application to the later columns
  for (int e = threadIdx.x; e < pc * kPanelMaxRows; e += kPanelThreads) {
    const int q = e / kPanelMaxRows, i = e - q * kPanelMaxRows;
    if (i < rows) U[e] = ush[q][i];
  }
  if (threadIdx.x < pc) s[threadIdx.x] = ssh[threadIdx.x];
}

// Apply the panel's reflectors P_0, P_1, ..., P_{pc-1} (in that order) to rows r0 .. r0+rows of
// the columns [cb, ce) of H and all k columns of B (leading dimension ldb): one 16-lane row per
// column, 16 columns a workgroup.  The reflectors and their scales are first staged in LDS, so
// the serial chain over q reads LDS rather than L2.
__global__ void __launch_bounds__(256)
k_panel_apply(double2* __restrict__ H, int ld, double2* __restrict__ B, int ldb, int k, int r0, int rows, int pc,
              int cb, int ce, const double2* __restrict__ U, const double* __restrict__ s) {
  __shared__ double2 Us[kPanelMaxCols * kPanelMaxRows];
  __shared__ double ss[kPanelMaxCols];
  for (int e = threadIdx.x; e < pc * kPanelMaxRows; e += blockDim.x) {
    const int i = e % kPanelMaxRows;
    Us[e] = i < rows ? U[e] : make_double2(0.0, 0.0);
  }
  if (threadIdx.x < pc) ss[threadIdx.x] = s[threadIdx.x];
  const int l16 = threadIdx.x & 15;
  const int col = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int nh = ce - cb;
  const bool live = col < nh + k;  // the whole row of 16 lanes agrees; rows past the end idle
  double2* y = !live ? nullptr : col < nh ? H + (size_t)(cb + col) * ld + r0 : B + (size_t)(col - nh) * ldb + r0;
  double2 v[kRowsPerLane];
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int i = l16 + 16 * t;
    v[t] = live && i < rows ? y[i] : make_double2(0.0, 0.0);
  }
  lds_sync();
  for (int q = 0; q < pc; ++q) {
    const double2* u = Us + q * kPanelMaxRows;
    double2 uq[kRowsPerLane];
    double2 d = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) {
      uq[t] = u[l16 + 16 * t];
      d = cfma_conj(uq[t], v[t], d);
    }
    d.x = sum16(d.x);
    d.y = sum16(d.y);
    const double sc = ss[q];
    const double2 f = make_double2(sc * d.x, sc * d.y);
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) {
      v[t].x -= uq[t].x * f.x - uq[t].y * f.y;
      v[t].y -= uq[t].x * f.y + uq[t].y * f.x;
    }
  }
  if (!live) return;
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int i = l16 + 16 * t;
    if (i < rows) y[i] = v[t];
  }
}


// ------------------------------------------------------------------ CholQR factor
// One workgroup of 1024 threads (16 row groups x 64 columns).  The Gram G is scaled to unit
// diagonal, S = D G D with D = diag(G)^-1/2, and eliminated column by column with one barrier per
// column: step j subtracts l_ij conj(S(c, j)) from S(i, c) (j < c <= i, l_ij = S(i, j) / d_j) and
// applies the same row operations to the identity, which leaves Mi = L~^-1 for S = L~ diag(d) L~^H.
// With L = L~ diag(d)^1/2 the factor of G = R^H R is R = L^H D^-1, R(i, c) = conj(S(c, i)) / sqrt(d_i)
// / D_c (i < c), sqrt(d_c) / D_c (i = c), and R^-1 = D L^-H, R^-1(i, c) = D_i conj(Mi(c, i)) / sqrt(d_c).
constexpr int kCholLd = kCholQRMax + 1;  // LDS row stride (double2)

template <class T>
__device__ __forceinline__ void put_c(c2<T>* p, double2 v) {
  *p = mk<T>((T)v.x, (T)v.y);
}

template <class T>
__global__ void __launch_bounds__(1024)
k_cholqr_factor(const double2* __restrict__ G, int p, double rel_tol, double single_piv, int pass,
                double2* __restrict__ R1, c2<T>* __restrict__ Rinv, int* __restrict__ flags, c2<T>* __restrict__ Hb,
                int ldh) {
  __shared__ double2 S[kCholQRMax * kCholLd];
  __shared__ double2 Mi[kCholQRMax * kCholLd];
  __shared__ double dinv[kCholQRMax], sdiag[kCholQRMax], dp[kCholQRMax], sqd[kCholQRMax], gd[kCholQRMax];
  const int tid = threadIdx.x, c = tid & 63, rg = tid >> 6;
  if (pass == 2 && !flags[2]) {  // one pass sufficed (or the first failed): H = R1
    for (int e = tid; e < p * p; e += blockDim.x) {
      const int i = e % p, cc = e / p;
      put_c<T>(Hb + (size_t)cc * ldh + i, i <= cc ? R1[e] : make_double2(0.0, 0.0));
    }
    if (tid == 0) {
      flags[3] = flags[0];
      flags[4] = 0;
    }
    return;
  }
  if (tid < p) {
    const double d = G[(size_t)tid * p + tid].x;
    const bool ok = d > 0.0 && isfinite(d);
    dinv[tid] = ok ? 1.0 / sqrt(d) : 0.0;
    sdiag[tid] = ok ? d * dinv[tid] * dinv[tid] : 0.0;
  }
  lds_sync();
  bool fail = false;
  double dmax = 0.0;
  for (int i = 0; i < p; ++i) {  // every thread takes the same decision
    if (dinv[i] == 0.0) fail = true;
    dmax = fmax(dmax, sdiag[i]);
  }
  if (!fail) {
    for (int i = rg; i < p; i += 16)
      if (c <= i) {
        const double2 g = G[(size_t)c * p + i];
        const double sc = dinv[i] * dinv[c];
        S[i * kCholLd + c] = make_double2(g.x * sc, g.y * sc);
        Mi[i * kCholLd + c] = make_double2(i == c ? 1.0 : 0.0, 0.0);
      }
    lds_sync();
    for (int j = 0; j < p; ++j) {
      const double d = S[j * kCholLd + j].x;
      if (!(d > rel_tol * dmax)) {  // uniform: every thread reads the same pivot
        fail = true;
        break;
      }
      if (tid == 0) dp[j] = d;
      const double rd = 1.0 / d;
      // this thread's rows j + 1 + rg + 16 r (at most four): every LDS read of the step is issued
      // before its writes, so that their latencies overlap
      const bool upd = c > j;  // S(i, c) -= l conj(S(c, j)); otherwise Mi(i, c) -= l Mi(j, c)
      const double2 o = upd ? (c < p ? S[c * kCholLd + j] : make_double2(0.0, 0.0)) : Mi[j * kCholLd + c];
      double2 li[4], v[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = j + 1 + rg + 16 * r;
        const bool live = i < p && (!upd || c <= i);
        const int ii = live ? i : j;  // a row that exists (not written)
        const double2 sij = S[ii * kCholLd + j];
        li[r] = make_double2(sij.x * rd, sij.y * rd);
        v[r] = upd ? S[ii * kCholLd + (live ? c : j)] : Mi[ii * kCholLd + c];
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = j + 1 + rg + 16 * r;
        if (i >= p || (upd && c > i)) continue;
        const double2 l = li[r];
        if (upd) {
          v[r].x -= l.x * o.x + l.y * o.y;
          v[r].y -= l.y * o.x - l.x * o.y;
          S[i * kCholLd + c] = v[r];
        } else {
          v[r].x -= l.x * o.x - l.y * o.y;
          v[r].y -= l.x * o.y + l.y * o.x;
          Mi[i * kCholLd + c] = v[r];
        }
      }
      lds_sync();
    }
  }
  if (fail) {
    if (tid == 0) {
      if (pass == 1) {
        flags[0] = 0;
        flags[1] = 0;
        flags[2] = 0;
        flags[5] = 1;
      } else {
        flags[3] = 0;
        flags[4] = 0;
      }
    }
    return;
  }
  if (tid < p) {
    sqd[tid] = sqrt(dp[tid]);
    gd[tid] = 1.0 / dinv[tid];
  }
  lds_sync();
  if (c < p)
    for (int i = rg; i < p; i += 16) {
      double2 ri = make_double2(0.0, 0.0);
      if (i <= c) {
        const double2 m = Mi[c * kCholLd + i];
        const double f = dinv[i] / sqd[c];
        ri = make_double2(m.x * f, -m.y * f);
      }
      put_c<T>(Rinv + (size_t)c * p + i, ri);
      if (pass == 1) {
        double2 r = make_double2(0.0, 0.0);
        if (i < c) {
          const double2 sv = S[c * kCholLd + i];
          const double f = gd[c] / sqd[i];
          r = make_double2(sv.x * f, -sv.y * f);
        } else if (i == c) {
          r = make_double2(sqd[c] * gd[c], 0.0);
        }
        R1[(size_t)c * p + i] = r;
      } else {  // H(i, c) = sum over i <= q <= c of R2(i, q) R1(q, c)
        double hx = 0.0, hy = 0.0;
        for (int q = i; q <= c; ++q) {
          double2 r2;
          if (q == i) {
            r2 = make_double2(sqd[i] * gd[i], 0.0);
          } else {
            const double2 sv = S[q * kCholLd + i];
            const double f = gd[q] / sqd[i];
            r2 = make_double2(sv.x * f, -sv.y * f);
          }
          const double2 r1 = R1[(size_t)c * p + q];
          hx += r2.x * r1.x - r2.y * r1.y;
          hy += r2.x * r1.y + r2.y * r1.x;
        }
        put_c<T>(Hb + (size_t)c * ldh + i, make_double2(hx, hy));
      }
    }
  if (tid == 0) {
    if (pass == 1) {
      double dmin = 1.0;
      for (int j = 0; j < p; ++j) dmin = fmin(dmin, dp[j] / dmax);
      const int single = dmin >= single_piv;
      flags[0] = 1;
      flags[1] = single;
      flags[2] = !single;
      flags[5] = 1;
    } else {
      flags[3] = 1;
      flags[4] = 1;
    }
  }
}

// Y = 0 unless *flag (a grid-stride loop over the n x p block; every block returns at once while
// the flag is set).
template <class T>
__global__ void __launch_bounds__(256)
k_zero_unless(c2<T>* __restrict__ Y, size_t ldy, size_t n, int p, const int* __restrict__ flag) {
  if (*flag) return;
  const size_t total = n * (size_t)p;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (size_t)gridDim.x * blockDim.x) {
    const size_t c = e / n, r = e - c * n;
    Y[c * ldy + r] = mk<T>((T)0, (T)0);
  }
}

}  // namespace

hipError_t launch_block_hessenberg_qr(double2* H, int ld, int mr, int nc, int p, double2* B, int ldb, int k,
                                      double2* U, double* s, hipStream_t st) {
  if (p < 1 || p > kPanelMaxCols || nc % p || mr > ld || mr < nc || k < 0) return hipErrorInvalidValue;
  for (int c0 = 0; c0 < nc; c0 += p) {
    const int rows = std::min(2 * p, mr - c0);
    if (rows < p || rows > kPanelMaxRows) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_panel_qr, dim3(1), dim3(kPanelThreads), 0, st, H, ld, c0, c0, rows, p, U, s);
    const int cb = c0 + p, ncols = (nc - cb) + k;
    if (ncols > 0)
      hipLaunchKernelGGL(k_panel_apply, dim3((ncols + 15) / 16), dim3(256), 0, st, H, ld, B, ldb, k, c0, rows, p, cb,
                         nc, U, s);
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cholqr_factor(const double2* G, int p, double rel_tol, double single_piv, int pass, double2* R1,
                                c2<T>* Rinv, int* flags, c2<T>* Hb, int ldh, hipStream_t st) {
  if (p < 1 || p > kCholQRMax || (pass != 1 && pass != 2) || (pass == 2 && (!Hb || ldh < p)) || !G || !R1 || !Rinv ||
      !flags)
    return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_cholqr_factor<T>), dim3(1), dim3(1024), 0, st, G, p, rel_tol, single_piv, pass, R1, Rinv, flags,
                     Hb, ldh);
  return hipGetLastError();
}
template hipError_t launch_cholqr_factor<float>(const double2*, int, double, double, int, double2*, c2<float>*, int*,
                                                c2<float>*, int, hipStream_t);
template hipError_t launch_cholqr_factor<double>(const double2*, int, double, double, int, double2*, c2<double>*,
                                                 int*, c2<double>*, int, hipStream_t);

template <class T>
hipError_t launch_zero_unless(c2<T>* Y, size_t ldy, size_t n, int p, const int* flag, hipStream_t st) {
  if (!Y || !flag || p < 1 || ldy < n) return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  const size_t total = n * (size_t)p;
  const unsigned grid = (unsigned)std::min<size_t>((total + 255) / 256, 1024);
  hipLaunchKernelGGL((k_zero_unless<T>), dim3(grid), dim3(256), 0, st, Y, ldy, n, p, flag);
  return hipGetLastError();
}
template hipError_t launch_zero_unless<float>(c2<float>*, size_t, size_t, int, const int*, hipStream_t);
template hipError_t launch_zero_unless<double>(c2<double>*, size_t, size_t, int, const int*, hipStream_t);

}  // namespace die
