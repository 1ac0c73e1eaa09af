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
// holding column q (which already carries P_0 .. P_{q-1}) forms u_q and publishes it in one of
// two LDS slots; after one barrier every row applies it to its column if that lies right of q.
// The slots alternate, so a slot is rewritten only after the barrier that follows its reads.
__global__ void __launch_bounds__(kPanelThreads)
k_panel_qr(double2* __restrict__ H, int ld, int r0, int c0, int rows, int pc, double2* __restrict__ U,
           double* __restrict__ s) {
  __shared__ double2 ub[2][kPanelMaxRows];
  __shared__ double sb[2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, l16 = lane & 15;
  const int j = w + kPanelWaves * g;  // this row's column
  double2 x[kRowsPerLane];
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int i = l16 + 16 * t;
    x[t] = (j < pc && i < rows) ? H[(size_t)(c0 + j) * ld + r0 + i] : make_double2(0.0, 0.0);
  }
  for (int q = 0; q < pc; ++q) {
    const int buf = q & 1;
    if (w == q % kPanelWaves) {  // the wave holding column q (wave-uniform); its row q / 16 writes
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
          ub[buf][i] = u;
          if (i < rows) U[(size_t)q * kPanelMaxRows + i] = u;
          // column q becomes R's: -e^{i arg a} |x| on the diagonal, zeros below
          if (i == q) x[t] = make_double2(-ph.x * nrm, -ph.y * nrm);
          else if (i > q) x[t] = make_double2(0.0, 0.0);
        }
        if (l16 == 0) {
          sb[buf] = sc;
          s[q] = sc;
        }
      }
    }
    lds_sync();
    const double sc = sb[buf];
    double2 u[kRowsPerLane];
    double2 d = make_double2(0.0, 0.0);
#pragma unroll
    for (int t = 0; t < kRowsPerLane; ++t) {
      u[t] = ub[buf][l16 + 16 * t];
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
  }
#pragma unroll
  for (int t = 0; t < kRowsPerLane; ++t) {
    const int i = l16 + 16 * t;
    if (j < pc && i < rows) H[(size_t)(c0 + j) * ld + r0 + i] = x[t];
  }
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

}  // namespace die
