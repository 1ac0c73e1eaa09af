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
    __syncthreads();
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
  __syncthreads();
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

// ---- binary16 planar GEMM path of the block Arnoldi step.  A complex block X (n x p,
// interleaved) is held planar as n x 2p real columns: the p real parts, then the p imaginary
// parts.  In that layout the block projection Q^H W and the update W -= Q H are each one real
// GEMM with the same flop count as the complex one (see launch_planar_combine).

// One thread per pair of consecutive rows of one column: X (interleaved, leading dimension ldx)
// to Xs (FP32 planar, leading dimension ldo) and/or Xh (binary16 planar); n even.
__global__ void k_planar_split(const float2* __restrict__ X, size_t ldx, size_t n2, int p, float* __restrict__ Xs,
                               _Float16* __restrict__ Xh, size_t ldo) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 * (size_t)p) return;
  const size_t col = e / n2, r = 2 * (e - col * n2);
  const float4 v = *reinterpret_cast<const float4*>(X + col * ldx + r);
  const size_t ore = col * ldo + r, oim = (p + col) * ldo + r;
  if (Xs) {
    *reinterpret_cast<float2*>(Xs + ore) = make_float2(v.x, v.z);
    *reinterpret_cast<float2*>(Xs + oim) = make_float2(v.y, v.w);
  }
  if (Xh) {
    Xh[ore] = (_Float16)v.x;
    Xh[ore + 1] = (_Float16)v.z;
    Xh[oim] = (_Float16)v.y;
    Xh[oim + 1] = (_Float16)v.w;
  }
}

// The inverse of the FP32 split: Xs (planar, leading dimension lds) to X (interleaved).
__global__ void k_planar_merge(const float* __restrict__ Xs, size_t lds, size_t n2, int p, float2* __restrict__ X,
                               size_t ldx) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 * (size_t)p) return;
  const size_t col = e / n2, r = 2 * (e - col * n2);
  const float2 re = *reinterpret_cast<const float2*>(Xs + col * lds + r);
  const float2 im = *reinterpret_cast<const float2*>(Xs + (p + col) * lds + r);
  *reinterpret_cast<float4*>(X + col * ldx + r) = make_float4(re.x, im.x, re.y, im.y);
}

// Binary16 copy of a planar FP32 block (n x 2p, both leading dimensions ld), two values a thread.
__global__ void k_planar_to_half(const float* __restrict__ Xs, size_t ld, size_t n2, int p2, _Float16* __restrict__ Xh) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n2 * (size_t)p2) return;
  const size_t col = e / n2, r = 2 * (e - col * n2);
  const float2 v = *reinterpret_cast<const float2*>(Xs + col * ld + r);
  Xh[col * ld + r] = (_Float16)v.x;
  Xh[col * ld + r + 1] = (_Float16)v.y;
}

// One thread per entry (q, k) of the complex projection H = Q^H W (nq x p): sums the nch chunk
// products C_b = Qs^T Ws (2nq x 2p each, leading dimension 2nq) in chunk order, then
//   Re H = Qr^T Wr + Qi^T Wi,  Im H = Qr^T Wi - Qi^T Wr,
// rounds H to binary16 and writes it twice: H (complex FP32 of the rounded values) and the real
// update matrix Hb (2nq x 2p binary16) with which Ws -= Qs Hb is W -= Q H:
//   Hb[re row, k] = Re H, Hb[re row, p + k] = Im H, Hb[im row, k] = -Im H, Hb[im row, p + k] = Re H.
// Row q = j p + c of Q (block j, column c) is real row 2 p j + c and imaginary row 2 p j + p + c of Qs.
__global__ void k_planar_combine(const float* __restrict__ C, int nch, size_t cstride, int nq, int p,
                                 float2* __restrict__ H, _Float16* __restrict__ Hb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * p) return;
  const int k = e / nq, q = e - k * nq;
  const int j = q / p, cc = q - j * p;
  const int M = 2 * nq, rre = 2 * p * j + cc, rim = rre + p;
  double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
  for (int b = 0; b < nch; ++b) {
    const float* Cb = C + (size_t)b * cstride;
    rr += Cb[(size_t)k * M + rre];
    ii += Cb[(size_t)(p + k) * M + rim];
    ri += Cb[(size_t)(p + k) * M + rre];
    ir += Cb[(size_t)k * M + rim];
  }
  const _Float16 hr = (_Float16)(rr + ii), hi = (_Float16)(ri - ir);
  H[(size_t)k * nq + q] = make_float2((float)hr, (float)hi);
  Hb[(size_t)k * M + rre] = hr;
  Hb[(size_t)(p + k) * M + rre] = hi;
  Hb[(size_t)k * M + rim] = -hi;
  Hb[(size_t)(p + k) * M + rim] = hr;
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

hipError_t launch_planar_split(const float2* X, size_t ldx, size_t n, int p, float* Xs, _Float16* Xh, size_t ldo,
                               hipStream_t st) {
  if (n % 2 || p < 1 || ldx < n || ldo < n) return hipErrorInvalidValue;
  const size_t tot = n / 2 * (size_t)p;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_planar_split, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, X, ldx, n / 2, p, Xs, Xh,
                     ldo);
  return hipGetLastError();
}

hipError_t launch_planar_merge(const float* Xs, size_t lds, size_t n, int p, float2* X, size_t ldx, hipStream_t st) {
  if (n % 2 || p < 1 || ldx < n || lds < n) return hipErrorInvalidValue;
  const size_t tot = n / 2 * (size_t)p;
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_planar_merge, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Xs, lds, n / 2, p, X, ldx);
  return hipGetLastError();
}

hipError_t launch_planar_to_half(const float* Xs, size_t ld, size_t n, int p, _Float16* Xh, hipStream_t st) {
  if (n % 2 || p < 1 || ld < n || ld % 2) return hipErrorInvalidValue;
  const size_t tot = n / 2 * (size_t)(2 * p);
  if (tot == 0) return hipSuccess;
  hipLaunchKernelGGL(k_planar_to_half, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, Xs, ld, n / 2, 2 * p, Xh);
  return hipGetLastError();
}

hipError_t launch_planar_combine(const float* C, int nch, int nq, int p, float2* H, _Float16* Hb, hipStream_t st) {
  if (nch < 1 || p < 1 || nq < p || nq % p) return hipErrorInvalidValue;
  const int tot = nq * p;
  hipLaunchKernelGGL(k_planar_combine, dim3((tot + 255) / 256), dim3(256), 0, st, C, nch, (size_t)2 * nq * 2 * p, nq,
                     p, H, Hb);
  return hipGetLastError();
}

}  // namespace die
