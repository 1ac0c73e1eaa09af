// FFT passes of the TE DIE operator product (gfx950).
//
// The product y = A x = x - T (chi x) is a linear convolution of the contrast
// source chi x with the Green tensor T sampled on all cell separations
// (Section 4, eq. A11 family).  Embedded circulantly in a px x py grid
// (px >= 2 nx - 1, py >= 2 ny - 1) it becomes three passes over HBM:
//   pass 1  rows:    W = FFT_x(pad(chi x)), stored transposed [x][y] (ny rows only)
//   pass 2  columns: Y = IFFT_y(That * FFT_y(pad W)), That the 2x2 symbol, ny rows kept
//   pass 3  rows:    y = x - crop(IFFT_x(Y))
// The 1/(px py) normalisation is folded into That.  Each pass keeps whole
// transforms in LDS; the transposed intermediate makes both the column reads of
// pass 2 and the row reads of passes 1 and 3 contiguous per transform.
#include "fft.hpp"
#include "ops.hpp"

#include <algorithm>
#include <cmath>
#include <mutex>
#include <type_traits>
#include <vector>

namespace die {

// Per-thread element count (the radix of the register stages): radix 8 in FP64 (register
// budget of the paired column pass); in FP32 radix 8 where log2 N is a multiple of 3 (the
// same stage count as radix 16 with lighter butterflies and more resident waves), else
// radix 16 (one stage fewer).  Tile sizes keep the LDS exchange buffer near 72 KB.
template <class T> __host__ __device__ constexpr int fft_loge(int logn) {
  return (sizeof(c2<T>) == 8 && logn % 3 != 0) ? 4 : 3;
}
constexpr int kLdsBudget = 76000;

// Variants of the three product passes, chosen at run time by the library's autotuner:
// bit 0 takes the other radix (8 <-> 16), bit 1 halves the tile (rows per block in the row
// passes, columns per block in the column pass).  Transforms shorter than 2^kFftTunedMinLog
// compile the default variant only.  A tile change moves no arithmetic (results are equal
// bit for bit); a radix change rounds differently.
template <class T> __host__ __device__ constexpr int fft_le(int logn, int v) {
  const int d = fft_loge<T>(logn), le = (v & 1) ? 7 - d : d;
  return le < logn ? le : logn;
}
template <class T> __host__ __device__ constexpr int fft_e(int logn, int v = 0) { return 1 << fft_le<T>(logn, v); }
template <class T> __host__ __device__ constexpr int rows_ty(int logn, int v = 0) {
  int n = 1 << logn, es = (int)sizeof(c2<T>), ty = 16;
  while (ty > 1 && (ty * fft_row_stride(n, es) * es > kLdsBudget || ty * n / fft_e<T>(logn, v) > 1024)) ty >>= 1;
  return (v & 2) && ty > 1 ? ty >> 1 : ty;
}
template <class T> __host__ __device__ constexpr int rows_threads(int logn, int v = 0) {
  return rows_ty<T>(logn, v) * (1 << logn) / fft_e<T>(logn, v);
}
// Columns per block of the column passes.  The exchange buffer holds one field component at a
// time; at least kWTile columns where it fits, so that a block reads and writes whole lines of
// the tiled intermediate (kWTile columns x kWTile rows).
template <class T> __host__ __device__ constexpr int cols_cx(int logn, int v = 0) {
  int n = 1 << logn, es = (int)sizeof(c2<T>), cx = 16;
  while (cx > 1 && (2 * cx * fft_row_stride(n, es) * es > kLdsBudget || cx * n / fft_e<T>(logn, v) > 1024)) cx >>= 1;
  while (cx < kWTile && 2 * cx * fft_row_stride(n, es) * es <= kLdsBudget && 2 * cx * n / fft_e<T>(logn, v) <= 1024)
    cx <<= 1;
  return (v & 2) && cx > 1 ? cx >> 1 : cx;
}
template <class T> __host__ __device__ constexpr int cols_threads(int logn, int v = 0) {
  return cols_cx<T>(logn, v) * (1 << logn) / fft_e<T>(logn, v);
}

// ------------------------------------------------------------------ pass 1
// Block: TY consecutive rows of the sets of `rb` right-hand sides (spr sets each).
// Loads rows position-fast (coalesced), stores W[s][x][y] array-fast (TY-contiguous).
// HALF: the rows hold at most N/2 values (nx <= N/2, the zero-padded product), so inputs in
// the upper half are known zeros at compile time and the first stage folds them away.
template <class T, class S, int LOGN, bool INV, bool HALF, int V = 0>
__global__ void __launch_bounds__(rows_threads<T>(LOGN, V))
k_rows_fwd(const c2<S>* __restrict__ x, const c2<T>* __restrict__ chi0, const c2<T>* __restrict__ chi20,
           c2<T>* __restrict__ W, const c2<T>* __restrict__ tw, int nx, int nrows, int ntiles, int nrhs, int spr,
           int rb, int rpo, const int* __restrict__ live) {
  using F = RegFft<T, LOGN, rows_ty<T>(LOGN, V), fft_le<T>(LOGN, V), 1, false, kPosFast, kArrFast>;
  constexpr int N = F::N, E = F::E, TY = rows_ty<T>(LOGN, V);
  __shared__ c2<T> lds[F::LDS_ELEMS];
  // logical order group-fastest: the blocks of one row tile run on one XCD close together, so the
  // contrast rows they all multiply by are read from HBM about once
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int ngrp = gridDim.x / ntiles;
  const int tile = L / ngrp, grp = L % ngrp;
  const int y0 = tile * TY;
  const int r1 = min(nrhs, (grp + 1) * rb);
  for (int r = grp * rb; r < r1; ++r) {
    if (live && !live[r]) continue;
    // right-hand side r belongs to object r / rpo (rpo = 0: a single object)
    const size_t oo = rpo > 0 ? (size_t)(r / rpo) * nrows * nx : 0;
    for (int c = 0; c < spr; ++c) {
      // components from the third on (H3 of the full TE system) take the second contrast
      const c2<T>* chi = (c >= 2 && chi20) ? chi20 + oo : (chi0 ? chi0 + oo : nullptr);
      const size_t s = (size_t)r * spr + c;
      const c2<S>* xs = x + s * nrows * nx;
      // keep per-element address arithmetic inside the loop (hoisting it costs ~100 VGPRs)
      int t = threadIdx.x;
      asm volatile("" : "+v"(t));
      c2<T> v[1][E];
#pragma unroll
      for (int u = 0; u < E / F::R0; ++u)
#pragma unroll
        for (int q = 0; q < F::R0; ++q) {
          int b, pos;
          F::in_pos(t, u, q, b, pos);
          const int yy = y0 + b;
          c2<T> a = mk<T>(0, 0);
          if (!HALF || q * (N / F::R0) < N / 2) {
            // unconditional loads at a clamped address, zero by selection: no branch per element,
            // so the loads of all elements are in flight together
            const bool ok = pos < nx && yy < nrows;
            const size_t o = (size_t)min(yy, nrows - 1) * nx + min(pos, nx - 1);
            a = ld<T, S>(xs + o);
            if (chi) a = cmul<T>(a, chi[o]);
            if (!ok) a = mk<T>(0, 0);
          }
          v[0][u * F::R0 + q] = a;
        }
      F::template run<INV>(v, lds, tw, t);
      // the product's intermediate is tiled (wtile_index); the plain transforms store W[s][x][y]
      const int rows4 = wtile_rows(nrows);
      c2<T>* Ws = W + s * (HALF ? (size_t)wtile_cols(N) * rows4 : (size_t)N * nrows);
#pragma unroll
      for (int u = 0; u < E / F::RL; ++u)
#pragma unroll
        for (int q = 0; q < F::RL; ++q) {
          int b, pos;
          F::out_pos(t, u, q, b, pos);
          const int yy = y0 + b;
          if (yy < nrows)
            Ws[HALF ? wtile_index(pos, yy, rows4) : (size_t)pos * nrows + yy] = v[0][u * F::RL + q];
        }
    }
  }
}

// ------------------------------------------------------------------ pass 2
// Block: CX columns of one right-hand side, both components held by the same threads,
// so the 2x2 symbol multiply runs in registers between the forward and the inverse
// transform.  Logical blocks sharing symbol columns run on the same XCD close together.
// With more than one stage, the first stage loads and the last stage stores array-fast
// (consecutive lanes on the CX columns of one row first), so that a wave moves whole lines of
// the tiled intermediate; the symbol multiply between the transforms runs position-fast
// (consecutive lanes on consecutive frequencies: contiguous symbol reads).
// NC field components per right-hand side (1: TM, 2: TE, 3: TE with H3); the symbol holds
// sym_planes(NC) values per frequency, the upper triangle of the symmetric NC x NC matrix
// (11 | 11, 12, 22 | 11, 12, 22, 13, 23, 33).
template <class T, int LOGN, int V = 0, int NC = 2>
__global__ void __launch_bounds__(cols_threads<T>(LOGN, V))
k_cols_symbol(c2<T>* __restrict__ W, const c2<T>* __restrict__ sym, const c2<T>* __restrict__ tw, int ncols,
              int nrows, int nrhs, const int* __restrict__ live) {
  constexpr int NPL = sym_planes(NC);
  constexpr int CX = cols_cx<T>(LOGN, V);
  constexpr int LE = fft_le<T>(LOGN, V);
  constexpr int MEDGE = LOGN > LE ? kArrFast : kPosFast;  // one stage only: position-fast throughout
  using F = RegFft<T, LOGN, CX, LE, NC, false, MEDGE, kPosFast, kPosFast>;
  using G = RegFft<T, LOGN, CX, LE, NC, true, kPosFast, kPosFast, MEDGE>;
  static_assert(G::R0 == F::RL, "inverse must start with the forward's last radix");
  constexpr int N = F::N, E = F::E;
  __shared__ c2<T> lds[F::LDS_ELEMS];
  // logical order rhs-fastest: blocks sharing symbol columns run on the same XCD together
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int r = L % nrhs, x0 = (L / nrhs) * CX;
  int t = threadIdx.x;
  if (live && !live[r]) return;
  const int rows4 = wtile_rows(nrows);
  const size_t plane = (size_t)wtile_cols(ncols) * rows4;  // one component of the tiled intermediate
  c2<T>* Wr = W + (size_t)r * NC * plane;
  c2<T> v[NC][E];
#pragma unroll
  for (int u = 0; u < E / F::R0; ++u)
#pragma unroll
    for (int q = 0; q < F::R0; ++q) {
      int b, pos;
      F::in_pos(t, u, q, b, pos);
      const int xx = x0 + b, e = u * F::R0 + q;
      // nrows <= N/2 (zero padding to at least 2 nrows - 1): the upper half is known zero
      const bool lower = q * (N / F::R0) < N / 2;
      const bool ok = xx < ncols && pos < nrows;
      const size_t o = wtile_index(min(xx, ncols - 1), min(pos, nrows - 1), rows4);  // clamped: no branch
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        v[c][e] = mk<T>(0, 0);
        if (lower) {
          const c2<T> a = Wr[c * plane + o];
          if (ok) v[c][e] = a;
        }
      }
    }
  F::template run<false>(v, lds, tw, t);
  asm volatile("" : "+v"(t));  // per-phase address arithmetic (hoisting it costs VGPRs)
#pragma unroll
  for (int u = 0; u < E / F::RL; ++u)
#pragma unroll
    for (int q = 0; q < F::RL; ++q) {
      int b, pos;
      F::out_pos(t, u, q, b, pos);
      const int xx = x0 + b, e = u * F::RL + q;
      {
        // columns past ncols (a partial last block) multiply a clamped column's symbol; their
        // results are never stored
        const c2<T>* sp = sym + ((size_t)min(xx, ncols - 1) * N + pos) * NPL;
        if constexpr (NC == 1) {
          v[0][e] = cmul<T>(sp[0], v[0][e]);
        } else if constexpr (NC == 2) {
          const c2<T> s11 = sp[0], s12 = sp[1], s22 = sp[2];
          const c2<T> a = v[0][e], bb = v[1][e];
          v[0][e] = cadd<T>(cmul<T>(s11, a), cmul<T>(s12, bb));
          v[1][e] = cadd<T>(cmul<T>(s12, a), cmul<T>(s22, bb));
        } else {
          const c2<T> s11 = sp[0], s12 = sp[1], s22 = sp[2], s13 = sp[3], s23 = sp[4], s33 = sp[5];
          const c2<T> a = v[0][e], bb = v[1][e], cc = v[2][e];
          v[0][e] = cadd<T>(cadd<T>(cmul<T>(s11, a), cmul<T>(s12, bb)), cmul<T>(s13, cc));
          v[1][e] = cadd<T>(cadd<T>(cmul<T>(s12, a), cmul<T>(s22, bb)), cmul<T>(s23, cc));
          v[2][e] = cadd<T>(cadd<T>(cmul<T>(s13, a), cmul<T>(s23, bb)), cmul<T>(s33, cc));
        }
      }
    }
  G::template run<true>(v, lds, tw, t);
  asm volatile("" : "+v"(t));
#pragma unroll
  for (int u = 0; u < E / G::RL; ++u)
#pragma unroll
    for (int q = 0; q < G::RL; ++q) {
      int b, pos;
      G::out_pos(t, u, q, b, pos);
      const int xx = x0 + b, e = u * G::RL + q;
      if (q * (N / G::RL) < N / 2 && xx < ncols && pos < nrows) {  // only rows < nrows <= N/2 are kept
#pragma unroll
        for (int c = 0; c < NC; ++c) Wr[c * plane + wtile_index(xx, pos, rows4)] = v[c][e];
      }
    }
}

// Full-length transforms along the contiguous axis of W[set][col][0:N], in place
// (symbol setup and diagnostics).
template <class T, int LOGN, bool INV>
__global__ void __launch_bounds__(cols_threads<T>(LOGN))
k_cols_plain(c2<T>* __restrict__ W, const c2<T>* __restrict__ tw, int ncols, int ntiles) {
  constexpr int NB = cols_cx<T>(LOGN);
  using F = RegFft<T, LOGN, NB, fft_le<T>(LOGN, 0), 1, false, kPosFast, kPosFast>;
  constexpr int N = F::N, E = F::E;
  __shared__ c2<T> lds[F::LDS_ELEMS];
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int s = L / ntiles, x0 = (L % ntiles) * NB, t = threadIdx.x;
  c2<T>* Ws = W + (size_t)s * ncols * N;
  c2<T> v[1][E];
#pragma unroll
  for (int u = 0; u < E / F::R0; ++u)
#pragma unroll
    for (int q = 0; q < F::R0; ++q) {
      int b, pos;
      F::in_pos(t, u, q, b, pos);
      v[0][u * F::R0 + q] = (x0 + b < ncols) ? Ws[(size_t)(x0 + b) * N + pos] : mk<T>(0, 0);
    }
  F::template run<INV>(v, lds, tw, t);
#pragma unroll
  for (int u = 0; u < E / F::RL; ++u)
#pragma unroll
    for (int q = 0; q < F::RL; ++q) {
      int b, pos;
      F::out_pos(t, u, q, b, pos);
      if (x0 + b < ncols) Ws[(size_t)(x0 + b) * N + pos] = v[0][u * F::RL + q];
    }
}

// ------------------------------------------------------------------ pass 3
// Block: TY rows of one set.  Loads W[s][x][y] array-fast (TY-contiguous), stores
// y = u - crop(IFFT) position-fast (coalesced).
template <class T, class S, int LOGN, int V = 0>
__global__ void __launch_bounds__(rows_threads<T>(LOGN, V))
k_rows_inv_sub(const c2<T>* __restrict__ W, const c2<S>* __restrict__ u, c2<S>* __restrict__ y,
               const c2<T>* __restrict__ tw, int nx, int nrows, int ntiles, int spr, const int* __restrict__ live,
               S* __restrict__ planar, size_t ldp, int pw) {
  using F = RegFft<T, LOGN, rows_ty<T>(LOGN, V), fft_le<T>(LOGN, V), 1, false, kArrFast, kPosFast>;
  constexpr int N = F::N, E = F::E, TY = rows_ty<T>(LOGN, V);
  __shared__ c2<T> lds[F::LDS_ELEMS];
  const int L = xcd_remap(blockIdx.x, gridDim.x);
  const int tile = L % ntiles, s = L / ntiles, t = threadIdx.x;
  if (live && !live[s / spr]) return;
  const int y0 = tile * TY;
  const int rows4 = wtile_rows(nrows);
  const c2<T>* Ws = W + (size_t)s * wtile_cols(N) * rows4;
  c2<T> v[1][E];
#pragma unroll
  for (int uu = 0; uu < E / F::R0; ++uu)
#pragma unroll
    for (int q = 0; q < F::R0; ++q) {
      int b, pos;
      F::in_pos(t, uu, q, b, pos);
      const int yy = y0 + b;
      const c2<T> a = Ws[wtile_index(pos, min(yy, nrows - 1), rows4)];  // clamped: no branch
      v[0][uu * F::R0 + q] = yy < nrows ? a : mk<T>(0, 0);
    }
  F::template run<true>(v, lds, tw, t);
  const size_t so = (size_t)s * nrows * nx;
#pragma unroll
  for (int uu = 0; uu < E / F::RL; ++uu)
#pragma unroll
    for (int q = 0; q < F::RL; ++q) {
      int b, pos;
      F::out_pos(t, uu, q, b, pos);
      const int yy = y0 + b;
      if (q * (N / F::RL) < N / 2) {  // only columns < nx <= N/2 are kept
        const size_t o = so + (size_t)min(yy, nrows - 1) * nx + min(pos, nx - 1);
        const c2<T> d = csub<T>(ld<T, S>(u + o), v[0][uu * F::RL + q]);  // unconditional (clamped) load
        if (pos < nx && yy < nrows) {
          if (planar) {  // uniform: right-hand side s / spr, component s % spr
            const size_t i = (size_t)(s % spr) * nrows * nx + (size_t)yy * nx + pos, r = (size_t)(s / spr);
            planar[r * ldp + i] = (S)d.x;
            planar[((size_t)pw + r) * ldp + i] = (S)d.y;
          } else {
            st<S, T>(y + o, d);
          }
        }
      }
    }
}

// ------------------------------------------------------------------ helpers
template <class T>
__global__ void __launch_bounds__(256) k_transpose(const c2<T>* __restrict__ in, c2<T>* __restrict__ out,
                                                   int rows, int cols) {
  __shared__ c2<T> tile[32][33];
  const int b = blockIdx.z;
  const c2<T>* ib = in + (size_t)b * rows * cols;
  c2<T>* ob = out + (size_t)b * rows * cols;
  const int c0 = blockIdx.x * 32, r0 = blockIdx.y * 32;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int k = ty; k < 32; k += 8) {
    const int rr = r0 + k, cc = c0 + tx;
    if (rr < rows && cc < cols) tile[k][tx] = ib[(size_t)rr * cols + cc];
  }
  lds_sync();
  for (int k = ty; k < 32; k += 8) {
    const int cc = c0 + k, rr = r0 + tx;
    if (rr < rows && cc < cols) ob[(size_t)cc * rows + rr] = tile[tx][k];
  }
}

__global__ void __launch_bounds__(256) k_pack_symbol(const double2* __restrict__ W, double2* __restrict__ s64,
                                                     float2* __restrict__ s32, size_t plane, int npl, double scale) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= plane) return;
  for (int a = 0; a < npl; ++a) {
    double2 v = W[a * plane + e];
    v.x *= scale;
    v.y *= scale;
    s64[e * npl + a] = v;
    s32[e * npl + a] = make_float2((float)v.x, (float)v.y);
  }
}

// ------------------------------------------------------------------ tables
namespace {
struct DevTables {
  double2* tw64 = nullptr;
  float2* tw32 = nullptr;
};
std::mutex g_tw_mu;
DevTables g_tw[64];
}  // namespace

hipError_t fft_tables(const double2** tw64, const float2** tw32) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_tw_mu);
  DevTables& t = g_tw[dev];
  if (!t.tw64) {
    std::vector<double2> h64(kTw);
    std::vector<float2> h32(kTw);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int j = 0; j < kTw; ++j) {
      // exp(-2 pi i j / 4096): evaluate in extended precision, round once
      const long double a = two_pi * (long double)j / (long double)kTw;
      const long double c = cosl(a), s = -sinl(a);
      h64[j] = make_double2((double)c, (double)s);
      h32[j] = make_float2((float)c, (float)s);
    }
    double2* d64 = nullptr;
    float2* d32 = nullptr;
    if ((e = hipMalloc(&d64, kTw * sizeof(double2))) != hipSuccess) return e;
    if ((e = hipMalloc(&d32, kTw * sizeof(float2))) != hipSuccess) { (void)hipFree(d64); return e; }
    if ((e = hipMemcpy(d64, h64.data(), kTw * sizeof(double2), hipMemcpyHostToDevice)) != hipSuccess) return e;
    if ((e = hipMemcpy(d32, h32.data(), kTw * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess) return e;
    t.tw64 = d64;
    t.tw32 = d32;
  }
  *tw64 = t.tw64;
  *tw32 = t.tw32;
  return hipSuccess;
}

namespace {
template <class T> const c2<T>* table_for();
template <> const double2* table_for<double>() {
  const double2* a; const float2* b;
  return fft_tables(&a, &b) == hipSuccess ? a : nullptr;
}
template <> const float2* table_for<float>() {
  const double2* a; const float2* b;
  return fft_tables(&a, &b) == hipSuccess ? b : nullptr;
}
}  // namespace

#define DIE_LOGN_CASES(X) X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8) X(9) X(10) X(11) X(12)

namespace {
// Calls f(std::integral_constant<int, V>) for the pass variant v (default only below the
// tuned lengths).
template <int L, class F> void for_variant(int v, F&& f) {
  if constexpr (L < kFftTunedMinLog) {
    (void)v;
    f(std::integral_constant<int, 0>{});
  } else {
    switch (v & (kFftVariants - 1)) {
      case 1: f(std::integral_constant<int, 1>{}); break;
      case 2: f(std::integral_constant<int, 2>{}); break;
      case 3: f(std::integral_constant<int, 3>{}); break;
      default: f(std::integral_constant<int, 0>{}); break;
    }
  }
}
}  // namespace

template <class T, class S>
hipError_t launch_rows_fwd(int logn, bool inverse, const c2<S>* x, const c2<T>* chi, const c2<T>* chi2, c2<T>* W,
                           int nx, int nrows, int nrhs, int spr, int rb, int rpo, const int* live, hipStream_t st,
                           int v) {
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nrhs <= 0 || nrows <= 0) return hipSuccess;
  const bool half = !inverse && 2 * nx <= (1 << logn);  // the zero-padded product: the tuned kernels
  switch (logn) {
#define CASE(L)                                                                                         \
  case L: {                                                                                             \
    for_variant<L>(half ? v : 0, [&](auto vc) {                                                         \
      constexpr int V = decltype(vc)::value;                                                            \
      const int ntiles = (nrows + rows_ty<T>(L, V) - 1) / rows_ty<T>(L, V);                             \
      const int rbv = rb > 0 ? rb : std::max(1, std::min(nrhs, ntiles * nrhs / 2048));                  \
      dim3 grid((unsigned)(ntiles * ((nrhs + rbv - 1) / rbv)));                                         \
      dim3 block(rows_threads<T>(L, V));                                                                \
      if (half)                                                                                         \
        hipLaunchKernelGGL((k_rows_fwd<T, S, L, false, true, V>), grid, block, 0, st, x, chi, chi2, W, tw, nx, nrows, \
                           ntiles, nrhs, spr, rbv, rpo, live);                                          \
      else if constexpr (V == 0) {                                                                      \
        if (inverse)                                                                                    \
          hipLaunchKernelGGL((k_rows_fwd<T, S, L, true, false>), grid, block, 0, st, x, chi, chi2, W, tw, nx, nrows, \
                             ntiles, nrhs, spr, rbv, rpo, live);                                        \
        else                                                                                            \
          hipLaunchKernelGGL((k_rows_fwd<T, S, L, false, false>), grid, block, 0, st, x, chi, chi2, W, tw, nx, nrows, \
                             ntiles, nrhs, spr, rbv, rpo, live);                                        \
      }                                                                                                 \
    });                                                                                                 \
    break;                                                                                              \
  }
    DIE_LOGN_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cols_symbol(int logn, int ncomp, c2<T>* W, const c2<T>* sym, int ncols, int nrows, int nrhs,
                              const int* live, hipStream_t st, int v) {
  if (ncomp < 1 || ncomp > 3) return hipErrorInvalidValue;
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nrhs <= 0) return hipSuccess;
  if (2 * nrows > (1 << logn)) return hipErrorInvalidValue;  // the upper half must be padding
  switch (logn) {
#define CASE(L)                                                                                         \
  case L: {                                                                                             \
    for_variant<L>(v, [&](auto vc) {                                                                    \
      constexpr int V = decltype(vc)::value;                                                            \
      dim3 grid((unsigned)(((ncols + cols_cx<T>(L, V) - 1) / cols_cx<T>(L, V)) * nrhs));                \
      if (ncomp == 1)                                                                                   \
        hipLaunchKernelGGL((k_cols_symbol<T, L, V, 1>), grid, dim3(cols_threads<T>(L, V)), 0, st, W, sym, tw, \
                           ncols, nrows, nrhs, live);                                                   \
      else if (ncomp == 2)                                                                              \
        hipLaunchKernelGGL((k_cols_symbol<T, L, V, 2>), grid, dim3(cols_threads<T>(L, V)), 0, st, W, sym, tw, \
                           ncols, nrows, nrhs, live);                                                   \
      else                                                                                              \
        hipLaunchKernelGGL((k_cols_symbol<T, L, V, 3>), grid, dim3(cols_threads<T>(L, V)), 0, st, W, sym, tw, \
                           ncols, nrows, nrhs, live);                                                   \
    });                                                                                                 \
    break;                                                                                              \
  }
    DIE_LOGN_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T, class S>
hipError_t launch_rows_inv_sub(int logn, const c2<T>* W, const c2<S>* u, c2<S>* y, int nx, int nrows, int nsets,
                               int spr, const int* live, hipStream_t st, int v, S* planar, size_t ldp, int pw) {
  if (planar && (ldp < (size_t)spr * nrows * nx || pw < nsets / spr)) return hipErrorInvalidValue;
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nsets <= 0 || nrows <= 0) return hipSuccess;
  if (2 * nx > (1 << logn)) return hipErrorInvalidValue;  // the upper half must be padding
  switch (logn) {
#define CASE(L)                                                                                         \
  case L: {                                                                                             \
    for_variant<L>(v, [&](auto vc) {                                                                    \
      constexpr int V = decltype(vc)::value;                                                            \
      const int ntiles = (nrows + rows_ty<T>(L, V) - 1) / rows_ty<T>(L, V);                             \
      dim3 grid((unsigned)(ntiles * nsets));                                                            \
      hipLaunchKernelGGL((k_rows_inv_sub<T, S, L, V>), grid, dim3(rows_threads<T>(L, V)), 0, st, W, u, y, tw, nx, \
                         nrows, ntiles, spr, live, planar, ldp, pw);                                    \
    });                                                                                                 \
    break;                                                                                              \
  }
    DIE_LOGN_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cols_plain(int logn, bool inverse, c2<T>* W, int ncols, int nsets, hipStream_t st) {
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nsets <= 0 || ncols <= 0) return hipSuccess;
  switch (logn) {
#define CASE(L)                                                                                         \
  case L: {                                                                                             \
    const int ntiles = (ncols + cols_cx<T>(L) - 1) / cols_cx<T>(L);                                     \
    dim3 grid((unsigned)(ntiles * nsets));                                                              \
    if (inverse)                                                                                        \
      hipLaunchKernelGGL((k_cols_plain<T, L, true>), grid, dim3(cols_threads<T>(L)), 0, st, W, tw, ncols, ntiles); \
    else                                                                                                \
      hipLaunchKernelGGL((k_cols_plain<T, L, false>), grid, dim3(cols_threads<T>(L)), 0, st, W, tw, ncols, ntiles); \
    break;                                                                                              \
  }
    DIE_LOGN_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_transpose(const c2<T>* in, c2<T>* out, int rows, int cols, int nb, hipStream_t st) {
  if (nb <= 0 || rows <= 0 || cols <= 0) return hipSuccess;
  dim3 grid((cols + 31) / 32, (rows + 31) / 32, nb);
  hipLaunchKernelGGL((k_transpose<T>), grid, dim3(256), 0, st, in, out, rows, cols);
  return hipGetLastError();
}

hipError_t launch_pack_symbol(const double2* W, double2* s64, float2* s32, int px, int py, int npl, double scale,
                              hipStream_t st) {
  const size_t plane = (size_t)px * py;
  hipLaunchKernelGGL(k_pack_symbol, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, st, W, s64, s32,
                     plane, npl, scale);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_rows_fwd<double, double>(int, bool, const double2*, const double2*, const double2*,
                                                    double2*, int, int, int, int, int, int, const int*, hipStream_t,
                                                    int);
template hipError_t launch_rows_fwd<float, float>(int, bool, const float2*, const float2*, const float2*, float2*,
                                                  int, int, int, int, int, int, const int*, hipStream_t, int);
template hipError_t launch_cols_symbol<double>(int, int, double2*, const double2*, int, int, int, const int*,
                                               hipStream_t, int);
template hipError_t launch_cols_symbol<float>(int, int, float2*, const float2*, int, int, int, const int*,
                                              hipStream_t, int);
template hipError_t launch_rows_inv_sub<double, double>(int, const double2*, const double2*, double2*, int,
                                                        int, int, int, const int*, hipStream_t, int, double*, size_t,
                                                        int);
template hipError_t launch_rows_inv_sub<float, float>(int, const float2*, const float2*, float2*, int, int,
                                                      int, int, const int*, hipStream_t, int, float*, size_t, int);
template hipError_t launch_cols_plain<double>(int, bool, double2*, int, int, hipStream_t);
template hipError_t launch_cols_plain<float>(int, bool, float2*, int, int, hipStream_t);
template hipError_t launch_transpose<double>(const double2*, double2*, int, int, int, hipStream_t);
template hipError_t launch_transpose<float>(const float2*, float2*, int, int, int, hipStream_t);

}  // namespace die
