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

#include <cmath>
#include <mutex>
#include <vector>

namespace die {

template <class T> __host__ __device__ constexpr int rows_ty(int logn) {
  int n = 1 << logn, e = fft_elems(logn), ty = 16;
  while (ty > 1 && (ty * (n + 1) * (int)sizeof(c2<T>) > 66000 || ty * n / e > 1024)) ty >>= 1;
  return ty;
}
template <class T> __host__ __device__ constexpr int rows_threads(int logn) {
  return rows_ty<T>(logn) * (1 << logn) / fft_elems(logn);
}
template <class T> __host__ __device__ constexpr int cols_cx(int logn) {
  int n = 1 << logn, e = fft_elems(logn), cx = 8;
  while (cx > 1 && (2 * cx * (n + 1) * (int)sizeof(c2<T>) > 66000 || 2 * cx * n / e > 1024)) cx >>= 1;
  return cx;
}
template <class T> __host__ __device__ constexpr int cols_threads(int logn) {
  return 2 * cols_cx<T>(logn) * (1 << logn) / fft_elems(logn);
}

// ------------------------------------------------------------------ pass 1
template <class T, class S, int LOGN, bool INV>
__global__ void __launch_bounds__(rows_threads<T>(LOGN))
k_rows_fwd(const c2<S>* __restrict__ x, const c2<T>* __restrict__ chi, c2<T>* __restrict__ W,
           const c2<T>* __restrict__ tw, int nx, int nrows, int sets_per_rhs,
           const int* __restrict__ live) {
  constexpr int N = 1 << LOGN, TY = rows_ty<T>(LOGN), NT = rows_threads<T>(LOGN), LD = N + 1;
  __shared__ c2<T> buf[TY * LD];
  const int s = blockIdx.y;
  if (live && !live[s / sets_per_rhs]) return;
  const int y0 = blockIdx.x * TY;
  const c2<S>* xs = x + (size_t)s * nrows * nx;
  for (int e = threadIdx.x; e < TY * N; e += NT) {
    const int row = e >> LOGN, ix = e & (N - 1), yy = y0 + row;
    c2<T> v = mk<T>(0, 0);
    if (ix < nx && yy < nrows) {
      v = ld<T, S>(xs + (size_t)yy * nx + ix);
      if (chi) v = cmul<T>(v, chi[(size_t)yy * nx + ix]);
    }
    buf[row * LD + ix] = v;
  }
  __syncthreads();
  lds_fft<T, LOGN, INV>(buf, LD, tw, threadIdx.x, NT);
  c2<T>* Ws = W + (size_t)s * N * nrows;
  for (int e = threadIdx.x; e < TY * N; e += NT) {
    const int row = e % TY, ix = e / TY, yy = y0 + row;
    if (yy < nrows) Ws[(size_t)ix * nrows + yy] = buf[row * LD + ix];
  }
}

// ------------------------------------------------------------------ pass 2
template <class T, int LOGN>
__global__ void __launch_bounds__(cols_threads<T>(LOGN))
k_cols_symbol(c2<T>* __restrict__ W, const c2<T>* __restrict__ sym, const c2<T>* __restrict__ tw,
              int ncols, int nrows, const int* __restrict__ live) {
  constexpr int N = 1 << LOGN, CX = cols_cx<T>(LOGN), NT = cols_threads<T>(LOGN), LD = N + 1;
  __shared__ c2<T> buf[2 * CX * LD];
  const int r = blockIdx.y;
  if (live && !live[r]) return;
  const int x0 = blockIdx.x * CX;
  c2<T>* Wr = W + (size_t)r * 2 * ncols * nrows;
  // transform t = c * CX + cx holds column x0 + cx of component c
  for (int e = threadIdx.x; e < 2 * CX * N; e += NT) {
    const int t = e >> LOGN, ky = e & (N - 1), c = t / CX, xx = x0 + t % CX;
    c2<T> v = mk<T>(0, 0);
    if (ky < nrows && xx < ncols) v = Wr[((size_t)c * ncols + xx) * nrows + ky];
    buf[t * LD + ky] = v;
  }
  __syncthreads();
  lds_fft<T, LOGN, false>(buf, LD, tw, threadIdx.x, NT);
  for (int e = threadIdx.x; e < CX * N; e += NT) {
    const int cx = e >> LOGN, ky = e & (N - 1), xx = x0 + cx;
    if (xx < ncols) {
      const c2<T>* sp = sym + ((size_t)xx * N + ky) * 3;
      const c2<T> s11 = sp[0], s12 = sp[1], s22 = sp[2];
      const c2<T> a = buf[cx * LD + ky], b = buf[(CX + cx) * LD + ky];
      buf[cx * LD + ky] = cadd<T>(cmul<T>(s11, a), cmul<T>(s12, b));
      buf[(CX + cx) * LD + ky] = cadd<T>(cmul<T>(s12, a), cmul<T>(s22, b));
    }
  }
  __syncthreads();
  lds_fft<T, LOGN, true>(buf, LD, tw, threadIdx.x, NT);
  for (int e = threadIdx.x; e < 2 * CX * N; e += NT) {
    const int t = e >> LOGN, ky = e & (N - 1), c = t / CX, xx = x0 + t % CX;
    if (ky < nrows && xx < ncols) Wr[((size_t)c * ncols + xx) * nrows + ky] = buf[t * LD + ky];
  }
}

// Full-length transforms along the contiguous axis of W[set][col][0:N] (setup and diagnostics).
template <class T, int LOGN, bool INV>
__global__ void __launch_bounds__(cols_threads<T>(LOGN))
k_cols_plain(c2<T>* __restrict__ W, const c2<T>* __restrict__ tw, int ncols) {
  constexpr int N = 1 << LOGN, NTR = 2 * cols_cx<T>(LOGN), NT = cols_threads<T>(LOGN), LD = N + 1;
  __shared__ c2<T> buf[NTR * LD];
  const int s = blockIdx.y;
  const int x0 = blockIdx.x * NTR;
  c2<T>* Ws = W + (size_t)s * ncols * N;
  for (int e = threadIdx.x; e < NTR * N; e += NT) {
    const int t = e >> LOGN, ky = e & (N - 1), xx = x0 + t;
    buf[t * LD + ky] = xx < ncols ? Ws[(size_t)xx * N + ky] : mk<T>(0, 0);
  }
  __syncthreads();
  lds_fft<T, LOGN, INV>(buf, LD, tw, threadIdx.x, NT);
  for (int e = threadIdx.x; e < NTR * N; e += NT) {
    const int t = e >> LOGN, ky = e & (N - 1), xx = x0 + t;
    if (xx < ncols) Ws[(size_t)xx * N + ky] = buf[t * LD + ky];
  }
}

// ------------------------------------------------------------------ pass 3
template <class T, class S, int LOGN>
__global__ void __launch_bounds__(rows_threads<T>(LOGN))
k_rows_inv_sub(const c2<T>* __restrict__ W, const c2<S>* __restrict__ u, c2<S>* __restrict__ y,
               const c2<T>* __restrict__ tw, int nx, int nrows, int sets_per_rhs,
               const int* __restrict__ live) {
  constexpr int N = 1 << LOGN, TY = rows_ty<T>(LOGN), NT = rows_threads<T>(LOGN), LD = N + 1;
  __shared__ c2<T> buf[TY * LD];
  const int s = blockIdx.y;
  if (live && !live[s / sets_per_rhs]) return;
  const int y0 = blockIdx.x * TY;
  const c2<T>* Ws = W + (size_t)s * N * nrows;
  for (int e = threadIdx.x; e < TY * N; e += NT) {
    const int row = e % TY, ix = e / TY, yy = y0 + row;
    buf[row * LD + ix] = yy < nrows ? Ws[(size_t)ix * nrows + yy] : mk<T>(0, 0);
  }
  __syncthreads();
  lds_fft<T, LOGN, true>(buf, LD, tw, threadIdx.x, NT);
  const size_t so = (size_t)s * nrows * nx;
  for (int e = threadIdx.x; e < TY * N; e += NT) {
    const int row = e >> LOGN, ix = e & (N - 1), yy = y0 + row;
    if (ix < nx && yy < nrows) {
      const size_t o = so + (size_t)yy * nx + ix;
      st<S, T>(y + o, csub<T>(ld<T, S>(u + o), buf[row * LD + ix]));
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
  __syncthreads();
  for (int k = ty; k < 32; k += 8) {
    const int cc = c0 + k, rr = r0 + tx;
    if (rr < rows && cc < cols) ob[(size_t)cc * rows + rr] = tile[tx][k];
  }
}

__global__ void __launch_bounds__(256) k_pack_symbol(const double2* __restrict__ W, double2* __restrict__ s64,
                                                     float2* __restrict__ s32, size_t plane, double scale) {
  const size_t e = (size_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= plane) return;
  for (int a = 0; a < 3; ++a) {
    double2 v = W[a * plane + e];
    v.x *= scale;
    v.y *= scale;
    s64[e * 3 + a] = v;
    s32[e * 3 + a] = make_float2((float)v.x, (float)v.y);
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

template <class T, class S>
hipError_t launch_rows_fwd(int logn, bool inverse, const c2<S>* x, const c2<T>* chi, c2<T>* W, int nx,
                           int nrows, int nsets, int sets_per_rhs, const int* live, hipStream_t st) {
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nsets <= 0 || nrows <= 0) return hipSuccess;
  switch (logn) {
#define CASE(L)                                                                                    \
  case L: {                                                                                        \
    dim3 grid((nrows + rows_ty<T>(L) - 1) / rows_ty<T>(L), nsets);                                 \
    if (inverse)                                                                                   \
      hipLaunchKernelGGL((k_rows_fwd<T, S, L, true>), grid, dim3(rows_threads<T>(L)), 0, st, x, chi, W, tw, \
                         nx, nrows, sets_per_rhs, live);                                           \
    else                                                                                           \
      hipLaunchKernelGGL((k_rows_fwd<T, S, L, false>), grid, dim3(rows_threads<T>(L)), 0, st, x, chi, W, tw, \
                         nx, nrows, sets_per_rhs, live);                                           \
    break;                                                                                         \
  }
    DIE_LOGN_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T>
hipError_t launch_cols_symbol(int logn, c2<T>* W, const c2<T>* sym, int ncols, int nrows, int nrhs,
                              const int* live, hipStream_t st) {
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nrhs <= 0) return hipSuccess;
  switch (logn) {
#define CASE(L)                                                                                    \
  case L: {                                                                                        \
    dim3 grid((ncols + cols_cx<T>(L) - 1) / cols_cx<T>(L), nrhs);                                  \
    hipLaunchKernelGGL((k_cols_symbol<T, L>), grid, dim3(cols_threads<T>(L)), 0, st, W, sym, tw, ncols, \
                       nrows, live);                                                               \
    break;                                                                                         \
  }
    DIE_LOGN_CASES(CASE)
#undef CASE
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class T, class S>
hipError_t launch_rows_inv_sub(int logn, const c2<T>* W, const c2<S>* u, c2<S>* y, int nx, int nrows,
                               int nsets, int sets_per_rhs, const int* live, hipStream_t st) {
  const c2<T>* tw = table_for<T>();
  if (!tw) return hipErrorNotInitialized;
  if (nsets <= 0 || nrows <= 0) return hipSuccess;
  switch (logn) {
#define CASE(L)                                                                                    \
  case L: {                                                                                        \
    dim3 grid((nrows + rows_ty<T>(L) - 1) / rows_ty<T>(L), nsets);                                 \
    hipLaunchKernelGGL((k_rows_inv_sub<T, S, L>), grid, dim3(rows_threads<T>(L)), 0, st, W, u, y, tw, nx, \
                       nrows, sets_per_rhs, live);                                                 \
    break;                                                                                         \
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
#define CASE(L)                                                                                    \
  case L: {                                                                                        \
    const int ntr = 2 * cols_cx<T>(L);                                                             \
    dim3 grid((ncols + ntr - 1) / ntr, nsets);                                                     \
    if (inverse)                                                                                   \
      hipLaunchKernelGGL((k_cols_plain<T, L, true>), grid, dim3(cols_threads<T>(L)), 0, st, W, tw, ncols); \
    else                                                                                           \
      hipLaunchKernelGGL((k_cols_plain<T, L, false>), grid, dim3(cols_threads<T>(L)), 0, st, W, tw, ncols); \
    break;                                                                                         \
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

hipError_t launch_pack_symbol(const double2* W, double2* s64, float2* s32, int px, int py, double scale,
                              hipStream_t st) {
  const size_t plane = (size_t)px * py;
  hipLaunchKernelGGL(k_pack_symbol, dim3((unsigned)((plane + 255) / 256)), dim3(256), 0, st, W, s64, s32,
                     plane, scale);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_rows_fwd<double, double>(int, bool, const double2*, const double2*, double2*, int,
                                                    int, int, int, const int*, hipStream_t);
template hipError_t launch_rows_fwd<float, float>(int, bool, const float2*, const float2*, float2*, int, int,
                                                  int, int, const int*, hipStream_t);
template hipError_t launch_cols_symbol<double>(int, double2*, const double2*, int, int, int, const int*,
                                               hipStream_t);
template hipError_t launch_cols_symbol<float>(int, float2*, const float2*, int, int, int, const int*,
                                              hipStream_t);
template hipError_t launch_rows_inv_sub<double, double>(int, const double2*, const double2*, double2*, int,
                                                        int, int, int, const int*, hipStream_t);
template hipError_t launch_rows_inv_sub<float, float>(int, const float2*, const float2*, float2*, int, int,
                                                      int, int, const int*, hipStream_t);
template hipError_t launch_cols_plain<double>(int, bool, double2*, int, int, hipStream_t);
template hipError_t launch_cols_plain<float>(int, bool, float2*, int, int, hipStream_t);
template hipError_t launch_transpose<double>(const double2*, double2*, int, int, int, hipStream_t);
template hipError_t launch_transpose<float>(const float2*, float2*, int, int, int, hipStream_t);

}  // namespace die
