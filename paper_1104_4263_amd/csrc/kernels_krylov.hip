// Krylov kernels: multi-dot / multi-axpy for classical Gram-Schmidt with one
// re-orthogonalisation (CGS2) in the Arnoldi process of restarted GMRES, the
// deflation projector x + V (C (V^* x)), norms, scaling, and the FP64 Givens
// least-squares update of the GMRES Hessenberg column.  All reductions are
// two-stage (per-block partials, then a fixed-order sum), so results are
// deterministic run to run.
#include "ops.hpp"

#include <algorithm>
#include <cmath>

namespace die {

namespace {

constexpr int NT = kBlasThreads;
constexpr int EPT = kBlasEpt;
constexpr int NW = NT / 64;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Sum over the block; the result is valid in thread 0.  `red` holds NW entries.
__device__ __forceinline__ double2 block_sum(double2 v, double2* red) {
  v.x = wave_sum(v.x);
  v.y = wave_sum(v.y);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  lds_sync();
  double2 s = make_double2(0.0, 0.0);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NW; ++k) { s.x += red[k].x; s.y += red[k].y; }
  }
  lds_sync();
  return s;
}

__device__ __forceinline__ double block_sum1(double v, double* red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red[w] = v;
  lds_sync();
  double s = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < NW; ++k) s += red[k];
  }
  lds_sync();
  return s;
}

// Cross-block partial sums: the partials are written and read with agent-scope atomic
// accesses, which are coherent across the XCDs' L2 caches without a cache write-back;
// waiting for the stores to complete (vmcnt 0) orders them before the counter update.
__device__ __forceinline__ void st_agent(double2* p, double2 v) {
  __hip_atomic_store(&p->x, v.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&p->y, v.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double2 ld_agent(const double2* p) {
  return make_double2(__hip_atomic_load(&p->x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
                      __hip_atomic_load(&p->y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ bool arrive_last(int* counter, int total) {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  return __hip_atomic_fetch_add(counter, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == total - 1;
}

__device__ __forceinline__ double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 zcmul(double2 a, double2 b) {  // conj(a) * b
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

}  // namespace

// ---------------------------------------------------------------- multi-dot
template <class SA, class SB>
__global__ void __launch_bounds__(NT)
k_mdot(const c2<SA>* __restrict__ A, size_t a_vs, size_t a_rs, int nv, const int* __restrict__ nv_dev,
       const c2<SB>* __restrict__ B, size_t b_rs, size_t n, double2* __restrict__ part,
       const int* __restrict__ live) {
  const int r = blockIdx.y;
  if (live && !live[r]) return;
  __shared__ double2 red[NW];
  const int nblk = gridDim.x;
  const int nvr = nv_dev ? min(nv_dev[r], nv) : nv;
  const size_t e0 = (size_t)blockIdx.x * NT * EPT + threadIdx.x;
  const c2<SB>* Br = B + (size_t)r * b_rs;
  double2 b[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = e0 + (size_t)k * NT;
    b[k] = e < n ? ld<double, SB>(Br + e) : make_double2(0.0, 0.0);
  }
  for (int i = 0; i < nv; ++i) {
    double2 acc = make_double2(0.0, 0.0);
    if (i < nvr) {
      const c2<SA>* Ai = A + (size_t)i * a_vs + (size_t)r * a_rs;
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        const size_t e = e0 + (size_t)k * NT;
        if (e < n) {
          const double2 a = ld<double, SA>(Ai + e);
          const double2 p = zcmul(a, b[k]);
          acc.x += p.x;
          acc.y += p.y;
        }
      }
    }
    acc = block_sum(acc, red);
    if (threadIdx.x == 0) part[((size_t)r * nv + i) * nblk + blockIdx.x] = acc;
  }
}

// ---------------------------------------------------------------- reduce
constexpr int kMaxReduceNv = 1024;

__global__ void __launch_bounds__(NT)
k_reduce(const double2* __restrict__ part, int nv, int nblk, double sign, const double2* __restrict__ C,
         double2* __restrict__ out, const int* __restrict__ live) {
  const int r = blockIdx.x;
  if (live && !live[r]) return;
  __shared__ double2 tmp[kMaxReduceNv];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int i = w; i < nv; i += NW) {
    const double2* p = part + ((size_t)r * nv + i) * nblk;
    double sx = 0.0, sy = 0.0;
    for (int b = lane; b < nblk; b += 64) { sx += p[b].x; sy += p[b].y; }
    sx = wave_sum(sx);
    sy = wave_sum(sy);
    if (lane == 0) tmp[i] = make_double2(sign * sx, sign * sy);
  }
  lds_sync();
  for (int i = threadIdx.x; i < nv; i += NT) {
    double2 v;
    if (C) {
      v = make_double2(0.0, 0.0);
      for (int l = 0; l < nv; ++l) {
        const double2 p = zmul(C[(size_t)i * nv + l], tmp[l]);
        v.x += p.x;
        v.y += p.y;
      }
    } else {
      v = tmp[i];
    }
    out[(size_t)r * nv + i] = v;
  }
}

// ---------------------------------------------------------------- multi-axpy
template <class SA, class SX, class SY, int MODE>
__global__ void __launch_bounds__(NT)
k_maxpy(const c2<SA>* __restrict__ A, size_t a_vs, size_t a_rs, int nv, const int* __restrict__ nv_dev,
        const double2* __restrict__ coef, int ldc, const c2<SX>* X, size_t x_rs, double alpha, c2<SY>* Y,
        size_t y_rs, double beta, size_t n, double2* __restrict__ part, double* __restrict__ partn,
        const int* __restrict__ live) {
  const int r = blockIdx.y;
  if (live && !live[r]) return;
  __shared__ double2 red[NW];
  __shared__ double red1[NW];
  const int nblk = gridDim.x;
  const int nvr = nv_dev ? min(nv_dev[r], nv) : nv;
  const size_t e0 = (size_t)blockIdx.x * NT * EPT + threadIdx.x;
  c2<SY>* Yr = Y + (size_t)r * y_rs;
  const c2<SX>* Xr = X ? X + (size_t)r * x_rs : nullptr;
  double2 y[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = e0 + (size_t)k * NT;
    double2 v = make_double2(0.0, 0.0);
    if (e < n) {
      if (beta != 0.0) {
        const double2 yo = ld<double, SY>(Yr + e);
        v.x = beta * yo.x;
        v.y = beta * yo.y;
      }
      if (Xr) {
        const double2 xv = ld<double, SX>(Xr + e);
        v.x += alpha * xv.x;
        v.y += alpha * xv.y;
      }
    }
    y[k] = v;
  }
  for (int i = 0; i < nvr; ++i) {
    const double2 c = coef[(size_t)r * ldc + i];
    const c2<SA>* Ai = A + (size_t)i * a_vs + (size_t)r * a_rs;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const size_t e = e0 + (size_t)k * NT;
      if (e < n) {
        const double2 p = zmul(c, ld<double, SA>(Ai + e));
        y[k].x += p.x;
        y[k].y += p.y;
      }
    }
  }
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = e0 + (size_t)k * NT;
    if (e < n) {
      st<SY, double>(Yr + e, y[k]);
      y[k] = ld<double, SY>(Yr + e);  // continue with the stored (rounded) value
    }
  }
  if constexpr (MODE == 1) {
    for (int i = 0; i < nv; ++i) {
      double2 acc = make_double2(0.0, 0.0);
      if (i < nvr) {
        const c2<SA>* Ai = A + (size_t)i * a_vs + (size_t)r * a_rs;
#pragma unroll
        for (int k = 0; k < EPT; ++k) {
          const size_t e = e0 + (size_t)k * NT;
          if (e < n) {
            const double2 p = zcmul(ld<double, SA>(Ai + e), y[k]);
            acc.x += p.x;
            acc.y += p.y;
          }
        }
      }
      acc = block_sum(acc, red);
      if (threadIdx.x == 0) part[((size_t)r * nv + i) * nblk + blockIdx.x] = acc;
    }
  } else if constexpr (MODE == 2) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < EPT; ++k) s += y[k].x * y[k].x + y[k].y * y[k].y;
    s = block_sum1(s, red1);
    if (threadIdx.x == 0) partn[(size_t)r * nblk + blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------- norms, scaling
template <class S>
__global__ void __launch_bounds__(NT)
k_norm2(const c2<S>* __restrict__ X, size_t x_rs, size_t n, double* __restrict__ partn,
        const int* __restrict__ live) {
  const int r = blockIdx.y;
  if (live && !live[r]) return;
  __shared__ double red1[NW];
  const size_t e0 = (size_t)blockIdx.x * NT * EPT + threadIdx.x;
  const c2<S>* Xr = X + (size_t)r * x_rs;
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = e0 + (size_t)k * NT;
    if (e < n) {
      const double2 v = ld<double, S>(Xr + e);
      s += v.x * v.x + v.y * v.y;
    }
  }
  s = block_sum1(s, red1);
  if (threadIdx.x == 0) partn[(size_t)r * gridDim.x + blockIdx.x] = s;
}

__global__ void __launch_bounds__(64)
k_reduce_norm(const double* __restrict__ partn, int nblk, double* __restrict__ out, const int* __restrict__ live) {
  const int r = blockIdx.x;
  if (live && !live[r]) return;
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s += partn[(size_t)r * nblk + b];
  s = wave_sum(s);
  if (threadIdx.x == 0) out[r] = s;
}

template <class SX, class SY>
__global__ void __launch_bounds__(NT)
k_scale(const c2<SX>* X, size_t x_rs, c2<SY>* Y, size_t y_rs, const double* __restrict__ scale, int sstride,
        size_t n, const int* __restrict__ live) {
  const int r = blockIdx.y;
  if (live && !live[r]) return;
  const double s = scale[(size_t)r * sstride];
  const size_t e0 = (size_t)blockIdx.x * NT * EPT + threadIdx.x;
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = e0 + (size_t)k * NT;
    if (e < n) {
      const double2 v = ld<double, SX>(X + (size_t)r * x_rs + e);
      st<SY, double>(Y + (size_t)r * y_rs + e, make_double2(s * v.x, s * v.y));
    }
  }
}

// ---------------------------------------------------------------- Givens / least squares
__global__ void __launch_bounds__(64)
k_givens(const double2* __restrict__ h1, const double2* __restrict__ h2, int ldh, double hsign,
         const double* __restrict__ partn,
         int nblk, GmresState* __restrict__ state, double2* __restrict__ Rm, double* __restrict__ cs,
         double2* __restrict__ sn, double2* __restrict__ g, double2* __restrict__ y, int m, int* __restrict__ live,
         const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (!live[r] || (active && !active[r])) return;
  double s2 = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) s2 += partn[(size_t)r * nblk + b];
  s2 = wave_sum(s2);
  if (threadIdx.x != 0) return;
  GmresState S = state[r];
  if (S.done) return;
  const int j = S.j;
  const int ld = m + 1;
  double2* R = Rm + (size_t)r * ld * m;
  double2* gr = g + (size_t)r * ld;
  double* csr = cs + (size_t)r * m;
  double2* snr = sn + (size_t)r * m;
  const double beta = sqrt(s2);
  for (int i = 0; i <= j; ++i) {
    const double2 a = h1[(size_t)r * ldh + i];
    const double2 b = h2 ? h2[(size_t)r * ldh + i] : make_double2(0.0, 0.0);
    R[i + (size_t)j * ld] = make_double2(hsign * (a.x + b.x), hsign * (a.y + b.y));
  }
  for (int i = 0; i < j; ++i) {
    const double c = csr[i];
    const double2 s = snr[i];
    const double2 a = R[i + (size_t)j * ld], b = R[i + 1 + (size_t)j * ld];
    const double2 sb = zmul(s, b);
    const double2 sa = zcmul(s, a);  // conj(s) * a
    R[i + (size_t)j * ld] = make_double2(c * a.x + sb.x, c * a.y + sb.y);
    R[i + 1 + (size_t)j * ld] = make_double2(c * b.x - sa.x, c * b.y - sa.y);
  }
  const double2 a = R[j + (size_t)j * ld];
  const double absa = hypot(a.x, a.y);
  const double rho = hypot(absa, beta);
  double c;
  double2 s;
  if (absa > 0.0) {
    c = absa / rho;
    s = make_double2(a.x / absa * beta / rho, a.y / absa * beta / rho);
    R[j + (size_t)j * ld] = make_double2(a.x / absa * rho, a.y / absa * rho);
  } else {
    c = 0.0;
    s = make_double2(1.0, 0.0);
    R[j + (size_t)j * ld] = make_double2(beta, 0.0);
  }
  csr[j] = c;
  snr[j] = s;
  const double2 gj = gr[j];
  gr[j] = make_double2(c * gj.x, c * gj.y);
  const double2 sg = zcmul(s, gj);  // conj(s) * g_j
  gr[j + 1] = make_double2(-sg.x, -sg.y);
  const double resid = hypot(gr[j + 1].x, gr[j + 1].y);
  const int j1 = j + 1;
  const bool fin = isfinite(resid) && isfinite(rho) && rho > 0.0;
  S.j = j1;
  S.resid = resid;
  S.invbeta = (beta > 0.0 && fin) ? 1.0 / beta : 0.0;
  if (!fin) S.breakdown = 1;
  if (!fin || resid <= S.target || j1 >= m) {
    S.done = 1;
    live[r] = 0;
    double2* yr = y + (size_t)r * m;
    if (fin) {
      for (int i = j1 - 1; i >= 0; --i) {
        double2 acc = gr[i];
        for (int l = i + 1; l < j1; ++l) {
          const double2 p = zmul(R[i + (size_t)l * ld], yr[l]);
          acc.x -= p.x;
          acc.y -= p.y;
        }
        const double2 d = R[i + (size_t)i * ld];
        const double dd = d.x * d.x + d.y * d.y;
        yr[i] = make_double2((acc.x * d.x + acc.y * d.y) / dd, (acc.y * d.x - acc.x * d.y) / dd);
      }
    } else {
      for (int i = 0; i < j1; ++i) yr[i] = make_double2(0.0, 0.0);
    }
  }
  state[r] = S;
}

// ---------------------------------------------------------------- launchers
template <class SA, class SB>
hipError_t launch_mdot(const c2<SA>* A, size_t a_vs, size_t a_rs, int nv, const int* nv_dev, const c2<SB>* B,
                       size_t b_rs, size_t n, int nrhs, double2* part, const int* live, hipStream_t st) {
  if (nrhs <= 0 || nv <= 0) return hipSuccess;
  dim3 grid(blas_blocks(n), nrhs);
  hipLaunchKernelGGL((k_mdot<SA, SB>), grid, dim3(NT), 0, st, A, a_vs, a_rs, nv, nv_dev, B, b_rs, n, part, live);
  return hipGetLastError();
}

hipError_t launch_reduce(const double2* part, int nv, int nblk, int nrhs, double sign, const double2* C,
                         double2* out, const int* live, hipStream_t st) {
  if (nrhs <= 0 || nv <= 0) return hipSuccess;
  if (nv > kMaxReduceNv) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_reduce, dim3(nrhs), dim3(NT), 0, st, part, nv, nblk, sign, C, out, live);
  return hipGetLastError();
}

template <class SA, class SX, class SY>
hipError_t launch_maxpy(int mode, const c2<SA>* A, size_t a_vs, size_t a_rs, int nv, const int* nv_dev,
                        const double2* coef, int ldc, const c2<SX>* X, size_t x_rs, double alpha, c2<SY>* Y,
                        size_t y_rs, double beta, size_t n, int nrhs, double2* part, double* partn,
                        const int* live, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  dim3 grid(blas_blocks(n), nrhs);
  switch (mode) {
    case 0:
      hipLaunchKernelGGL((k_maxpy<SA, SX, SY, 0>), grid, dim3(NT), 0, st, A, a_vs, a_rs, nv, nv_dev, coef, ldc, X,
                         x_rs, alpha, Y, y_rs, beta, n, part, partn, live);
      break;
    case 1:
      hipLaunchKernelGGL((k_maxpy<SA, SX, SY, 1>), grid, dim3(NT), 0, st, A, a_vs, a_rs, nv, nv_dev, coef, ldc, X,
                         x_rs, alpha, Y, y_rs, beta, n, part, partn, live);
      break;
    case 2:
      hipLaunchKernelGGL((k_maxpy<SA, SX, SY, 2>), grid, dim3(NT), 0, st, A, a_vs, a_rs, nv, nv_dev, coef, ldc, X,
                         x_rs, alpha, Y, y_rs, beta, n, part, partn, live);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <class S>
hipError_t launch_norm2(const c2<S>* X, size_t x_rs, size_t n, int nrhs, double* partn, const int* live,
                        hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  dim3 grid(blas_blocks(n), nrhs);
  hipLaunchKernelGGL((k_norm2<S>), grid, dim3(NT), 0, st, X, x_rs, n, partn, live);
  return hipGetLastError();
}

hipError_t launch_reduce_norm(const double* partn, int nblk, int nrhs, double* out, const int* live,
                              hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_norm, dim3(nrhs), dim3(64), 0, st, partn, nblk, out, live);
  return hipGetLastError();
}

template <class SX, class SY>
hipError_t launch_scale(const c2<SX>* X, size_t x_rs, c2<SY>* Y, size_t y_rs, const double* scale, int sstride,
                        size_t n, int nrhs, const int* live, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  dim3 grid(blas_blocks(n), nrhs);
  hipLaunchKernelGGL((k_scale<SX, SY>), grid, dim3(NT), 0, st, X, x_rs, Y, y_rs, scale, sstride, n, live);
  return hipGetLastError();
}

hipError_t launch_givens(const double2* h1, const double2* h2, int ldh, double hsign, const double* partn,
                         int nblk, GmresState* state, double2* R, double* cs, double2* sn, double2* g, double2* y, int m,
                         int nrhs, int* live, const int* active, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_givens, dim3(nrhs), dim3(64), 0, st, h1, h2, ldh, hsign, partn, nblk, state, R, cs, sn, g, y, m,
                     live, active);
  return hipGetLastError();
}

// explicit instantiations (basis / vector precisions used by the solver)
#define DIE_INST_MDOT(SA, SB)                                                                              \
  template hipError_t launch_mdot<SA, SB>(const c2<SA>*, size_t, size_t, int, const int*, const c2<SB>*,   \
                                          size_t, size_t, int, double2*, const int*, hipStream_t);
DIE_INST_MDOT(double, double)
DIE_INST_MDOT(float, float)
DIE_INST_MDOT(double, float)
#define DIE_INST_MAXPY(SA, SX, SY)                                                                          \
  template hipError_t launch_maxpy<SA, SX, SY>(int, const c2<SA>*, size_t, size_t, int, const int*,          \
                                               const double2*, int, const c2<SX>*, size_t, double, c2<SY>*,  \
                                               size_t, double, size_t, int, double2*, double*, const int*,   \
                                               hipStream_t);
DIE_INST_MAXPY(double, double, double)
DIE_INST_MAXPY(float, float, float)
DIE_INST_MAXPY(double, float, float)
DIE_INST_MAXPY(double, float, double)
DIE_INST_MAXPY(float, float, double)
template hipError_t launch_norm2<double>(const double2*, size_t, size_t, int, double*, const int*, hipStream_t);
template hipError_t launch_norm2<float>(const float2*, size_t, size_t, int, double*, const int*, hipStream_t);
#define DIE_INST_SCALE(SX, SY)                                                                              \
  template hipError_t launch_scale<SX, SY>(const c2<SX>*, size_t, c2<SY>*, size_t, const double*, int,       \
                                           size_t, int, const int*, hipStream_t);
DIE_INST_SCALE(double, double)
DIE_INST_SCALE(float, float)
DIE_INST_SCALE(double, float)
DIE_INST_SCALE(float, double)

// u[idx[c]] += src[c] for c < k (vectors of n complex values; the sum in FP64).
template <class S>
__global__ void __launch_bounds__(NT)
k_add_cols(const c2<S>* __restrict__ src, size_t n, const int* __restrict__ idx, double2* __restrict__ u) {
  const int c = blockIdx.y;
  const c2<S>* sc = src + (size_t)c * n;
  double2* uc = u + (size_t)idx[c] * n;
  for (size_t e = (size_t)blockIdx.x * NT + threadIdx.x; e < n; e += (size_t)gridDim.x * NT) {
    const c2<S> a = sc[e];
    double2 v = uc[e];
    v.x += (double)a.x;
    v.y += (double)a.y;
    uc[e] = v;
  }
}

template <class S>
hipError_t launch_add_cols(const c2<S>* src, size_t n, const int* idx, int k, double2* u, hipStream_t st) {
  if (k <= 0 || n == 0) return hipSuccess;
  if (k > 65535) return hipErrorInvalidValue;
  dim3 grid((unsigned)std::min<size_t>((n + NT - 1) / NT, 1024), (unsigned)k);
  hipLaunchKernelGGL(k_add_cols<S>, grid, dim3(NT), 0, st, src, n, idx, u);
  return hipGetLastError();
}
template hipError_t launch_add_cols<double>(const double2*, size_t, const int*, int, double2*, hipStream_t);
template hipError_t launch_add_cols<float>(const float2*, size_t, const int*, int, double2*, hipStream_t);

}  // namespace die

// =====================================================================================
// Fused Arnoldi kernels for the GMRES inner loop.  Each kernel reduces its own partial
// sums: every block writes its partials, and the last block to finish (counted with a
// device-scope atomic) sums them in a fixed order, so results stay deterministic.
// =====================================================================================
namespace die {
namespace {

constexpr int kFusedMaxNv = 512;

}  // namespace

// Dot products out[r][i] = sign * conj(A_i,r) . B_r (optionally times C), GEMV style,
// one partial per (vector, chunk of kDotChunk elements) from one block reduction per
// vector.  WALK: one block per (chunk, rhs) loads its chunk of B_r once and walks all
// vectors in groups of kDotG (large batches).  Otherwise one block per (chunk, group of
// kDotG vectors, rhs), for more blocks when the batch is small; completion is then counted
// per (rhs, group) first.  The last block of rhs r (counted with agent-scope atomics)
// sums each vector's chunk partials in a fixed order and, when C is given, applies it.
// Both shapes compute the same partials and sums, so results do not depend on the shape.
// counter: [nrhs][kCounterStride] zeroed ints (left zeroed).
constexpr int kDotEpt = 8;
constexpr int kDotChunk = NT * kDotEpt;
constexpr int kDotG = 4;
constexpr int kNormGroup = 64;
static_assert(kDotChunk == kDotChunkElems, "partial-buffer sizing assumes this chunk");

// Accumulate conj(A_i) . b over this thread's kDotEpt elements for kDotG vectors, FP64
// fused multiply-adds on widened values.  FULL: the whole chunk is inside the vector.
template <class SA, bool FULL>
__device__ __forceinline__ void dots_group(const c2<SA>* __restrict__ Ar, size_t a_vs, int i0, int gn, size_t base,
                                           size_t n, const double2 (&b)[kDotEpt], double (&v)[2 * kDotG]) {
#pragma unroll
  for (int g = 0; g < kDotG; ++g) {
    double sx = 0.0, sy = 0.0;
    if (g < gn) {
      const c2<SA>* Ai = Ar + (size_t)(i0 + g) * a_vs + base;
#pragma unroll
      for (int k = 0; k < kDotEpt; ++k) {
        if (FULL || base + (size_t)k * NT < n) {
          const double2 a = ld<double, SA>(Ai + (size_t)k * NT);
          sx = fma(a.x, b[k].x, sx);
          sx = fma(a.y, b[k].y, sx);
          sy = fma(a.x, b[k].y, sy);
          sy = fma(-a.y, b[k].x, sy);
        }
      }
    }
    v[2 * g] = sx;
    v[2 * g + 1] = sy;
  }
}

template <class SA, class SB, bool WALK>
__global__ void __launch_bounds__(NT)
k_dots(const c2<SA>* __restrict__ A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const c2<SB>* __restrict__ B,
       size_t b_rs, size_t n, double2* __restrict__ part, double sign, const double2* __restrict__ C0,
       size_t c_stride, double2* __restrict__ out, int* __restrict__ counter, const int* __restrict__ live) {
  const int r = WALK ? blockIdx.y : blockIdx.z;
  if (live && !live[r]) return;
  // block reduction of the 2 kDotG values of every thread: transposed through LDS
  // (value v of thread t at red[v][t]); a team of 32 lanes per value then sums entries
  // l, l + 32, ..., l + 224 in lane l and finishes with a 32-lane butterfly.
  __shared__ double red[2 * kDotG][NT];
  __shared__ double2 acc[kFusedMaxNv];
  __shared__ int s_last;
  static_assert(2 * kDotG * 32 == NT, "one 32-lane team per reduced value");
  const int nchunk = gridDim.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const size_t base = (size_t)blockIdx.x * kDotChunk + t;
  const bool full = (size_t)(blockIdx.x + 1) * kDotChunk <= n;
  const c2<SA>* Ar = A + (size_t)(r / a_rpo) * a_rs;
  const double2* C = C0 ? C0 + (size_t)(r / a_rpo) * c_stride : nullptr;
  const c2<SB>* Br = B + (size_t)r * b_rs;
  double2 b[kDotEpt];
#pragma unroll
  for (int k = 0; k < kDotEpt; ++k) {
    const size_t e = base + (size_t)k * NT;
    b[k] = e < n ? ld<double, SB>(Br + e) : make_double2(0.0, 0.0);
  }
  const int ifirst = WALK ? 0 : blockIdx.y * kDotG, iend = WALK ? nv : min(nv, ifirst + kDotG);
  const int rv = t >> 5, rl = t & 31;  // reduced value and lane of this thread's team
  for (int i0 = ifirst; i0 < iend; i0 += kDotG) {
    const int gn = min(kDotG, nv - i0);
    double v[2 * kDotG];
    if (full) dots_group<SA, true>(Ar, a_vs, i0, gn, base, n, b, v);
    else dots_group<SA, false>(Ar, a_vs, i0, gn, base, n, b, v);
#pragma unroll
    for (int q = 0; q < 2 * kDotG; ++q) red[q][t] = v[q];
    lds_sync();
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 32; ++k) s += red[rv][k * 32 + rl];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) s += __shfl_xor(s, off, 32);
    if (rl == 0 && (rv >> 1) < gn) {
      double* dst = reinterpret_cast<double*>(part + ((size_t)r * nv + i0 + (rv >> 1)) * nchunk + blockIdx.x);
      __hip_atomic_store(dst + (rv & 1), s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    lds_sync();
  }
  // the partials were stored by lanes of every wave: each wave waits for its own stores
  // before the block's completion is counted
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  lds_sync();
  int* cnt = counter + (size_t)r * kCounterStride;
  if (!WALK) {  // first level: the chunks of this vector group
    if (t == 0) s_last = arrive_last(cnt + 1 + blockIdx.y, nchunk);
    lds_sync();
    if (!s_last) return;
    if (t == 0) {
      cnt[1 + blockIdx.y] = 0;
      s_last = arrive_last(cnt, gridDim.y);
    }
  } else if (t == 0) {
    s_last = arrive_last(cnt, nchunk);
  }
  lds_sync();
  if (!s_last) return;
  // last block of rhs r: sum each vector's chunk partials in a fixed order
  for (int g = w; g < nv; g += NW) {
    const double2* p = part + ((size_t)r * nv + g) * nchunk;
    double ax = 0.0, ay = 0.0;
    for (int c = lane; c < nchunk; c += 64) {
      const double2 v = ld_agent(p + c);
      ax += v.x;
      ay += v.y;
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    if (lane == 0) {
      const double2 v = make_double2(sign * ax, sign * ay);
      if (C) acc[g] = v;
      else out[(size_t)r * nv + g] = v;
    }
  }
  if (t == 0) cnt[0] = 0;
  if (!C) return;
  lds_sync();
  for (int ii = t; ii < nv; ii += NT) {
    double2 v = make_double2(0.0, 0.0);
    for (int l = 0; l < nv; ++l) {
      const double2 q = zmul(C[(size_t)ii * nv + l], acc[l]);
      v.x += q.x;
      v.y += q.y;
    }
    out[(size_t)r * nv + ii] = v;
  }
}

// W_r += sum_i coef[r * nv + i] A_i,r (element parallel, EPT elements per thread so that
// EPT loads of each basis vector are in flight together).  GIVENS: also beta = ||W_r||
// (last block) and the Givens update of column j = nv - 1 with h = -(h1neg + coef).
template <class SA, class SW, bool GIVENS, int EPT>
__global__ void __launch_bounds__(NT)
k_axpy(const c2<SA>* __restrict__ A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const double2* __restrict__ coef,
       const c2<SW>* X, c2<SW>* W, size_t w_rs, size_t n, double2* __restrict__ part, int* __restrict__ counter,
       const int* __restrict__ live_in, const double2* __restrict__ h1, GmresState* __restrict__ state,
       double2* __restrict__ Rm, double* __restrict__ cs, double2* __restrict__ sn, double2* __restrict__ g, int m,
       int* __restrict__ live_out) {
  const int r = blockIdx.y;
  if (live_in && !live_in[r]) return;
  __shared__ int s_last;
  const int nblk = gridDim.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  c2<SW>* Wr = W + (size_t)r * w_rs;
  const c2<SW>* Xr = X ? X + (size_t)r * w_rs : Wr;
  const c2<SA>* Ar = A + (size_t)(r / a_rpo) * a_rs;
  const size_t base = (size_t)blockIdx.x * (NT * EPT) + t;
  double2 y[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = base + (size_t)k * NT;
    y[k] = e < n ? ld<double, SW>(Xr + e) : make_double2(0.0, 0.0);
  }
  const bool full = (size_t)(blockIdx.x + 1) * (NT * EPT) <= n;
  for (int i = 0; i < nv; ++i) {
    const double2 cf = coef[(size_t)r * nv + i];
    const c2<SA>* Ai = Ar + (size_t)i * a_vs + base;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      if (full || base + (size_t)k * NT < n) {
        const double2 a = ld<double, SA>(Ai + (size_t)k * NT);
        y[k].x = fma(cf.x, a.x, y[k].x);
        y[k].x = fma(-cf.y, a.y, y[k].x);
        y[k].y = fma(cf.x, a.y, y[k].y);
        y[k].y = fma(cf.y, a.x, y[k].y);
      }
    }
  }
  double s2[EPT];
#pragma unroll
  for (int k = 0; k < EPT; ++k) {
    const size_t e = base + (size_t)k * NT;
    s2[k] = 0.0;
    if (e < n) {
      const c2<SW> v = mk<SW>((SW)y[k].x, (SW)y[k].y);
      Wr[e] = v;
      if constexpr (GIVENS) s2[k] = (double)v.x * (double)v.x + (double)v.y * (double)v.y;  // of the stored value
    }
  }
  if constexpr (GIVENS) {
    // one partial per 256 consecutive elements (whatever EPT is), so the sum of squares is
    // associated the same way for every launch shape
    __shared__ double red1[EPT][NW];
    const int npart = nblk * EPT;
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const double v = wave_sum(s2[k]);
      if (lane == 0) red1[k][w] = v;
    }
    lds_sync();
    if (t < EPT) {  // wave 0 only: its vmcnt wait below orders these stores before the count
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NW; ++k) v += red1[t][k];
      st_agent(part + (size_t)r * npart + (size_t)blockIdx.x * EPT + t, make_double2(v, 0.0));
    }
    // two-level completion count: groups of kNormGroup partials, then the groups
    int* cnt = counter + (size_t)r * kCounterStride;
    constexpr int kBlocksPerGroup = kNormGroup / EPT;
    const int grp = blockIdx.x / kBlocksPerGroup, ngrp = (nblk + kBlocksPerGroup - 1) / kBlocksPerGroup;
    const int gblocks = min(kBlocksPerGroup, nblk - grp * kBlocksPerGroup);
    if (t == 0) s_last = arrive_last(cnt + 1 + grp, gblocks);
    lds_sync();
    if (!s_last) return;
    double2* gpart = part + (size_t)gridDim.y * npart;  // group sums after the partials
    const int gsize = gblocks * EPT;
    if (w == 0) {
      double gs = 0.0;
      for (int c = grp * kNormGroup + lane; c < grp * kNormGroup + gsize; c += 64)
        gs += ld_agent(part + (size_t)r * npart + c).x;
      gs = wave_sum(gs);
      if (lane == 0) {
        st_agent(gpart + (size_t)r * ngrp + grp, make_double2(gs, 0.0));
        cnt[1 + grp] = 0;
        s_last = arrive_last(cnt, ngrp);
      }
    }
    lds_sync();
    if (!s_last) return;
    __shared__ double2 col[kFusedMaxNv + 1];
    __shared__ double s_beta;
    __shared__ GmresState S;
    if (w == 0) {
      double bs = 0.0;
      for (int c = lane; c < ngrp; c += 64) bs += ld_agent(gpart + (size_t)r * ngrp + c).x;
      bs = wave_sum(bs);
      if (lane == 0) {
        s_beta = sqrt(bs);
        S = state[r];
        cnt[0] = 0;
      }
    }
    lds_sync();
    if (S.done) return;
    const int j = S.j, ld = m + 1;
    double2* R = Rm + (size_t)r * ld * m;
    double2* gr = g + (size_t)r * ld;
    double* csr = cs + (size_t)r * m;
    double2* snr = sn + (size_t)r * m;
    for (int i = t; i <= j; i += NT) {
      const double2 a = h1[(size_t)r * nv + i], b = coef[(size_t)r * nv + i];
      col[i] = make_double2(-(a.x + b.x), -(a.y + b.y));
    }
    lds_sync();
    if (t == 0) {
      // apply the previous rotations to the new column, then the new rotation
      const double beta = s_beta;
      for (int i = 0; i < j; ++i) {
        const double c = csr[i];
        const double2 sv = snr[i];
        const double2 a = col[i], b = col[i + 1];
        const double2 sb = zmul(sv, b), sa = zcmul(sv, a);
        col[i] = make_double2(c * a.x + sb.x, c * a.y + sb.y);
        col[i + 1] = make_double2(c * b.x - sa.x, c * b.y - sa.y);
      }
      const double2 a = col[j];
      const double absa = hypot(a.x, a.y), rho = hypot(absa, beta);
      double c;
      double2 sv;
      if (absa > 0.0) {
        c = absa / rho;
        sv = make_double2(a.x / absa * beta / rho, a.y / absa * beta / rho);
        col[j] = make_double2(a.x / absa * rho, a.y / absa * rho);
      } else {
        c = 0.0;
        sv = make_double2(1.0, 0.0);
        col[j] = make_double2(beta, 0.0);
      }
      csr[j] = c;
      snr[j] = sv;
      const double2 gj = gr[j];
      gr[j] = make_double2(c * gj.x, c * gj.y);
      const double2 sgj = zcmul(sv, gj);
      gr[j + 1] = make_double2(-sgj.x, -sgj.y);
      const double resid = hypot(sgj.x, sgj.y);
      const bool fin = isfinite(resid) && isfinite(rho) && rho > 0.0;
      GmresState Sn = S;
      Sn.j = j + 1;
      Sn.resid = resid;
      Sn.invbeta = (beta > 0.0 && fin) ? 1.0 / beta : 0.0;
      if (!fin) Sn.breakdown = 1;
      if (!fin || resid <= Sn.target || j + 1 >= m) {
        Sn.done = 1;
        live_out[r] = 0;
      }
      state[r] = Sn;
    }
    lds_sync();
    for (int i = t; i <= j; i += NT) R[i + (size_t)j * ld] = col[i];
  }
}

// y_r = R_r^-1 g_r for the j_r leading columns (cycle end), one wave per rhs, column
// oriented so each step is a parallel update.
__global__ void __launch_bounds__(64)
k_lsq(const GmresState* __restrict__ state, const double2* __restrict__ Rm, const double2* __restrict__ g,
      double2* __restrict__ y, int m, const int* __restrict__ active) {
  const int r = blockIdx.x;
  if (active && !active[r]) return;
  const GmresState S = state[r];
  const int jj = S.j, ld = m + 1, lane = threadIdx.x;
  const double2* R = Rm + (size_t)r * ld * m;
  double2* yr = y + (size_t)r * m;
  __shared__ double2 rhs[kFusedMaxNv];
  for (int i = lane; i < jj; i += 64) rhs[i] = g[(size_t)r * ld + i];
  lds_sync();
  for (int i = jj - 1; i >= 0; --i) {
    const double2 d = R[i + (size_t)i * ld];
    const double dd = d.x * d.x + d.y * d.y;
    const double2 a = rhs[i];
    const double2 yi = S.breakdown ? make_double2(0.0, 0.0)
                                   : make_double2((a.x * d.x + a.y * d.y) / dd, (a.y * d.x - a.x * d.y) / dd);
    if (lane == 0) yr[i] = yi;
    for (int l = lane; l < i; l += 64) {
      const double2 p = zmul(R[l + (size_t)i * ld], yi);
      rhs[l].x -= p.x;
      rhs[l].y -= p.y;
    }
    lds_sync();
  }
}

// Elements per thread of the multi-axpys: the largest power of two (up to 8) that still
// leaves about 2048 blocks (8 per CU) in the launch.
// ==================================================================== one-reduction Arnoldi
// CGS2 with the second projection of each new vector delayed to the next step (one
// block reduction and one pass of multi-axpys over the basis per step).  At step j of a
// cycle the basis holds q_0..q_{j-1} (final), the slot j holds v (the new vector after
// one projection, not yet normalised) and the slot j+1 holds w = M P^-1 v.
//   s = Q^H v, alpha = v^H v, z = Q^H w, beta = v^H w          (k_dots2, one pass)
//   nu = sqrt(alpha - |s|^2),  q_j = (v - Q s) / nu,
//   column j-1 of H = c_{j-1} + s with subdiagonal nu            (k_dcgs_update)
//   t = H s,  h_j = [(z - t_{<j}) / nu ; ((beta - s^H z) / nu - t_j) / nu],
//   d = t + nu h_j,  v_{j+1} = (w - Q d_{<j} - q_j d_j) / nu      (k_dcgs_axpy, one pass)
// using the Arnoldi relation M P^-1 Q = Q H to turn w into M P^-1 q_j without a product.
// c_j = h_j is the first projection of the next column.

constexpr int kDots2G = 2;  // vectors per group: 2 vectors x 2 targets x (re, im) = 8 values

// Two consecutive complex values in one access (8 bytes for binary16 parts, 16 for float,
// 32 for double).  The one-reduction kernels give each thread pairs (2t, 2t + 1) of every
// 2 NT elements; vector lengths are even (two field components), so a pair is either whole
// inside a vector or whole outside.
template <class S> struct alignas(2 * sizeof(c2<S>)) cpair {
  c2<S> a, b;
};
template <class A, class S> __device__ __forceinline__ void ld_pair(const c2<S>* p, c2<A>& x, c2<A>& y) {
  const cpair<S> v = *reinterpret_cast<const cpair<S>*>(p);
  x = mk<A>((A)v.a.x, (A)v.a.y);
  y = mk<A>((A)v.b.x, (A)v.b.y);
}
template <class S, class A> __device__ __forceinline__ cpair<S> mk_pair(c2<A> x, c2<A> y) {
  cpair<S> v;
  v.a = mk<S>((S)x.x, (S)x.y);
  v.b = mk<S>((S)y.x, (S)y.y);
  return v;
}

// Arithmetic inside a thread of the one-reduction kernels: FP64 for FP64 and FP32 bases;
// FP32 for the binary16 basis, whose storage rounding (2^-11) is far above FP32 rounding
// (2^-24), and where the binary16 operand widens inside the fused multiply-add
// (v_fma_mix_f32) instead of through two conversions.  Sums across threads and blocks,
// and every coefficient the scalar step computes, stay FP64.
template <class SQ> struct arn_acc { using type = double; };
template <> struct arn_acc<_Float16> { using type = float; };
__device__ __forceinline__ float afma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double afma(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <class SQ, class A, bool FULL>
__device__ __forceinline__ void dots2_group(const c2<SQ>* __restrict__ Qr, size_t q_vs, int i0, int gn, size_t base,
                                            size_t n, const c2<A> (&b0)[kDotEpt], const c2<A> (&b1)[kDotEpt],
                                            double (&v)[8]) {
#pragma unroll
  for (int g = 0; g < kDots2G; ++g) {
    A s0x = 0, s0y = 0, s1x = 0, s1y = 0;
    if (g < gn) {
      const c2<SQ>* Ai = Qr + (size_t)(i0 + g) * q_vs + base;
      cpair<SQ> raw[kDotEpt / 2];  // kept in storage precision until used
#pragma unroll
      for (int p = 0; p < kDotEpt / 2; ++p) {
        if (FULL || base + (size_t)p * 2 * NT < n) {
          raw[p] = *reinterpret_cast<const cpair<SQ>*>(Ai + (size_t)p * 2 * NT);
        } else {
          raw[p].a = mk<SQ>((SQ)0, (SQ)0);
          raw[p].b = raw[p].a;
        }
      }
#pragma unroll
      for (int k = 0; k < kDotEpt; ++k) {
        {
          const c2<SQ> ak = (k & 1) ? raw[k / 2].b : raw[k / 2].a;
          const A ax = (A)ak.x, ay = (A)ak.y;
          s0x = afma(ax, b0[k].x, s0x);
          s0x = afma(ay, b0[k].y, s0x);
          s0y = afma(ax, b0[k].y, s0y);
          s0y = afma(-ay, b0[k].x, s0y);
          s1x = afma(ax, b1[k].x, s1x);
          s1x = afma(ay, b1[k].y, s1x);
          s1y = afma(ax, b1[k].y, s1y);
          s1y = afma(-ay, b1[k].x, s1y);
        }
      }
    }
    v[4 * g + 0] = (double)s0x;
    v[4 * g + 1] = (double)s0y;
    v[4 * g + 2] = (double)s1x;
    v[4 * g + 3] = (double)s1y;
  }
}

// out[r ostride + 2 i + t] = conj(A_i,r) . T_t,r for A_0..A_{nq-1} = Q, A_nq = V, T_0 = V,
// T_1 = W (W null: T_1 = 0).  Same shapes and fixed-order sums as k_dots.  The basis Q is
// stored in SQ, V and W in SV.
template <class SQ, class SV, bool WALK>
__global__ void __launch_bounds__(NT)
k_dots2(const c2<SQ>* __restrict__ Q, size_t q_vs, int nq, const c2<SV>* __restrict__ V,
        const c2<SV>* __restrict__ Wt, size_t rs, size_t n, double2* __restrict__ part, double2* __restrict__ out,
        int ostride, int* __restrict__ counter, const int* __restrict__ live) {
  const int r = WALK ? blockIdx.y : blockIdx.z;
  if (live && !live[r]) return;
  __shared__ double red[8][NT];
  __shared__ int s_last;
  const int nA = nq + 1, nchunk = gridDim.x, t = threadIdx.x, w = t >> 6, lane = t & 63;
  const size_t base = (size_t)blockIdx.x * kDotChunk + 2 * t;  // pairs (base + 2 p NT, + 1)
  const bool full = (size_t)(blockIdx.x + 1) * kDotChunk <= n;
  const c2<SQ>* Qr = Q + (size_t)r * rs;
  const c2<SV>* Vr = V + (size_t)r * rs;
  const c2<SV>* Wr = Wt ? Wt + (size_t)r * rs : nullptr;
  using A = typename arn_acc<SQ>::type;
  c2<A> b0[kDotEpt], b1[kDotEpt];
#pragma unroll
  for (int p = 0; p < kDotEpt / 2; ++p) {
    const size_t e = base + (size_t)p * 2 * NT;
    b0[2 * p] = b0[2 * p + 1] = b1[2 * p] = b1[2 * p + 1] = mk<A>((A)0, (A)0);
    if (e < n) {
      ld_pair<A, SV>(Vr + e, b0[2 * p], b0[2 * p + 1]);
      if (Wr) ld_pair<A, SV>(Wr + e, b1[2 * p], b1[2 * p + 1]);
    }
  }
  const int ifirst = WALK ? 0 : blockIdx.y * kDots2G, iend = WALK ? nA : min(nA, ifirst + kDots2G);
  const int rv = t >> 5, rl = t & 31;
  // 8 values per thread -> one sum per 32-lane team -> partials of vectors i0 .. i0 + gn - 1
  auto reduce_store = [&](const double (&v)[8], int i0, int gn) {
#pragma unroll
    for (int q = 0; q < 8; ++q) red[q][t] = v[q];
    lds_sync();
    double sum = 0.0;
#pragma unroll
    for (int k = 0; k < NT / 32; ++k) sum += red[rv][k * 32 + rl];
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 32);
    const int gv = rv >> 2, tg = (rv >> 1) & 1, comp = rv & 1;
    if (rl == 0 && gv < gn) {
      double* dst =
          reinterpret_cast<double*>(part + (((size_t)r * nA + i0 + gv) * 2 + tg) * nchunk + blockIdx.x);
      __hip_atomic_store(dst + comp, sum, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    lds_sync();
  };
  // basis vectors Q_i, i < nq
  for (int i0 = ifirst; i0 < min(iend, nq); i0 += kDots2G) {
    const int gn = min(kDots2G, nq - i0);
    double v[8];
    if (full) dots2_group<SQ, A, true>(Qr, q_vs, i0, gn, base, n, b0, b1, v);
    else dots2_group<SQ, A, false>(Qr, q_vs, i0, gn, base, n, b0, b1, v);
    reduce_store(v, i0, gn);
  }
  // A_nq = V: v^H v and v^H w from the target values already in registers
  if (ifirst <= nq && nq < iend) {
    A a[4] = {0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kDotEpt; ++k) {
      a[0] = afma(b0[k].x, b0[k].x, a[0]);
      a[0] = afma(b0[k].y, b0[k].y, a[0]);
      a[2] = afma(b0[k].x, b1[k].x, a[2]);
      a[2] = afma(b0[k].y, b1[k].y, a[2]);
      a[3] = afma(b0[k].x, b1[k].y, a[3]);
      a[3] = afma(-b0[k].y, b1[k].x, a[3]);
    }
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = q < 4 ? (double)a[q] : 0.0;
    reduce_store(v, nq, 1);
  }
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
  lds_sync();
  int* cnt = counter + (size_t)r * kCounterStride;
  if (!WALK) {
    if (t == 0) s_last = arrive_last(cnt + 1 + blockIdx.y, nchunk);
    lds_sync();
    if (!s_last) return;
    if (t == 0) {
      cnt[1 + blockIdx.y] = 0;
      s_last = arrive_last(cnt, gridDim.y);
    }
  } else if (t == 0) {
    s_last = arrive_last(cnt, nchunk);
  }
  lds_sync();
  if (!s_last) return;
  for (int g = w; g < 2 * nA; g += NW) {
    const double2* p = part + ((size_t)r * nA * 2 + g) * nchunk;
    double ax = 0.0, ay = 0.0;
    for (int c = lane; c < nchunk; c += 64) {
      const double2 u = ld_agent(p + c);
      ax += u.x;
      ay += u.y;
    }
    ax = wave_sum(ax);
    ay = wave_sum(ay);
    if (lane == 0) out[(size_t)r * ostride + g] = make_double2(ax, ay);
  }
  if (t == 0) cnt[0] = 0;
}

// Scalar work of step j for one right-hand side (one block of 64 threads per rhs): the
// delayed correction and Givens rotation of column j-1, the stopping test, and the
// coefficients of k_dcgs_axpy.  D: [nrhs][dstride] from k_dots2; Hu: unrotated H
// [nrhs][(m+1) m]; c: [nrhs][m+1] first projection of the last column; coef: [nrhs][2(m+1)]
// (s at 0..j-1, d at m+1 .. m+1+j).
__global__ void __launch_bounds__(64)
k_dcgs_update(const double2* __restrict__ D, int dstride, int j, int m, GmresState* __restrict__ state,
              double2* __restrict__ Hu, double2* __restrict__ Rm, double* __restrict__ cs, double2* __restrict__ sn,
              double2* __restrict__ g, double2* __restrict__ c, double2* __restrict__ coef, int* __restrict__ live) {
  const int r = blockIdx.x, lane = threadIdx.x;
  if (!live[r]) return;
  __shared__ double2 col[kFusedMaxNv + 1], tt[kFusedMaxNv + 1];
  __shared__ double s_nu;
  __shared__ int s_stop;
  const int ld = m + 1;
  const double2* Dr = D + (size_t)r * dstride;  // Dr[2 i + 0] = q_i^H v, Dr[2 i + 1] = q_i^H w
  double2* Hr = Hu + (size_t)r * ld * m;
  double2* cr = c + (size_t)r * ld;
  double2* kr = coef + (size_t)r * 2 * ld;
  double s2 = 0.0;
  for (int i = lane; i < j; i += 64) {
    const double2 si = Dr[2 * i];
    s2 += si.x * si.x + si.y * si.y;
  }
  s2 = wave_sum(s2);
  if (lane == 0) {
    const double alpha = Dr[2 * j].x;
    const double nu2 = alpha - s2;
    GmresState S = state[r];
    // nu2 <= 0 (up to rounding) means v lies in span(Q): a lucky breakdown, nu = 0
    const bool ok = isfinite(nu2);
    const double nu = ok ? sqrt(fmax(nu2, 0.0)) : 0.0;
    s_nu = nu;
    int stop = 0;
    if (!ok) {
      S.breakdown = 1;
      stop = 1;
    } else if (j == 0) {
      const double2 g0 = g[(size_t)r * ld];  // q_0 = v / nu, so the start residual is beta0 nu q_0
      g[(size_t)r * ld] = make_double2(g0.x * nu, g0.y * nu);
      if (!(nu > 0.0)) {
        S.breakdown = 1;
        stop = 1;
      }
    }
    S.invbeta = nu > 0.0 ? 1.0 / nu : 0.0;
    s_stop = stop;
    state[r] = S;
  }
  lds_sync();
  const double nu = s_nu;
  if (j >= 1 && !s_stop) {
    // column j-1 of H: c_{j-1} + s, subdiagonal nu
    for (int i = lane; i < j; i += 64) {
      const double2 a = cr[i], si = Dr[2 * i];
      col[i] = make_double2(a.x + si.x, a.y + si.y);
      Hr[i + (size_t)(j - 1) * ld] = col[i];
    }
    if (lane == 0) {
      col[j] = make_double2(nu, 0.0);
      Hr[j + (size_t)(j - 1) * ld] = col[j];
    }
    lds_sync();
    if (lane == 0) {
      GmresState S = state[r];
      const int jc = j - 1;  // the column being rotated
      double* csr = cs + (size_t)r * m;
      double2* snr = sn + (size_t)r * m;
      double2* gr = g + (size_t)r * ld;
      for (int i = 0; i < jc; ++i) {
        const double cc = csr[i];
        const double2 sv = snr[i];
        const double2 a = col[i], b = col[i + 1];
        const double2 sb = zmul(sv, b), sa = zcmul(sv, a);
        col[i] = make_double2(cc * a.x + sb.x, cc * a.y + sb.y);
        col[i + 1] = make_double2(cc * b.x - sa.x, cc * b.y - sa.y);
      }
      const double2 a = col[jc];
      const double absa = hypot(a.x, a.y), rho = hypot(absa, nu);
      double cc;
      double2 sv;
      if (absa > 0.0) {
        cc = absa / rho;
        sv = make_double2(a.x / absa * nu / rho, a.y / absa * nu / rho);
        col[jc] = make_double2(a.x / absa * rho, a.y / absa * rho);
      } else {
        cc = 0.0;
        sv = make_double2(1.0, 0.0);
        col[jc] = make_double2(nu, 0.0);
      }
      csr[jc] = cc;
      snr[jc] = sv;
      const double2 gj = gr[jc];
      gr[jc] = make_double2(cc * gj.x, cc * gj.y);
      const double2 sgj = zcmul(sv, gj);
      gr[jc + 1] = make_double2(-sgj.x, -sgj.y);
      const double resid = hypot(sgj.x, sgj.y);
      const bool fin = isfinite(resid) && isfinite(rho) && rho > 0.0;
      S.j = j;
      S.resid = resid;
      if (!fin) S.breakdown = 1;
      if (!fin || resid <= S.target || j >= m || !(nu > 0.0)) s_stop = 1;
      state[r] = S;
    }
    lds_sync();
    for (int i = lane; i <= j - 1; i += 64) Rm[(size_t)r * ld * m + i + (size_t)(j - 1) * ld] = col[i];
  }
  lds_sync();
  if (s_stop || j >= m) {
    if (lane == 0) {
      GmresState S = state[r];
      S.done = 1;
      S.j = j;
      state[r] = S;
      live[r] = 0;
    }
    return;
  }
  // t = H s over the finalised columns 0..j-1 (rows 0..j), then h_j and d
  for (int i = lane; i <= j; i += 64) {
    double2 acc = make_double2(0.0, 0.0);
    for (int l = (i > 0 ? i - 1 : 0); l < j; ++l) {
      const double2 p = zmul(Hr[i + (size_t)l * ld], Dr[2 * l]);
      acc.x += p.x;
      acc.y += p.y;
    }
    tt[i] = acc;
  }
  double2 sz = make_double2(0.0, 0.0);
  for (int i = lane; i < j; i += 64) {
    const double2 p = zcmul(Dr[2 * i], Dr[2 * i + 1]);
    sz.x += p.x;
    sz.y += p.y;
  }
  sz.x = wave_sum(sz.x);
  sz.y = wave_sum(sz.y);
  lds_sync();
  const double inu = 1.0 / nu;
  for (int i = lane; i <= j; i += 64) {
    double2 h;
    if (i < j) {
      const double2 zi = Dr[2 * i + 1];
      h = make_double2((zi.x - tt[i].x) * inu, (zi.y - tt[i].y) * inu);
      kr[i] = Dr[2 * i];  // s_i
    } else {
      const double2 beta = Dr[2 * j + 1];
      h = make_double2(((beta.x - sz.x) * inu - tt[i].x) * inu, ((beta.y - sz.y) * inu - tt[i].y) * inu);
    }
    cr[i] = h;
    kr[ld + i] = make_double2(tt[i].x + nu * h.x, tt[i].y + nu * h.y);  // d_i
  }
}

// q_j = (v - Q s) / nu into basis slot j and v_{j+1} = (w - Q d_{<j} - q_j d_j) / nu into V
// (in place), one pass over Q_0..Q_{j-1} (EPT elements per thread).  Basis in SQ, V and W
// in SV; d_j multiplies the stored (rounded) q_j.
template <class SQ, class SV, int EPT>
__global__ void __launch_bounds__(NT)
k_dcgs_axpy(c2<SQ>* __restrict__ Q, size_t q_vs, int j, c2<SV>* __restrict__ V, const c2<SV>* __restrict__ Wt,
            size_t rs, size_t n, const double2* __restrict__ coef, int cld, const GmresState* __restrict__ state,
            const int* __restrict__ live) {
  const int r = blockIdx.y;
  if (!live[r]) return;
  using A = typename arn_acc<SQ>::type;
  const A inu = (A)state[r].invbeta;
  c2<SQ>* Qr = Q + (size_t)r * rs;
  c2<SQ>* Qj = Qr + (size_t)j * q_vs;
  c2<SV>* Vr = V + (size_t)r * rs;
  const c2<SV>* Wr = Wt + (size_t)r * rs;
  const double2* sr = coef + (size_t)r * 2 * cld;
  const double2* dr = sr + cld;
  static_assert(EPT % 2 == 0, "pairs of elements");
  constexpr int NPR = EPT / 2;
  const size_t base = (size_t)blockIdx.x * (NT * EPT) + 2 * threadIdx.x;  // pairs (base + 2 p NT, + 1)
  const bool full = (size_t)(blockIdx.x + 1) * (NT * EPT) <= n;
  c2<A> aq[EPT], aw[EPT];
#pragma unroll
  for (int p = 0; p < NPR; ++p) {
    const size_t e = base + (size_t)p * 2 * NT;
    aq[2 * p] = aq[2 * p + 1] = aw[2 * p] = aw[2 * p + 1] = mk<A>((A)0, (A)0);
    if (full || e < n) {
      ld_pair<A, SV>(Vr + e, aq[2 * p], aq[2 * p + 1]);
      ld_pair<A, SV>(Wr + e, aw[2 * p], aw[2 * p + 1]);
    }
  }
  for (int i = 0; i < j; ++i) {
    const c2<A> si = mk<A>((A)sr[i].x, (A)sr[i].y), di = mk<A>((A)dr[i].x, (A)dr[i].y);
    const c2<SQ>* Ai = Qr + (size_t)i * q_vs + base;
#pragma unroll
    for (int p = 0; p < NPR; ++p) {
      if (full || base + (size_t)p * 2 * NT < n) {
        const cpair<SQ> raw = *reinterpret_cast<const cpair<SQ>*>(Ai + (size_t)p * 2 * NT);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = 2 * p + h;
          const c2<SQ> a = h ? raw.b : raw.a;
          const A ax = (A)a.x, ay = (A)a.y;
          aq[k].x = afma(-si.x, ax, aq[k].x);
          aq[k].x = afma(si.y, ay, aq[k].x);
          aq[k].y = afma(-si.x, ay, aq[k].y);
          aq[k].y = afma(-si.y, ax, aq[k].y);
          aw[k].x = afma(-di.x, ax, aw[k].x);
          aw[k].x = afma(di.y, ay, aw[k].x);
          aw[k].y = afma(-di.x, ay, aw[k].y);
          aw[k].y = afma(-di.y, ax, aw[k].y);
        }
      }
    }
  }
  const c2<A> dj = mk<A>((A)dr[j].x, (A)dr[j].y);
#pragma unroll
  for (int p = 0; p < NPR; ++p) {
    const size_t e = base + (size_t)p * 2 * NT;
    if (full || e < n) {
      const cpair<SQ> q = mk_pair<SQ, A>(mk<A>(aq[2 * p].x * inu, aq[2 * p].y * inu),
                                         mk<A>(aq[2 * p + 1].x * inu, aq[2 * p + 1].y * inu));
      *reinterpret_cast<cpair<SQ>*>(Qj + e) = q;
      c2<A> y[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const c2<SQ> qh = h ? q.b : q.a;
        const A qx = (A)qh.x, qy = (A)qh.y;  // the stored (rounded) q_j
        c2<A> yy = aw[2 * p + h];
        yy.x = afma(-dj.x, qx, yy.x);
        yy.x = afma(dj.y, qy, yy.x);
        yy.y = afma(-dj.x, qy, yy.y);
        yy.y = afma(-dj.y, qx, yy.y);
        y[h] = mk<A>(yy.x * inu, yy.y * inu);
      }
      *reinterpret_cast<cpair<SV>*>(Vr + e) = mk_pair<SV, A>(y[0], y[1]);
    }
  }
}

inline int blocks_split(size_t units, int nrhs) {
  int e = 8;
  while (e > 1 && ((units + e - 1) / e) * (size_t)nrhs < 2048) e >>= 1;
  return e;
}

template <class SA, class SW, bool GIVENS>
hipError_t launch_axpy_ept(const c2<SA>* A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const double2* coef,
                           const c2<SW>* X, c2<SW>* W, size_t w_rs, size_t n, int nrhs, double2* part, int* counter,
                           const int* live_in, const double2* h1, GmresState* state, double2* R, double* cs,
                           double2* sn, double2* g, int m, int* live_out, hipStream_t st) {
  const int ept = blocks_split((n + NT - 1) / NT, nrhs);
  dim3 grid((unsigned)((n + (size_t)NT * ept - 1) / ((size_t)NT * ept)), nrhs);
#define DIE_AXPY_CASE(E)                                                                                         \
  case E:                                                                                                        \
    hipLaunchKernelGGL((k_axpy<SA, SW, GIVENS, E>), grid, dim3(NT), 0, st, A, a_vs, a_rs, a_rpo, nv, coef, X, W, \
                       w_rs, n, part, counter, live_in, h1, state, R, cs, sn, g, m, live_out);                   \
    break;
  switch (ept) {
    DIE_AXPY_CASE(1)
    DIE_AXPY_CASE(2)
    DIE_AXPY_CASE(4)
    DIE_AXPY_CASE(8)
    default: return hipErrorInvalidValue;
  }
#undef DIE_AXPY_CASE
  return hipGetLastError();
}

template <class SA, class SB>
hipError_t launch_fdot(const c2<SA>* A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const c2<SB>* B, size_t b_rs,
                       size_t n, int nrhs, double2* part, double sign, const double2* C, size_t c_stride,
                       double2* out, int* counter, const int* live, hipStream_t st) {
  if (nrhs <= 0 || nv <= 0) return hipSuccess;
  if (nv > kFusedMaxNv) return hipErrorInvalidValue;
  const unsigned nchunk = (unsigned)((n + kDotChunk - 1) / kDotChunk);
  if (a_rpo < 1) a_rpo = 1;
  if ((size_t)nchunk * nrhs >= 2048) {
    hipLaunchKernelGGL((k_dots<SA, SB, true>), dim3(nchunk, nrhs), dim3(NT), 0, st, A, a_vs, a_rs, a_rpo, nv, B,
                       b_rs, n, part, sign, C, c_stride, out, counter, live);
  } else {
    const unsigned ngrp = (unsigned)((nv + kDotG - 1) / kDotG);
    hipLaunchKernelGGL((k_dots<SA, SB, false>), dim3(nchunk, ngrp, nrhs), dim3(NT), 0, st, A, a_vs, a_rs, a_rpo, nv,
                       B, b_rs, n, part, sign, C, c_stride, out, counter, live);
  }
  return hipGetLastError();
}

template <class SA, class SW>
hipError_t launch_faxpy(const c2<SA>* A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const double2* coef,
                        const c2<SW>* X, c2<SW>* W, size_t w_rs, size_t n, int nrhs, const int* live,
                        hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (a_rpo < 1) a_rpo = 1;
  return launch_axpy_ept<SA, SW, false>(A, a_vs, a_rs, a_rpo, nv, coef, X, W, w_rs, n, nrhs, nullptr, nullptr, live,
                                        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0, nullptr, st);
}

template <class SA, class SW>
hipError_t launch_faxpy_givens(const c2<SA>* A, size_t a_vs, size_t a_rs, int nv, const double2* h2neg,
                               const double2* h1neg, c2<SW>* W, size_t w_rs, size_t n, int nrhs, double2* part,
                               int* counter, GmresState* state, double2* R, double* cs, double2* sn, double2* g,
                               int m, int* live, hipStream_t st) {
  if (nrhs <= 0 || nv <= 0) return hipSuccess;
  return launch_axpy_ept<SA, SW, true>(A, a_vs, a_rs, 1, nv, h2neg, (const c2<SW>*)nullptr, W, w_rs, n, nrhs, part,
                                       counter, live, h1neg, state, R, cs, sn, g, m, live, st);
}

hipError_t launch_lsq(const GmresState* state, const double2* R, const double2* g, double2* y, int m, int nrhs,
                      const int* active, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (m > kFusedMaxNv) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lsq, dim3(nrhs), dim3(64), 0, st, state, R, g, y, m, active);
  return hipGetLastError();
}

template <class SQ, class SV>
hipError_t launch_dots2(const c2<SQ>* Q, size_t q_vs, int nq, const c2<SV>* V, const c2<SV>* W, size_t rs, size_t n,
                        int nrhs, double2* part, double2* out, int ostride, int* counter, const int* live,
                        hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (nq < 0 || nq + 1 > kFusedMaxNv || ostride < 2 * (nq + 1) || n % 2) return hipErrorInvalidValue;
  const unsigned nchunk = (unsigned)((n + kDotChunk - 1) / kDotChunk);
  if ((size_t)nchunk * nrhs >= 2048) {
    hipLaunchKernelGGL((k_dots2<SQ, SV, true>), dim3(nchunk, nrhs), dim3(NT), 0, st, Q, q_vs, nq, V, W, rs, n, part,
                       out, ostride, counter, live);
  } else {
    const unsigned ngrp = (unsigned)((nq + 1 + kDots2G - 1) / kDots2G);
    hipLaunchKernelGGL((k_dots2<SQ, SV, false>), dim3(nchunk, ngrp, nrhs), dim3(NT), 0, st, Q, q_vs, nq, V, W, rs,
                       n, part, out, ostride, counter, live);
  }
  return hipGetLastError();
}

hipError_t launch_dcgs_update(const double2* D, int dstride, int j, int m, int nrhs, GmresState* state, double2* Hu,
                              double2* R, double* cs, double2* sn, double2* g, double2* c, double2* coef, int* live,
                              hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (m > kFusedMaxNv || j > m) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_dcgs_update, dim3(nrhs), dim3(64), 0, st, D, dstride, j, m, state, Hu, R, cs, sn, g, c, coef,
                     live);
  return hipGetLastError();
}

template <class SQ, class SV>
hipError_t launch_dcgs_axpy(c2<SQ>* Q, size_t q_vs, int j, c2<SV>* V, const c2<SV>* W, size_t rs, size_t n, int nrhs,
                            const double2* coef, int ld, const GmresState* state, const int* live, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  // at most 4 elements per thread: 8 needs 84 VGPRs and measured 4.4 against 5.3 TB/s
  if (n % 2) return hipErrorInvalidValue;  // pairs of elements
  const int ept = std::max(2, std::min(4, blocks_split((n + NT - 1) / NT, nrhs)));
  dim3 grid((unsigned)((n + (size_t)NT * ept - 1) / ((size_t)NT * ept)), nrhs);
#define DIE_DCGS_CASE(E)                                                                                       \
  case E:                                                                                                      \
    hipLaunchKernelGGL((k_dcgs_axpy<SQ, SV, E>), grid, dim3(NT), 0, st, Q, q_vs, j, V, W, rs, n, coef, ld, state, \
                       live);                                                                                  \
    break;
  switch (ept) {
    DIE_DCGS_CASE(2)
    DIE_DCGS_CASE(4)
    default: return hipErrorInvalidValue;
  }
#undef DIE_DCGS_CASE
  return hipGetLastError();
}

#define DIE_INST_DCGS(SQ, SV)                                                                                      \
  template hipError_t launch_dots2<SQ, SV>(const c2<SQ>*, size_t, int, const c2<SV>*, const c2<SV>*, size_t,       \
                                           size_t, int, double2*, double2*, int, int*, const int*, hipStream_t);   \
  template hipError_t launch_dcgs_axpy<SQ, SV>(c2<SQ>*, size_t, int, c2<SV>*, const c2<SV>*, size_t, size_t, int,  \
                                               const double2*, int, const GmresState*, const int*, hipStream_t);
DIE_INST_DCGS(double, double)
DIE_INST_DCGS(float, float)
DIE_INST_DCGS(_Float16, float)
template hipError_t launch_maxpy<_Float16, float, float>(int, const half2c*, size_t, size_t, int, const int*,
                                                         const double2*, int, const float2*, size_t, double, float2*,
                                                         size_t, double, size_t, int, double2*, double*, const int*,
                                                         hipStream_t);

#define DIE_INST_FUSED(SA, SB)                                                                                    \
  template hipError_t launch_fdot<SA, SB>(const c2<SA>*, size_t, size_t, int, int, const c2<SB>*, size_t, size_t, \
                                          int, double2*, double, const double2*, size_t, double2*, int*, const int*, \
                                          hipStream_t);
DIE_INST_FUSED(double, double)
DIE_INST_FUSED(float, float)
DIE_INST_FUSED(double, float)
#define DIE_INST_FAXPY(SA, SW)                                                                                     \
  template hipError_t launch_faxpy<SA, SW>(const c2<SA>*, size_t, size_t, int, int, const double2*,              \
                                           const c2<SW>*, c2<SW>*, size_t, size_t, int, const int*, hipStream_t);   \
  template hipError_t launch_faxpy_givens<SA, SW>(const c2<SA>*, size_t, size_t, int, const double2*,              \
                                                  const double2*, c2<SW>*, size_t, size_t, int, double2*, int*,     \
                                                  GmresState*, double2*, double*, double2*, double2*, int, int*,    \
                                                  hipStream_t);
DIE_INST_FAXPY(double, double)
DIE_INST_FAXPY(float, float)
template hipError_t launch_faxpy<double, float>(const double2*, size_t, size_t, int, int, const double2*,
                                                const float2*, float2*, size_t, size_t, int, const int*, hipStream_t);


// ---- helpers of the alternative Krylov solvers and of the dense operator

// X[j][e] = 1 if e == col0 + j else 0 (complex128), j < ncols, e < n.
__global__ void k_unit_cols(double2* __restrict__ X, size_t n, size_t col0, int ncols) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (e >= n || j >= ncols) return;
  X[(size_t)j * n + e] = make_double2(e == col0 + (size_t)j ? 1.0 : 0.0, 0.0);
}

// Y_r = c[r][0] X0_r + c[r][1] X1_r + c[r][2] X2_r for live right-hand sides (an input may be null,
// or alias Y: each element is read before it is written by the same thread).
__global__ void k_comb3(double2* __restrict__ Y, const double2* X0, const double2* X1, const double2* X2,
                        const double2* __restrict__ coef, size_t n, const int* __restrict__ live) {
  const int r = blockIdx.y;
  if (live && !live[r]) return;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const size_t o = (size_t)r * n + e;
  double2 acc = make_double2(0.0, 0.0);
  const double2* cr = coef + (size_t)r * 3;
  if (X0) acc = cadd<double>(acc, cmul<double>(cr[0], X0[o]));
  if (X1) acc = cadd<double>(acc, cmul<double>(cr[1], X1[o]));
  if (X2) acc = cadd<double>(acc, cmul<double>(cr[2], X2[o]));
  Y[o] = acc;
}

hipError_t launch_unit_cols(double2* X, size_t n, size_t col0, int ncols, hipStream_t st) {
  if (ncols < 1 || ncols > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_unit_cols, dim3((unsigned)((n + 255) / 256), (unsigned)ncols), dim3(256), 0, st, X, n, col0,
                     ncols);
  return hipGetLastError();
}

hipError_t launch_comb3(double2* Y, const double2* X0, const double2* X1, const double2* X2, const double2* coef,
                        size_t n, int nrhs, const int* live, hipStream_t st) {
  if (nrhs <= 0) return hipSuccess;
  if (nrhs > 65535) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_comb3, dim3((unsigned)((n + 255) / 256), (unsigned)nrhs), dim3(256), 0, st, Y, X0, X1, X2, coef,
                     n, live);
  return hipGetLastError();
}

}  // namespace die
