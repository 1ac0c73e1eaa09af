// LDS-resident Stockham FFT for power-of-two lengths up to 4096 (gfx950).
//
// A block holds NB transforms of length N = 2^LOGN in LDS (transform b starts
// at buf + b * stride).  Every stage is a Stockham autosort step of radix
// R = 2^LOGR: butterfly i of a transform reads x[i + q N/R] (q < R), multiplies
// by w^(q k), k = i mod p (p = product of the radices already applied,
// w = exp(-+2 pi i / (p R))), runs an in-register DFT of size R and writes
// y[(i - k) R + k + q p].  The output is in natural order.  Stages are radix 8
// (the first stage takes the remaining 1 or 2 bits), so a 4096-point transform
// needs 4 LDS round trips.  Each thread owns E = 8 values per stage.
#pragma once
#include "common.hpp"

namespace die {

__device__ __forceinline__ double2 twiddle_ld(const double2* t, int j) { return t[j]; }
__device__ __forceinline__ float2 twiddle_ld(const float2* t, int j) { return t[j]; }

template <class T, bool INV> __device__ __forceinline__ void dft2(c2<T>* v) {
  c2<T> a = v[0];
  v[0] = cadd<T>(a, v[1]);
  v[1] = csub<T>(a, v[1]);
}

template <class T, bool INV> __device__ __forceinline__ void dft4(c2<T>* v) {
  c2<T> a0 = cadd<T>(v[0], v[2]), a1 = csub<T>(v[0], v[2]);
  c2<T> b0 = cadd<T>(v[1], v[3]), b1 = csub<T>(v[1], v[3]);
  b1 = INV ? mul_pi<T>(b1) : mul_mi<T>(b1);
  v[0] = cadd<T>(a0, b0);
  v[2] = csub<T>(a0, b0);
  v[1] = cadd<T>(a1, b1);
  v[3] = csub<T>(a1, b1);
}

template <class T, bool INV> __device__ __forceinline__ void dft8(c2<T>* v) {
  c2<T> e[4] = {v[0], v[2], v[4], v[6]};
  c2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const T c = (T)0.70710678118654752440084436210485;
  c2<T> t1 = INV ? mk<T>(c * (o[1].x - o[1].y), c * (o[1].x + o[1].y))
                 : mk<T>(c * (o[1].x + o[1].y), c * (o[1].y - o[1].x));
  c2<T> t2 = INV ? mul_pi<T>(o[2]) : mul_mi<T>(o[2]);
  c2<T> t3 = INV ? mk<T>(-c * (o[3].x + o[3].y), c * (o[3].x - o[3].y))
                 : mk<T>(c * (o[3].y - o[3].x), -c * (o[3].x + o[3].y));
  v[0] = cadd<T>(e[0], o[0]);
  v[4] = csub<T>(e[0], o[0]);
  v[1] = cadd<T>(e[1], t1);
  v[5] = csub<T>(e[1], t1);
  v[2] = cadd<T>(e[2], t2);
  v[6] = csub<T>(e[2], t2);
  v[3] = cadd<T>(e[3], t3);
  v[7] = csub<T>(e[3], t3);
}

template <class T, int LOGR, bool INV> __device__ __forceinline__ void dftR(c2<T>* v) {
  if constexpr (LOGR == 1) dft2<T, INV>(v);
  else if constexpr (LOGR == 2) dft4<T, INV>(v);
  else dft8<T, INV>(v);
}

__host__ __device__ constexpr int fft_elems(int logn) { return logn >= 3 ? 8 : (1 << logn); }

// One Stockham stage on all NB transforms of the block.  nthr threads each own
// E/R butterflies.  `tw` is the exp(-2 pi i j / 4096) table.
template <class T, int LOGN, int LOGR, int LOGP, int E, bool INV>
__device__ __forceinline__ void fft_stage(c2<T>* buf, int stride, const c2<T>* __restrict__ tw,
                                          int tid, int nthr) {
  constexpr int R = 1 << LOGR;
  constexpr int NR = 1 << (LOGN - LOGR);
  constexpr int P = 1 << LOGP;
  constexpr int NBF = E / R;  // butterflies per thread
  c2<T> v[NBF][R];
  int base[NBF], ii[NBF];
#pragma unroll
  for (int u = 0; u < NBF; ++u) {
    const int t = tid + u * nthr;
    base[u] = (t >> (LOGN - LOGR)) * stride;
    ii[u] = t & (NR - 1);
#pragma unroll
    for (int q = 0; q < R; ++q) v[u][q] = buf[base[u] + ii[u] + q * NR];
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NBF; ++u) {
    const int i = ii[u];
    const int k = i & (P - 1);
    if constexpr (LOGP > 0) {
#pragma unroll
      for (int q = 1; q < R; ++q) {
        c2<T> w = twiddle_ld(tw, (q * k) << (kLogTw - LOGP - LOGR));
        if (INV) w.y = -w.y;
        v[u][q] = cmul<T>(v[u][q], w);
      }
    }
    dftR<T, LOGR, INV>(v[u]);
    const int j = ((i - k) << LOGR) + k;
#pragma unroll
    for (int q = 0; q < R; ++q) buf[base[u] + j + q * P] = v[u][q];
  }
  __syncthreads();
}

template <class T, int LOGN, int E, bool INV, int S, int LOGP> struct FftStages {
  static __device__ __forceinline__ void run(c2<T>* buf, int stride, const c2<T>* __restrict__ tw,
                                             int tid, int nthr) {
    constexpr int REM = LOGN % 3;
    constexpr int LOGR = (S == 0 && REM != 0) ? REM : 3;
    fft_stage<T, LOGN, LOGR, LOGP, E, INV>(buf, stride, tw, tid, nthr);
    if constexpr (LOGP + LOGR < LOGN)
      FftStages<T, LOGN, E, INV, S + 1, LOGP + LOGR>::run(buf, stride, tw, tid, nthr);
  }
};

// In-place FFT of all transforms of the block; buf must be filled and synchronised.
template <class T, int LOGN, bool INV>
__device__ __forceinline__ void lds_fft(c2<T>* buf, int stride, const c2<T>* __restrict__ tw, int tid,
                                        int nthr) {
  FftStages<T, LOGN, fft_elems(LOGN), INV, 0, 0>::run(buf, stride, tw, tid, nthr);
}

}  // namespace die
