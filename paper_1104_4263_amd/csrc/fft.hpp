// Register-resident Stockham FFT for power-of-two lengths up to 4096 (gfx950).
//
// A block transforms NB arrays of length N = 2^LOGN (times NP arrays held in
// lock step by the same threads, e.g. the two field components).  Each of the
// NT = NB N / E threads owns E values.  A stage of radix R = 2^LR maps each
// butterfly (b, i), i < N / R, to a thread; the butterfly reads x[b][i + q N/R]
// (q < R), multiplies by w^(q k) with k = i mod p (p = product of the radices
// already applied, w = exp(-+2 pi i / (p R))), does an in-register DFT of size
// R and writes y[b][(i - k) R + k + q p].  The output is in natural order for
// any sequence of radices.
//
// The first stage takes its inputs from registers (the caller loads them from
// global memory) and the last stage leaves its outputs in registers, so a
// transform costs only (stages - 1) exchanges through LDS.  Which thread owns
// which butterfly is chosen per stage: "position fast" (consecutive lanes,
// consecutive i of one array) or "array fast" (consecutive lanes, the same i of
// consecutive arrays).  Switching between the two inside the transform turns a
// row-major load into a transposed store (and back) at no extra LDS cost.
// LDS rows are padded by one element per 256 bytes (gfx950 LDS: 64 banks of 4 bytes)
// plus five elements per array, which spreads the stride-R accesses of the early
// stages and the array-fast accesses over the banks.
#pragma once
#include "common.hpp"

namespace die {

// ------------------------------------------------------------------ small DFTs
template <class T, bool INV> __device__ __forceinline__ void dft2(c2<T>* v) {
  const c2<T> a = v[0];
  v[0] = cadd<T>(a, v[1]);
  v[1] = csub<T>(a, v[1]);
}

template <class T, bool INV> __device__ __forceinline__ void dft4(c2<T>* v) {
  const c2<T> a0 = cadd<T>(v[0], v[2]), a1 = csub<T>(v[0], v[2]);
  const c2<T> b0 = cadd<T>(v[1], v[3]);
  c2<T> b1 = csub<T>(v[1], v[3]);
  b1 = INV ? mul_pi<T>(b1) : mul_mi<T>(b1);
  v[0] = cadd<T>(a0, b0);
  v[2] = csub<T>(a0, b0);
  v[1] = cadd<T>(a1, b1);
  v[3] = csub<T>(a1, b1);
}

// exp(-+2 pi i m / 16) for m < 16
template <class T, bool INV> __device__ __forceinline__ c2<T> w16(int m) {
  constexpr double C[16] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0,
                            -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613, -1.0,
                            -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173, 0.0,
                            0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613};
  constexpr double S[16] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128675613, 1.0,
                            0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0,
                            -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128675613, -1.0,
                            -0.92387953251128675613, -0.70710678118654752440, -0.38268343236508977173};
  return mk<T>((T)C[m], INV ? (T)S[m] : (T)-S[m]);
}

// a * exp(-+2 pi i M / 16) with the trivial and the eighth-turn factors written out
// (no multiplications by 0 or 1).
template <class T, bool INV, int M> __device__ __forceinline__ c2<T> mulw16(c2<T> a) {
  constexpr int m = M & 15;
  if constexpr (m == 0) return a;
  else if constexpr (m == 8) return mk<T>(-a.x, -a.y);
  else if constexpr (m == 4) return INV ? mul_pi<T>(a) : mul_mi<T>(a);
  else if constexpr (m == 12) return INV ? mul_mi<T>(a) : mul_pi<T>(a);
  else if constexpr (m % 4 == 2) {
    // exp(-+i pi / 4) a, then the remaining quarter turns
    constexpr T c = (T)0.70710678118654752440;
    const c2<T> e = INV ? mk<T>((a.x - a.y) * c, (a.x + a.y) * c) : mk<T>((a.x + a.y) * c, (a.y - a.x) * c);
    return mulw16<T, INV, m - 2>(e);
  } else {
    return cmul<T>(a, w16<T, INV>(m));
  }
}

template <class T, bool INV> __device__ __forceinline__ void dft8(c2<T>* v) {
  c2<T> e[4] = {v[0], v[2], v[4], v[6]};
  c2<T> o[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, INV>(e);
  dft4<T, INV>(o);
  const c2<T> t[4] = {o[0], mulw16<T, INV, 2>(o[1]), mulw16<T, INV, 4>(o[2]), mulw16<T, INV, 6>(o[3])};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[k] = cadd<T>(e[k], t[k]);
    v[k + 4] = csub<T>(e[k], t[k]);
  }
}

template <class T, bool INV> __device__ __forceinline__ void dft16(c2<T>* v) {
  c2<T> a[4][4];
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) {
    c2<T> t[4] = {v[n2], v[4 + n2], v[8 + n2], v[12 + n2]};
    dft4<T, INV>(t);
    a[n2][0] = t[0];
    if (n2 == 0) {
      a[0][1] = t[1], a[0][2] = t[2], a[0][3] = t[3];
    } else if (n2 == 1) {
      a[1][1] = mulw16<T, INV, 1>(t[1]), a[1][2] = mulw16<T, INV, 2>(t[2]), a[1][3] = mulw16<T, INV, 3>(t[3]);
    } else if (n2 == 2) {
      a[2][1] = mulw16<T, INV, 2>(t[1]), a[2][2] = mulw16<T, INV, 4>(t[2]), a[2][3] = mulw16<T, INV, 6>(t[3]);
    } else {
      a[3][1] = mulw16<T, INV, 3>(t[1]), a[3][2] = mulw16<T, INV, 6>(t[2]), a[3][3] = mulw16<T, INV, 9>(t[3]);
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) {
    c2<T> t[4] = {a[0][k1], a[1][k1], a[2][k1], a[3][k1]};
    dft4<T, INV>(t);
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) v[k1 + 4 * k2] = t[k2];
  }
}

template <class T, int LR, bool INV> __device__ __forceinline__ void dftR(c2<T>* v) {
  if constexpr (LR == 1) dft2<T, INV>(v);
  else if constexpr (LR == 2) dft4<T, INV>(v);
  else if constexpr (LR == 3) dft8<T, INV>(v);
  else dft16<T, INV>(v);
}

// The table entries w, w^2, w^4, w^8 (as far as R needs them) of w = tw[base].
template <class T, int LR>
__device__ __forceinline__ void twiddle_load(c2<T>* p4, const c2<T>* __restrict__ tw, int base) {
  constexpr int R = 1 << LR;
  p4[0] = tw[base];
  if constexpr (R > 2) p4[1] = tw[(2 * base) & (kTw - 1)];
  if constexpr (R > 4) p4[2] = tw[(4 * base) & (kTw - 1)];
  if constexpr (R > 8) p4[3] = tw[(8 * base) & (kTw - 1)];
}

// Multiply v[q] (q = 1 .. R-1) by w^q (^* for INV), forming the powers from w, w^2, w^4, w^8
// (twiddle_load) with at most three products each.
template <class T, int LR, bool INV>
__device__ __forceinline__ void twiddle(c2<T>* v, const c2<T>* p4) {
  constexpr int R = 1 << LR;
  c2<T> p[R];
  p[1] = p4[0];
  if constexpr (R > 2) p[2] = p4[1];
  if constexpr (R > 4) p[4] = p4[2];
  if constexpr (R > 8) p[8] = p4[3];
#pragma unroll
  for (int q = 3; q < R; ++q) {
    if (q == 4 || q == 8) continue;
    const int hi = q >= 8 ? 8 : (q >= 4 ? 4 : 2);
    p[q] = cmul<T>(p[hi], p[q - hi]);
  }
#pragma unroll
  for (int q = 1; q < R; ++q) {
    c2<T> w = p[q];
    if (INV) w.y = -w.y;
    v[q] = cmul<T>(v[q], w);
  }
}

enum : int { kPosFast = 0, kArrFast = 1 };

__host__ __device__ constexpr int fft_pad_shift(int elem_bytes) { return elem_bytes == 8 ? 5 : 4; }
__host__ __device__ constexpr int fft_row_stride(int n, int elem_bytes) {
  return n + (n >> fft_pad_shift(elem_bytes)) + 5;
}

// MAP0: thread mapping of the first stage, MAPR of the stages after it, MAPL of the last stage
// (when there is more than one).
template <class T, int LOGN, int NB, int LOGE, int NP, bool REV, int MAP0, int MAPR, int MAPL = MAPR> struct RegFft {
  static constexpr int N = 1 << LOGN;
  static constexpr int LE = LOGE < LOGN ? LOGE : LOGN;
  static constexpr int E = 1 << LE;
  static constexpr int NT = NB * N / E;
  static constexpr int REM = LOGN % LE;
  static constexpr int NS = LOGN / LE + (REM ? 1 : 0);
  static constexpr int ES = (int)sizeof(c2<T>);
  static constexpr int PS = fft_pad_shift(ES);
  static constexpr int LDB = fft_row_stride(N, ES);
  static constexpr int LDS_ELEMS = NB * LDB;  // one array set at a time (see stage)

  static constexpr int lr(int s) { return (REM && (REV ? s == NS - 1 : s == 0)) ? REM : LE; }
  static constexpr int lp(int s) { return s == 0 ? 0 : lp(s - 1) + lr(s - 1); }
  static constexpr int map(int s) { return s == 0 ? MAP0 : (s == NS - 1 ? MAPL : MAPR); }
  static __host__ __device__ constexpr int f(int j) { return j + (j >> PS); }

  // butterfly (array b, index i) of thread t, slot u, in stage S
  template <int S> static __device__ __forceinline__ void bi(int t, int u, int& b, int& i) {
    constexpr int NR = N >> lr(S);
    const int g = t + u * NT;
    if constexpr (map(S) == kArrFast) {
      b = g % NB;
      i = g / NB;
    } else {
      b = g / NR;
      i = g % NR;
    }
  }
  // element position held in v[u * R + q] before stage 0 (inputs) / after the last stage (outputs)
  static constexpr int R0 = 1 << lr(0);
  static constexpr int RL = 1 << lr(NS - 1);
  static __device__ __forceinline__ void in_pos(int t, int u, int q, int& b, int& pos) {
    int i;
    bi<0>(t, u, b, i);
    pos = i + q * (N / R0);
  }
  static __device__ __forceinline__ void out_pos(int t, int u, int q, int& b, int& pos) {
    int i;
    bi<NS - 1>(t, u, b, i);
    pos = i + q * (N / RL);
  }

  // Twiddle base values of the butterflies a thread owns in stage S (none in stage 0).
  template <int S> struct Tw {
    c2<T> p[(E >> lr(S)) > 0 ? (E >> lr(S)) : 1][4];
  };
  template <int S> static __device__ __forceinline__ void load_tw(Tw<S>& w, const c2<T>* __restrict__ tw, int t) {
    constexpr int LR = lr(S), LP = lp(S), P = 1 << LP, NU = E >> LR;
    if constexpr (LP > 0) {
#pragma unroll
      for (int u = 0; u < NU; ++u) {
        int b, i;
        bi<S>(t, u, b, i);
        twiddle_load<T, LR>(w.p[u], tw, (i & (P - 1)) << (kLogTw - LP - LR));
      }
    }
  }

  // Stage S on registers (its twiddle bases in w), then (except after the last stage) the
  // exchange into the layout of stage S+1 through LDS.  The table loads of stage S+1 are issued
  // before the exchange, whose barriers hide their latency.  The NP arrays held in lock step go
  // through one LDS buffer in turn, so the buffer is NP times smaller than all the data (more
  // blocks per CU).
  template <int S, bool INV>
  static __device__ __forceinline__ void stage(c2<T> (&v)[NP][E], c2<T>* lds, const c2<T>* __restrict__ tw, int t,
                                               const Tw<S>& w) {
    constexpr int LR = lr(S), R = 1 << LR, LP = lp(S), P = 1 << LP, NU = E / R;
#pragma unroll
    for (int u = 0; u < NU; ++u) {
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        if constexpr (LP > 0) twiddle<T, LR, INV>(&v[p][u * R], w.p[u]);
        dftR<T, LR, INV>(&v[p][u * R]);
      }
    }
    if constexpr (S < NS - 1) {
      constexpr int LR1 = lr(S + 1), R1 = 1 << LR1, NR1 = N >> LR1, NU1 = E / R1;
      Tw<S + 1> w1;
      load_tw<S + 1>(w1, tw, t);
#pragma unroll
      for (int p = 0; p < NP; ++p) {
#pragma unroll
        for (int u = 0; u < NU; ++u) {
          int b, i;
          bi<S>(t, u, b, i);
          const int k = i & (P - 1);
          const int j = ((i - k) << LR) + k;
          // f(j + q P) = f(j) + f(q P): j mod 2^PS plus q P mod 2^PS never carries past 2^PS
          // (j = multiple of P R plus k < P), so each element is a constant offset from f(j)
          c2<T>* wr = lds + b * LDB + f(j);
#pragma unroll
          for (int q = 0; q < R; ++q) wr[f(q * P)] = v[p][u * R + q];
        }
        lds_sync();
#pragma unroll
        for (int u = 0; u < NU1; ++u) {
          int b, i;
          bi<S + 1>(t, u, b, i);
          // the same for i + q NR1 (i < NR1, both powers of two)
          const c2<T>* r = lds + b * LDB + f(i);
#pragma unroll
          for (int q = 0; q < R1; ++q) v[p][u * R1 + q] = r[f(q * NR1)];
        }
        lds_sync();
      }
      stage<S + 1, INV>(v, lds, tw, t, w1);
    }
  }

  // v holds the stage-0 inputs; on return it holds the outputs (see out_pos).
  // LDS may be reused by the caller right after the call returns.
  template <bool INV>
  static __device__ __forceinline__ void run(c2<T> (&v)[NP][E], c2<T>* lds, const c2<T>* __restrict__ tw, int t) {
    Tw<0> w0;
    stage<0, INV>(v, lds, tw, t, w0);
  }
};

// Physical block id -> logical block id such that each of the 8 XCDs (which
// receive blocks round robin) processes a contiguous range of logical blocks.
__device__ __forceinline__ int xcd_remap(int b, int total) {
  const int q = total >> 3;
  if (b >= (q << 3)) return b;
  return (b & 7) * q + (b >> 3);
}

}  // namespace die
