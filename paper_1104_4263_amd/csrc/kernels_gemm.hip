// Block Gram-Schmidt of block GMRES on the matrix cores, and the small dense steps around it.
//
// A complex block X (n x p) is held planar: 2p real columns, the p real parts, then the p
// imaginary parts; a basis of nq complex columns in p-column blocks is 2 nq real columns (block
// j at columns 2 p j .. 2 p (j + 1)).  In that form the block projection Q^H W and the update
// W -= Q H are real matrix products: the projection's four real blocks combine into the complex
// H, and the update multiplies by the real matrix Hb that represents H (see k_tsq_combine).
//
// The products are tall and skinny: the reduction of the projection and the rows of the update
// run over the vector length n (10^5 .. 10^7), the other dimensions over at most a few thousand
// basis columns and 2p <= 128 columns of W.  They are HBM-bound at these shapes, so the operands
// are laid out for the MFMA instructions: each lane's share of one MFMA operand is one 16-byte
// load, and the 64 lanes of a wave read one contiguous kilobyte.
//
// Element types E and their MFMA: binary16 v_mfma_f32_32x32x16_f16, FP32 v_mfma_f32_32x32x2_f32,
// FP64 v_mfma_f64_16x16x4_f64 (GemmTile in ops.hpp: R rows per tile, KV values per lane load,
// KS reduction values per tile).  Layouts (nrow, ccap multiples of 32):
//   T1 (reduction over rows, the projection's operands): element (n, c) at
//     ((c / R) (nrow / KS) + n / KS) 64 KV + ((c % R) + R ((n % KS) / KV)) KV + n % KV;
//   T2 (reduction over columns, the update's basis operand): element (n, c) at
//     ((n / R) (ccap / KS) + c / KS) 64 KV + ((n % R) + R ((c % KS) / KV)) KV + c % KV.
// MFMA lane layouts: for the 32-row shapes lane l supplies row (l % 32) of A and column (l % 32)
// of B for the reduction indices KV (l / 32) .. + KV - 1 of each KS (in the FP32 shape one
// index per instruction, the KV values of a load feeding KV instructions), and accumulator
// element r holds D[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]; for the FP64 16 x 16 x 4 shape
// lane l supplies row / column l % 16 for index l / 16 and holds D[4 r + l / 16][l % 16].
// Every reduction is in a fixed order: results do not depend on timing.
#include "ops.hpp"

namespace die {
namespace {

typedef _Float16 h8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));
typedef float f16v __attribute__((ext_vector_type(16)));
typedef double d4v __attribute__((ext_vector_type(4)));

template <class E> struct Mf;
template <> struct Mf<_Float16> {
  using V = h8v;
  using C = f16v;
  static constexpr int NC = 16;
  static __device__ __forceinline__ C mma(V a, V b, C c) { return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  static __device__ __forceinline__ int col(int l) { return l & 31; }
};
template <> struct Mf<float> {
  using V = f4v;
  using C = f16v;
  static constexpr int NC = 16;
  static __device__ __forceinline__ C mma(V a, V b, C c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[0], b[0], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[1], b[1], c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(a[2], b[2], c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a[3], b[3], c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 8 * (r >> 2) + 4 * (l >> 5) + (r & 3); }
  static __device__ __forceinline__ int col(int l) { return l & 31; }
};
template <> struct Mf<double> {
  using V = d2v;
  using C = d4v;
  static constexpr int NC = 4;
  static __device__ __forceinline__ C mma(V a, V b, C c) {
    c = __builtin_amdgcn_mfma_f64_16x16x4f64(a[0], b[0], c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a[1], b[1], c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row(int l, int r) { return 4 * r + (l >> 4); }
  static __device__ __forceinline__ int col(int l) { return l & 15; }
};

template <class E> __device__ __forceinline__ typename Mf<E>::V ld16(const E* p) {
  return *reinterpret_cast<const typename Mf<E>::V*>(p);
}

// The one-value-per-lane MFMA shapes (the complex right-multiplication): FP32 32 x 32 x 2 and
// FP64 16 x 16 x 4, lane l supplying index l / R of the reduction.
template <class T> struct Mf1;
template <> struct Mf1<float> {
  using C = f16v;
  static constexpr int R = 32, NC = 16;
  static __device__ __forceinline__ C mma(float a, float b, C c) { return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int l, int r) { return Mf<float>::row(l, r); }
  static __device__ __forceinline__ int col(int l) { return l & 31; }
};
template <> struct Mf1<double> {
  using C = d4v;
  static constexpr int R = 16, NC = 4;
  static __device__ __forceinline__ C mma(double a, double b, C c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  static __device__ __forceinline__ int row(int l, int r) { return Mf<double>::row(l, r); }
  static __device__ __forceinline__ int col(int l) { return l & 15; }
};

// ---- layout conversions

// The planar copy Ws (accumulation type A, leading dimension ldw, rows n .. nrow - 1 zero) of the
// complex block X (n x p): one thread per row and column, the two parts to columns q and p + q.
template <class T, class A>
__global__ void k_split_planar(const c2<T>* __restrict__ X, size_t ldx, size_t n, int p, size_t nrow,
                               A* __restrict__ Ws, size_t ldw, const int* __restrict__ gate) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gate && !*gate) || e >= nrow * (size_t)p) return;
  const size_t q = e / nrow, r = e - q * nrow;
  c2<T> z = mk<T>((T)0, (T)0);
  if (r < n) z = X[q * ldx + r];
  Ws[q * ldw + r] = (A)z.x;
  Ws[(p + q) * ldw + r] = (A)z.y;
}

// Columns [c0, c0 + 2p) of the T1 copy A1 (nrow rows, rows past n zero) of the planar X: one
// thread per planar column and group of KV rows, consecutive threads on consecutive columns (so
// that the 16-byte writes of a tile are contiguous).
template <class T, class E>
__global__ void k_split_t1(const c2<T>* __restrict__ X, size_t ldx, size_t n, int p, int c0, size_t nrow,
                           E* __restrict__ A1) {
  using V = typename Mf<E>::V;
  constexpr int KV = GemmTile<E>::KV;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrow / KV * 2 * (size_t)p) return;
  const int c = (int)(e % (2 * (size_t)p));
  const size_t n0 = e / (2 * (size_t)p) * KV;
  const bool im = c >= p;
  const c2<T>* xc = X + (size_t)(im ? c - p : c) * ldx;
  V v{};
#pragma unroll
  for (int i = 0; i < KV; ++i)
    if (n0 + i < n) {
      const c2<T> z = xc[n0 + i];
      v[i] = (E)(im ? z.y : z.x);
    }
  *reinterpret_cast<V*>(A1 + GemmTile<E>::t1(n0, (size_t)(c0 + c), nrow)) = v;
}

// Columns [c0, c0 + 2p) of the T2 copy A2 (capacity ccap) of the planar X: one thread per row
// and group of KV columns (consecutive threads take consecutive rows, so the reads of X and the
// 16-byte writes of A2 are contiguous); only the block's own columns are written.
template <class T, class E>
__global__ void k_split_t2(const c2<T>* __restrict__ X, size_t ldx, size_t n, int p, int c0, size_t nrow, size_t ccap,
                           E* __restrict__ A2) {
  using V = typename Mf<E>::V;
  constexpr int KV = GemmTile<E>::KV;
  const int g0 = c0 / KV, g1 = (c0 + 2 * p + KV - 1) / KV;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nrow * (size_t)(g1 - g0)) return;
  const int g = g0 + (int)(e / nrow);
  const size_t r = e % nrow;
  V v{};
  bool full = true;
#pragma unroll
  for (int i = 0; i < KV; ++i) {
    const int c = g * KV + i - c0;
    if (c < 0 || c >= 2 * p) {
      full = false;
      continue;
    }
    if (r < n) {
      const c2<T> z = X[(size_t)(c < p ? c : c - p) * ldx + r];
      v[i] = (E)(c < p ? z.x : z.y);
    }
  }
  E* d = A2 + GemmTile<E>::t2(r, (size_t)g * KV, ccap);
  if (full) {
    *reinterpret_cast<V*>(d) = v;
  } else {
#pragma unroll
    for (int i = 0; i < KV; ++i) {
      const int c = g * KV + i - c0;
      if (c >= 0 && c < 2 * p) d[i] = v[i];
    }
  }
}

// Both shadows at once (KV x KV planar sub-squares, p % KV == 0 and c0 % KV == 0): one thread per
// group of KV rows and KV complex columns reads their KV x KV values once (KV consecutive rows of
// each column, consecutive threads on consecutive row groups) and writes the 2 KV vectors of their
// real and imaginary columns into A1 (KV rows each) and the 2 KV vectors of their rows into A2
// (KV columns each).
template <class T, class E>
__global__ void __launch_bounds__(256) k_split_t12(const c2<T>* __restrict__ X, size_t ldx, size_t n, int p, int c0, size_t nrow,
                            size_t ccap, E* __restrict__ A1, E* __restrict__ A2) {
  using V = typename Mf<E>::V;
  constexpr int KV = GemmTile<E>::KV;
  const size_t groups = nrow / KV;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= groups * (size_t)(p / KV)) return;
  const int cg = (int)(e / groups);
  const size_t n0 = (e - (size_t)cg * groups) * KV;
  V re[KV], im[KV];  // re[i][r]: column cg KV + i, row n0 + r
#pragma unroll
  for (int i = 0; i < KV; ++i) {
    const c2<T>* xc = X + (size_t)(cg * KV + i) * ldx + n0;
#pragma unroll
    for (int r = 0; r < KV; ++r) {
      const c2<T> z = n0 + r < n ? xc[r] : mk<T>((T)0, (T)0);
      re[i][r] = (E)z.x;
      im[i][r] = (E)z.y;
    }
  }
#pragma unroll
  for (int i = 0; i < KV; ++i) {
    *reinterpret_cast<V*>(A1 + GemmTile<E>::t1(n0, (size_t)(c0 + cg * KV + i), nrow)) = re[i];
    *reinterpret_cast<V*>(A1 + GemmTile<E>::t1(n0, (size_t)(c0 + p + cg * KV + i), nrow)) = im[i];
  }
#pragma unroll
  for (int r = 0; r < KV; ++r) {
    V vr, vi;
#pragma unroll
    for (int i = 0; i < KV; ++i) {
      vr[i] = re[i][r];
      vi[i] = im[i][r];
    }
    *reinterpret_cast<V*>(A2 + GemmTile<E>::t2(n0 + r, (size_t)(c0 + cg * KV), ccap)) = vr;
    *reinterpret_cast<V*>(A2 + GemmTile<E>::t2(n0 + r, (size_t)(c0 + p + cg * KV), ccap)) = vi;
  }
}

// T1 copy (columns 0 .. nb - 1) of the planar block Ws (nrow rows, leading dimension ldw).
template <class A, class E>
__global__ void k_planar_to_t1(const A* __restrict__ Ws, size_t ldw, size_t nrow, int nb, E* __restrict__ B1) {
  constexpr int KV = GemmTile<E>::KV;
  const size_t chunks = nrow / KV;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= chunks * (size_t)nb) return;
  const int c = (int)(e / chunks);
  const size_t n0 = (e - (size_t)c * chunks) * KV;
  E* d = B1 + GemmTile<E>::t1(n0, (size_t)c, nrow);
  const A* s = Ws + (size_t)c * ldw + n0;
#pragma unroll
  for (int i = 0; i < KV; ++i) d[i] = (E)s[i];
}

// ---- projection: part[h][b ma + a] = sum over the rows n of chunk h of A(n, a) B(n, b)
// for a < ma, b < nb.  A and B in T1 with nrow rows, or (NF) planar with the rows contiguous
// (leading dimension nrow, rows past the data zero; a buffer of whole 32-column tiles).
// Block (h, y): four waves, one column tile of A each (tile 4 y + wave), every column tile of B
// (NT of them).  B is staged through LDS GK k-steps at a time and shared by the four waves;
// the next group's tiles of A (per wave) and of B (per block) are in flight while a group is
// multiplied, double-buffered.  The blocks of one chunk share its rows of B, so they are
// placed on one XCD (blocks go to the 8 XCDs in turn) one after another; the grid is 1-D with
// nch a multiple of 8.
template <class E> constexpr int proj_group() { return sizeof(E) == 8 ? 4 : 8; }
template <class E, int NT, bool NF>
__global__ void __launch_bounds__(256)
k_tsq_proj(const E* __restrict__ A1, int ma, const E* __restrict__ B1, int nb, size_t nrow, int kc, int gy,
           typename GemmTile<E>::Acc* __restrict__ part, const int* __restrict__ gate) {
  if (gate && !*gate) return;  // the whole block: before any barrier
  using M = Mf<E>;
  using Tl = GemmTile<E>;
  using V = typename M::V;
  constexpr int R = Tl::R, KV = Tl::KV, KS = Tl::KS, TILE = 64 * KV, GK = proj_group<E>();
  constexpr int BV = GK * NT * 64, BPT = BV / 256;  // vectors of B per group, per thread
  static_assert(BV % 256 == 0, "B staging");
  __shared__ __attribute__((aligned(16))) E bsh[2][GK * NT * TILE];
  const int lane = threadIdx.x & 63;
  const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
  const int h = (slot / gy) * 8 + xcd, y = slot % gy;
  const int mt = (ma + R - 1) / R;
  const int ta = y * 4 + (threadIdx.x >> 6);
  const int tac = ta < mt ? ta : mt - 1;  // a wave past the last tile re-reads it (not stored)
  const size_t tpc = nrow / KS;            // tiles per column strip
  const size_t s0 = (size_t)h * kc < tpc ? (size_t)h * kc : tpc;  // chunks past the rows are empty
  const size_t s1 = s0 + kc < tpc ? s0 + kc : tpc;
  const int ns = (int)(s1 - s0), ng = (ns + GK - 1) / GK;
  // operand of column tile t at k-step s for lane l: base + t * tstride + s * sstride + loff(l)
  const size_t tstride = NF ? (size_t)R * nrow : tpc * TILE;
  const size_t sstride = NF ? KS : TILE;
  auto loff = [&](int l) { return NF ? (size_t)(l % R) * nrow + (l / R) * KV : (size_t)l * KV; };
  const E* pa = A1 + (size_t)tac * tstride + loff(lane);
  // k-step of group g, item f, clamped into the chunk (steps past it are loaded but not used)
  auto kstep = [&](int g, int f) {
    const int s = g * GK + f;
    return s0 + (size_t)(s < ns ? s : (ns > 0 ? ns - 1 : 0));
  };
  typename M::C acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = typename M::C{};
  V a[GK], an[GK], bst[BPT];
  if (ng > 0) {
#pragma unroll
    for (int i = 0; i < BPT; ++i) {  // B vector v = thread + 256 i: item f, tile t, lane l
      const int v = threadIdx.x + 256 * i, f = v / (NT * 64), t = (v / 64) % NT, l = v % 64;
      bst[i] = ld16(B1 + (size_t)t * tstride + kstep(0, f) * sstride + loff(l));
    }
#pragma unroll
    for (int f = 0; f < GK; ++f) a[f] = ld16(pa + kstep(0, f) * sstride);
#pragma unroll
    for (int i = 0; i < BPT; ++i) *reinterpret_cast<V*>(&bsh[0][(threadIdx.x + 256 * i) * KV]) = bst[i];
  }
  lds_sync();
  for (int g = 0; g < ng; ++g) {
    const int cur = g & 1;
    const bool more = g + 1 < ng;
    if (more) {  // the next group: B first, so that waiting for it leaves A in flight
#pragma unroll
      for (int i = 0; i < BPT; ++i) {
        const int v = threadIdx.x + 256 * i, f = v / (NT * 64), t = (v / 64) % NT, l = v % 64;
        bst[i] = ld16(B1 + (size_t)t * tstride + kstep(g + 1, f) * sstride + loff(l));
      }
#pragma unroll
      for (int f = 0; f < GK; ++f) an[f] = ld16(pa + kstep(g + 1, f) * sstride);
    }
    const int nf = ns - g * GK < GK ? ns - g * GK : GK;
    const E* bs = &bsh[cur][lane * KV];
    if (nf == GK) {
#pragma unroll
      for (int f = 0; f < GK; ++f)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[t] = M::mma(a[f], *reinterpret_cast<const V*>(bs + (f * NT + t) * TILE), acc[t]);
    } else {
#pragma unroll
      for (int f = 0; f < GK; ++f)
        if (f < nf)
#pragma unroll
          for (int t = 0; t < NT; ++t)
            acc[t] = M::mma(a[f], *reinterpret_cast<const V*>(bs + (f * NT + t) * TILE), acc[t]);
    }
    if (more) {
#pragma unroll
      for (int i = 0; i < BPT; ++i) *reinterpret_cast<V*>(&bsh[cur ^ 1][(threadIdx.x + 256 * i) * KV]) = bst[i];
#pragma unroll
      for (int f = 0; f < GK; ++f) a[f] = an[f];
    }
    lds_sync();
  }
  if (ta >= mt) return;
  typename Tl::Acc* out = part + (size_t)h * ma * nb;
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    const int b = t * R + M::col(lane);
    if (b >= nb) continue;
#pragma unroll
    for (int r = 0; r < M::NC; ++r) {
      const int a = ta * R + M::row(lane, r);
      if (a < ma) out[(size_t)b * ma + a] = acc[t][r];
    }
  }
}

// One thread per entry (q, k) of the complex projection H = Q^H W (nq x p, leading dimension
// nq): the chunk products C_h (2nq x 2p, leading dimension 2nq) summed in chunk order in FP64,
//   Re H = Qr^T Wr + Qi^T Wi,  Im H = Qr^T Wi - Qi^T Wr,
// rounded to E, and written twice: H (type T, the E-rounded values) and the real update matrix
// Hb (E, 2nq x 2p, leading dimension ldhb) with which Ws -= Qs Hb is W -= Q H:
//   Hb[re row, k] = Re H, Hb[re row, p + k] = Im H, Hb[im row, k] = -Im H, Hb[im row, p + k] = Re H.
// Row q = j p + c of Q (block j, column c) is real row 2 p j + c and imaginary row 2 p j + p + c.
template <class P, class E, class T>
__global__ void k_tsq_combine(const P* __restrict__ C, int nch, int nq, int p, c2<T>* __restrict__ H,
                              E* __restrict__ Hb, int ldhb) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nq * p) return;
  const int k = e / nq, q = e - k * nq;
  const int j = q / p, cc = q - j * p;
  const int M = 2 * nq, rre = 2 * p * j + cc, rim = rre + p;
  const size_t cs = (size_t)M * 2 * p;
  double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
  for (int h = 0; h < nch; ++h) {
    const P* Ch = C + (size_t)h * cs;
    rr += (double)Ch[(size_t)k * M + rre];
    ii += (double)Ch[(size_t)(p + k) * M + rim];
    ri += (double)Ch[(size_t)(p + k) * M + rre];
    ir += (double)Ch[(size_t)k * M + rim];
  }
  const E hr = (E)(rr + ii), hi = (E)(ri - ir);
  H[(size_t)k * nq + q] = mk<T>((T)hr, (T)hi);
  Hb[(size_t)k * ldhb + rre] = hr;
  Hb[(size_t)(p + k) * ldhb + rre] = hi;
  Hb[(size_t)k * ldhb + rim] = -hi;
  Hb[(size_t)(p + k) * ldhb + rim] = hr;
}

// The Gram matrix G = X^H X (p x p, FP64, leading dimension p) from the chunk products of the
// planar X (2p x 2p each, leading dimension 2p), summed in chunk order.
template <class P>
__global__ void k_gram_combine(const P* __restrict__ C, int nch, int p, double2* __restrict__ G,
                               const int* __restrict__ gate) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if ((gate && !*gate) || e >= p * p) return;
  const int b = e / p, a = e - b * p, P2 = 2 * p;
  double rr = 0.0, ii = 0.0, ri = 0.0, ir = 0.0;
  for (int h = 0; h < nch; ++h) {
    const P* Ch = C + (size_t)h * P2 * P2;
    rr += (double)Ch[(size_t)b * P2 + a];
    ii += (double)Ch[(size_t)(p + b) * P2 + p + a];
    ri += (double)Ch[(size_t)(p + b) * P2 + a];
    ir += (double)Ch[(size_t)b * P2 + p + a];
  }
  G[e] = make_double2(rr + ii, ri - ir);
}

// First stage of the sum over many chunk products: out[g][e] = the FP64 sum of the products of
// chunks g cpg .. (g + 1) cpg - 1, in chunk order, for the L entries e of one product.
template <class A>
__global__ void k_chunk_sum(const A* __restrict__ part, int nch, size_t L, int cpg, double* __restrict__ out,
                            const int* __restrict__ gate) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if ((gate && !*gate) || e >= L) return;
  const int h0 = blockIdx.y * cpg, h1 = h0 + cpg < nch ? h0 + cpg : nch;
  double acc = 0.0;
#pragma unroll 8
  for (int h = h0; h < h1; ++h) acc += (double)part[(size_t)h * L + e];
  out[(size_t)blockIdx.y * L + e] = acc;
}

// ---- update: Ws(n, b) -= sum_{c < mc} Q(n, c) Hb(c, b) for b < nb, all nrow rows of Ws
// (leading dimension ldw); Q in T2 with column capacity ccap, Hb column-major with leading
// dimension ldhb (a multiple of KV, at least mc).  Computed transposed, D[b][n] = sum_c
// Hb^T[b][c] Q^T[c][n], so that a wave's results are R consecutive rows of Ws per column.
// WAVES waves a block, one tile of R rows of Ws each; Hb is staged through LDS 256 bytes of c
// per column at a time (zero past mc and nb), double-buffered: the next chunk of Hb (per
// block) and of Q (per wave) are in flight while a chunk is multiplied.
template <class E, int NT, int WAVES>
__global__ void __launch_bounds__(64 * WAVES)
k_tsq_update(const E* __restrict__ A2, int mc, size_t ccap, size_t nrow, const E* __restrict__ Hb, int ldhb, int nb,
             typename GemmTile<E>::Acc* __restrict__ Ws, size_t ldw) {
  using M = Mf<E>;
  using Tl = GemmTile<E>;
  using V = typename M::V;
  constexpr int R = Tl::R, KV = Tl::KV, KS = Tl::KS, TILE = 64 * KV;
  constexpr int CK = 256 / (int)sizeof(E), CKP = CK + 16 / (int)sizeof(E), VPR = CK / KV, NS = CK / KS;
  constexpr int NV = NT * R * VPR, PER = (NV + 64 * WAVES - 1) / (64 * WAVES);  // staged vectors (per thread)
  __shared__ __attribute__((aligned(16))) E sh[2][NT * R * CKP];
  const int lane = threadIdx.x & 63;
  const size_t stripe = (size_t)blockIdx.x * WAVES + (threadIdx.x >> 6);
  const bool live = stripe * R < nrow;
  const size_t tpr = ccap / KS;  // tiles per row strip
  const E* pq = A2 + (live ? stripe : 0) * tpr * TILE + lane * KV;  // a wave past the rows reads the first strip
  const int nsteps = (mc + KS - 1) / KS;   // k-steps that hold columns < mc
  const int nchunk = (nsteps + NS - 1) / NS;
  typename M::C acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = typename M::C{};
  // chunk k's staged vector i of this thread (columns c0 + cc .. + KV of row b of Hb)
  auto stage_load = [&](int k, int i, int& b, int& cc) -> V {
    const int v = threadIdx.x + i * 64 * WAVES, vc = v < NV ? v : NV - 1;
    b = vc / VPR;
    cc = k * CK + (vc - b * VPR) * KV;
    const int ccl = cc + KV <= ldhb ? cc : ldhb - KV;  // stays in the row (masked below)
    return ld16(Hb + (size_t)(b < nb ? b : nb - 1) * ldhb + ccl);
  };
  auto stage_store = [&](int k, int buf, const V* x) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int v = threadIdx.x + i * 64 * WAVES;
      if (v >= NV) continue;
      const int b = v / VPR, col = (v - b * VPR) * KV, cc = k * CK + col;
      V y = x[i];
      if (b >= nb) y = V{};
      if (cc + KV > mc) {
#pragma unroll
        for (int e = 0; e < KV; ++e)
          if (cc + e >= mc) y[e] = (E)0;
      }
      *reinterpret_cast<V*>(sh[buf] + b * CKP + col) = y;
    }
  };
  auto q_load = [&](int k, V* q) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      const int st = k * NS + s;
      q[s] = ld16(pq + (size_t)(st < nsteps ? st : nsteps - 1) * TILE);
    }
  };
  V q[NS], qn[NS], x[PER];
  {
    int b, cc;
#pragma unroll
    for (int i = 0; i < PER; ++i) x[i] = stage_load(0, i, b, cc);
    q_load(0, q);
    stage_store(0, 0, x);
  }
  lds_sync();
  const E* pa = &sh[0][0] + (lane % R) * CKP + (lane / R) * KV;
  for (int k = 0; k < nchunk; ++k) {
    const int cur = k & 1;
    const bool more = k + 1 < nchunk;
    if (more) {  // the next chunk: Hb first, so that waiting for it leaves Q in flight
      int b, cc;
#pragma unroll
      for (int i = 0; i < PER; ++i) x[i] = stage_load(k + 1, i, b, cc);
      q_load(k + 1, qn);
    }
    const E* pak = pa + cur * (NT * R * CKP);
    if ((k + 1) * CK <= mc) {  // every column of the chunk is < mc
#pragma unroll
      for (int s = 0; s < NS; ++s)
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[t] = M::mma(*reinterpret_cast<const V*>(pak + t * R * CKP + s * KS), q[s], acc[t]);
    } else {  // the last chunk: columns >= mc masked
#pragma unroll
      for (int s = 0; s < NS; ++s) {
        const int cb = k * CK + s * KS + (lane / R) * KV;
        if (k * CK + s * KS >= mc) break;
        V qs = q[s];
#pragma unroll
        for (int e = 0; e < KV; ++e)
          if (cb + e >= mc) qs[e] = (E)0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
          acc[t] = M::mma(*reinterpret_cast<const V*>(pak + t * R * CKP + s * KS), qs, acc[t]);
      }
    }
    if (more) {
      stage_store(k + 1, cur ^ 1, x);
#pragma unroll
      for (int s = 0; s < NS; ++s) q[s] = qn[s];
    }
    lds_sync();
  }
  if (!live) return;
  const size_t nn = stripe * R + M::col(lane);
  typename Tl::Acc old[NT][M::NC];
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < M::NC; ++r) {
      const int b = t * R + M::row(lane, r);
      old[t][r] = Ws[(size_t)(b < nb ? b : nb - 1) * ldw + nn];
    }
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < M::NC; ++r) {
      const int b = t * R + M::row(lane, r);
      if (b < nb) Ws[(size_t)b * ldw + nn] = old[t][r] - acc[t][r];
    }
}

// ---- Y (n x q) = X (n x s) S (s x q), complex, on the matrix cores in T: per tile of R rows
// of Y, D^T = S^T X^T as four real products (Re Y = Sr Xr - Si Xi, Im Y = Si Xr + Sr Xi,
// transposed).  S is staged through LDS 64 rows at a time as real and imaginary planes [c][j]
// (zero past s and q); each lane reads one complex value of X per MFMA step (the loop is
// unrolled four steps deep, so that their loads are in flight together).  X and Y are distinct.
// PLANAR: X is held planar in T (column c's real parts at c ldx, its imaginary parts at (s + c) ldx).
template <class T, int NT, bool PLANAR = false>
__global__ void __launch_bounds__(256)
k_cplx_rmul(const void* __restrict__ Xv, size_t ldx, int s, const c2<T>* __restrict__ S, int lds, int q, size_t n,
            c2<T>* __restrict__ Y, size_t ldy, const int* __restrict__ ctl, c2<T>* __restrict__ Yalt) {
  if (ctl) {  // device control: ctl[0] == 0 skips the launch, ctl[1] == 0 writes Yalt instead of Y
    if (!ctl[0]) return;
    if (!ctl[1]) Y = Yalt;
  }
  using M = Mf1<T>;
  constexpr int R = M::R, G = 64 / R, SC = 64, QP = NT * R + 1;
  __shared__ T sr[SC * QP], si[SC * QP];
  const int lane = threadIdx.x & 63;
  const size_t stripe = (size_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const size_t row = stripe * R + (lane % R);
  const bool rok = row < n;
  const size_t rowc = rok ? row : n - 1;  // rows past n read row n - 1 (not stored)
  const int kg = lane / R;  // the lane's reduction index within an MFMA step
  typename M::C accr[NT], acci[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) {
    accr[t] = typename M::C{};
    acci[t] = typename M::C{};
  }
  for (int c0 = 0; c0 < s; c0 += SC) {
    const int cn = s - c0 < SC ? s - c0 : SC;
    lds_sync();  // the previous chunk's LDS reads are done
    {
      constexpr int PER = SC * NT * R / 256;  // staged values per thread
      c2<T> v[PER];
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256, i = e / (NT * R), j = e - i * (NT * R);
        v[k] = S[(size_t)(j < q ? j : q - 1) * lds + c0 + (i < cn ? i : cn - 1)];
      }
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int e = threadIdx.x + k * 256, i = e / (NT * R), j = e - i * (NT * R);
        const bool in = i < cn && j < q;
        sr[i * QP + j] = in ? v[k].x : (T)0;
        si[i * QP + j] = in ? v[k].y : (T)0;
      }
    }
    lds_sync();
    // partly unrolled: fully unrolled, the compiler hoisted every LDS read of the chunk's S into
    // registers (one wave per SIMD)
    // groups of four MFMA steps without early exit (steps past cn multiply zero rows of S by a
    // clamped, finite X): the four loads of a group are in flight together
    const int nu = (cn + G - 1) / G;
    for (int u0 = 0; u0 < nu; u0 += 4) {
      c2<T> xv[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int ci = (u0 + k) * G + kg, c = c0 + ci;
        const size_t cc = (size_t)(c < s ? c : s - 1);
        if constexpr (PLANAR) {
          const T* Xs = static_cast<const T*>(Xv);
          xv[k] = mk<T>(Xs[cc * ldx + rowc], Xs[(s + cc) * ldx + rowc]);
        } else {
          xv[k] = static_cast<const c2<T>*>(Xv)[cc * ldx + rowc];
        }
      }
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int ci = (u0 + k) * G + kg;
        const int cs = ci < SC ? ci : SC - 1;  // rows of the staged chunk past cn are zero
        const T xr = xv[k].x, xi = xv[k].y;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const T ar = sr[cs * QP + t * R + (lane % R)], ai = si[cs * QP + t * R + (lane % R)];
          accr[t] = M::mma(ar, xr, accr[t]);
          acci[t] = M::mma(ai, xr, acci[t]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          const T ar = sr[cs * QP + t * R + (lane % R)], ai = si[cs * QP + t * R + (lane % R)];
          accr[t] = M::mma(ai, -xi, accr[t]);
          acci[t] = M::mma(ar, xi, acci[t]);
        }
      }
    }
  }
  const size_t nn = stripe * R + M::col(lane);
  if (nn >= n) return;
#pragma unroll
  for (int t = 0; t < NT; ++t)
#pragma unroll
    for (int r = 0; r < M::NC; ++r) {
      const int j = t * R + M::row(lane, r);
      if (j < q) Y[(size_t)j * ldy + nn] = mk<T>(accr[t][r], acci[t][r]);
    }
}

// ---- R Y = B for the upper triangular R (nc x nc, leading dimension ldr), in place in B
// (nc x k, leading dimension ldb): one block of 1024 threads per KC columns of B, the columns
// in LDS.  Blocks of 64 rows from the bottom: the block's 64 x 64 triangle is staged in LDS
// with the reciprocals of its diagonal, wave c solves it for column c (lane t holds row t, the
// solved value moves by a lane broadcast), then every thread subtracts the block's contribution
// from its rows above it for all KC columns (one read of R serves KC columns).  Three barriers
// per block of rows.
template <int KC>
__global__ void __launch_bounds__(1024)
k_trsm_upper(const double2* __restrict__ R, int ldr, int nc, double2* __restrict__ B, int ldb, int k) {
  extern __shared__ double2 bsh[];  // [KC][nc]
  __shared__ double2 ysh[KC][64];
  __shared__ double2 dsh[64][65];  // the diagonal block, [column][row]
  __shared__ double2 rinv[64];     // 1 / its diagonal
  const int c0 = blockIdx.x * KC, kc = k - c0 < KC ? k - c0 : KC;
  for (int e = threadIdx.x; e < kc * nc; e += 1024) {
    const int j = e / nc, i = e - j * nc;
    bsh[j * nc + i] = B[(size_t)(c0 + j) * ldb + i];
  }
  const int wave = threadIdx.x >> 6, t = threadIdx.x & 63;
  for (int ie = nc; ie > 0; ie -= 64) {
    const int ib = ie > 64 ? ie - 64 : 0, nb = ie - ib;
    lds_sync();  // the previous block's updates (and the initial loads) are done
    for (int e = threadIdx.x; e < nb * nb; e += 1024) {
      const int jc = e / nb, ir = e - jc * nb;
      const double2 v = R[(size_t)(ib + jc) * ldr + ib + ir];
      dsh[jc][ir] = v;
      if (jc == ir) {
        const double dd = v.x * v.x + v.y * v.y;
        rinv[ir] = make_double2(v.x / dd, -v.y / dd);
      }
    }
    lds_sync();
    if (wave < kc) {
      double2 bt = t < nb ? bsh[wave * nc + ib + t] : make_double2(0.0, 0.0);
      double2 yt = make_double2(0.0, 0.0);
      for (int i = nb - 1; i >= 0; --i) {
        // lane i holds the final right-hand side of row ib + i
        const double br = __shfl(bt.x, i), bi = __shfl(bt.y, i);
        const double2 d = rinv[i];
        const double yr = br * d.x - bi * d.y, yi = br * d.y + bi * d.x;
        if (t == i) yt = make_double2(yr, yi);
        if (t < i) {
          const double2 rt = dsh[i][t];
          bt.x -= rt.x * yr - rt.y * yi;
          bt.y -= rt.x * yi + rt.y * yr;
        }
      }
      if (t < nb) {
        ysh[wave][t] = yt;
        B[(size_t)(c0 + wave) * ldb + ib + t] = yt;
      }
    }
    lds_sync();
    for (int row = threadIdx.x; row < ib; row += 1024) {
      double2 a[KC];
#pragma unroll
      for (int j = 0; j < KC; ++j) a[j] = j < kc ? bsh[j * nc + row] : make_double2(0.0, 0.0);
#pragma unroll 16
      for (int i = 0; i < nb; ++i) {
        const double2 rt = R[(size_t)(ib + i) * ldr + row];
#pragma unroll
        for (int j = 0; j < KC; ++j) {
          const double2 y = ysh[j][i];
          a[j].x -= rt.x * y.x - rt.y * y.y;
          a[j].y -= rt.x * y.y + rt.y * y.x;
        }
      }
#pragma unroll
      for (int j = 0; j < KC; ++j)
        if (j < kc) bsh[j * nc + row] = a[j];
    }
  }
}

// C = A + B for small matrices (rows x cols, leading dimensions lda, ldb, ldc).
template <class T>
__global__ void k_cadd2(const c2<T>* __restrict__ A, int lda, const c2<T>* __restrict__ B, int ldb, int rows, int cols,
                        c2<T>* __restrict__ C, int ldc) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * cols) return;
  const int j = e / rows, i = e - j * rows;
  C[(size_t)j * ldc + i] = cadd<T>(A[(size_t)j * lda + i], B[(size_t)j * ldb + i]);
}

inline unsigned blocks_for(size_t work, unsigned per = 256) { return (unsigned)((work + per - 1) / per); }

}  // namespace

template <class T, class A, class E>
hipError_t launch_tsq_split(const c2<T>* X, size_t ldx, size_t n, int p, int c0, size_t nrow, size_t ccap, A* Ws,
                            size_t ldw, E* A1, E* A2, hipStream_t st, const int* gate) {
  if (p < 1 || n > nrow || nrow % 32 || ccap % 32 || (Ws && ldw < nrow) || (A2 && (size_t)c0 + 2 * p > ccap) ||
      (Ws && A1 && c0 != 0) || (gate && (!Ws || A1 || A2)))  // a gate only for the planar copy alone
    return hipErrorInvalidValue;
  constexpr int KV = GemmTile<E>::KV;
  if (!Ws && A1 && A2 && p % KV == 0 && c0 % KV == 0) {  // both shadows from one read of X
    hipLaunchKernelGGL((k_split_t12<T, E>), dim3(blocks_for(nrow / KV * (size_t)(p / KV))), dim3(256), 0, st, X, ldx,
                       n, p, c0, nrow, ccap, A1, A2);
    return hipGetLastError();
  }
  if (Ws)
    hipLaunchKernelGGL((k_split_planar<T, A>), dim3(blocks_for(nrow * (size_t)p)), dim3(256), 0, st, X, ldx, n, p,
                       nrow, Ws, ldw, gate);
  if (A1) {
    if (Ws)  // the T1 copy from the planar one (contiguous reads and writes)
      hipLaunchKernelGGL((k_planar_to_t1<A, E>), dim3(blocks_for(nrow / KV * 2 * (size_t)p)), dim3(256), 0, st, Ws,
                         ldw, nrow, 2 * p, A1);
    else
      hipLaunchKernelGGL((k_split_t1<T, E>), dim3(blocks_for(nrow / KV * 2 * (size_t)p)), dim3(256), 0, st, X, ldx, n,
                         p, c0, nrow, A1);
  }
  if (A2) {
    const size_t groups = (size_t)((c0 + 2 * p + KV - 1) / KV - c0 / KV);
    hipLaunchKernelGGL((k_split_t2<T, E>), dim3(blocks_for(nrow * groups)), dim3(256), 0, st, X, ldx, n, p, c0, nrow,
                       ccap, A2);
  }
  return hipGetLastError();
}

template <class A, class E>
hipError_t launch_tsq_to_t1(const A* Ws, size_t ldw, size_t nrow, int nb, E* B1, hipStream_t st) {
  if (nb < 1 || nrow % 32 || ldw < nrow) return hipErrorInvalidValue;
  const size_t work = nrow / GemmTile<E>::KV * (size_t)nb;
  hipLaunchKernelGGL((k_planar_to_t1<A, E>), dim3(blocks_for(work)), dim3(256), 0, st, Ws, ldw, nrow, nb, B1);
  return hipGetLastError();
}

namespace {
template <class E, int NT, bool NF>
void launch_proj_kernel(unsigned nblocks, const E* A1, int ma, const E* B1, int nb, size_t nrow, int kc, int gy,
                        typename GemmTile<E>::Acc* part, hipStream_t st, const int* gate) {
  hipLaunchKernelGGL((k_tsq_proj<E, NT, NF>), dim3(nblocks), dim3(256), 0, st, A1, ma, B1, nb, nrow, kc, gy, part,
                     gate);
}
// Blocks of the projection kernel that the device holds at once (its compute units times the
// kernel's occupancy), per device and kernel.
template <class E, int NT, bool NF>
int proj_slots() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  if (cached[dev] > 0) return cached[dev];
  int cus = 0, per = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, reinterpret_cast<const void*>(&k_tsq_proj<E, NT, NF>), 256,
                                                   0) != hipSuccess ||
      cus < 1 || per < 1)
    return 1024;
  cached[dev] = cus * per;
  return cached[dev];
}
template <class E, bool NF>
int proj_slots_nt(int nt) {
  switch (nt) {
    case 1: return proj_slots<E, 1, NF>();
    case 2: return proj_slots<E, 2, NF>();
    case 3: return proj_slots<E, 3, NF>();
    case 4: return proj_slots<E, 4, NF>();
    default:
      if constexpr (128 / GemmTile<E>::R > 4) {
        switch (nt) {
          case 5: return proj_slots<E, 5, NF>();
          case 6: return proj_slots<E, 6, NF>();
          case 7: return proj_slots<E, 7, NF>();
          default: return proj_slots<E, 8, NF>();
        }
      }
      return 1024;
  }
}
template <class E, bool NF>
hipError_t proj_nt(int nt, unsigned nblocks, const E* A1, int ma, const E* B1, int nb, size_t nrow, int kc, int gy,
                   typename GemmTile<E>::Acc* part, hipStream_t st, const int* gate) {
  constexpr int NTMAX = 128 / GemmTile<E>::R;
  switch (nt) {
    case 1: launch_proj_kernel<E, 1, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
    case 2: launch_proj_kernel<E, 2, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
    case 3: launch_proj_kernel<E, 3, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
    case 4: launch_proj_kernel<E, 4, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
    default:
      if constexpr (NTMAX > 4) {
        switch (nt) {
          case 5: launch_proj_kernel<E, 5, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
          case 6: launch_proj_kernel<E, 6, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
          case 7: launch_proj_kernel<E, 7, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
          case 8: launch_proj_kernel<E, 8, NF>(nblocks, A1, ma, B1, nb, nrow, kc, gy, part, st, gate); break;
          default: return hipErrorInvalidValue;
        }
      } else {
        return hipErrorInvalidValue;
      }
  }
  return hipGetLastError();
}
// part = the chunk products of A^T B (see k_tsq_proj); the chunk count to *nch_out
template <class E, bool NF>
hipError_t proj_any(const E* A1, int ma, const E* B1, int nb, size_t nrow, typename GemmTile<E>::Acc* part,
                    size_t part_cap, int* nch_out, hipStream_t st, const int* gate = nullptr) {
  using Tl = GemmTile<E>;
  if (ma < 1 || nb < 1 || nb > 128 || nrow % 32 || nrow == 0) return hipErrorInvalidValue;
  const int mt = (ma + Tl::R - 1) / Tl::R, nt = (nb + Tl::R - 1) / Tl::R;
  const int gy = (mt + 3) / 4;
  const size_t tpc = nrow / Tl::KS;
  // one wave of blocks (the blocks the device holds at once, so that none waits for a second
  // round), at least 4 k-steps a chunk, the chunk products at most a quarter of the bytes of A
  // (and within part_cap); a multiple of 8 chunks
  const size_t pbytes = (size_t)ma * nb * sizeof(typename Tl::Acc);
  size_t nch = (size_t)proj_slots_nt<E, NF>(nt) / (size_t)gy;
  if (nch > tpc / 4) nch = tpc / 4;
  const size_t byA = (size_t)nrow * ma * sizeof(E) / 4 / pbytes;
  if (nch > byA) nch = byA;
  const size_t cap_ch = part_cap / ((size_t)ma * nb);
  if (cap_ch < 8) return hipErrorInvalidValue;
  if (nch > cap_ch) nch = cap_ch;
  nch = nch / 8 * 8;
  if (nch < 8) nch = 8;
  const size_t kc = (tpc + nch - 1) / nch;
  *nch_out = (int)nch;
  const unsigned nblocks = (unsigned)(nch * gy);
  return proj_nt<E, NF>(nt, nblocks, A1, ma, B1, nb, nrow, (int)kc, gy, part, st, gate);
}
// Sums groups of 16 chunk products when there are more than 16 (FP64, into scratch); returns the
// products the final combine reads and their count.
template <class A>
hipError_t chunk_groups(const A* part, int nch, size_t L, double* scratch, size_t scratch_cap, const double** out,
                        int* nout, hipStream_t st, const int* gate = nullptr) {
  constexpr int kCpg = 16;
  const int g = (nch + kCpg - 1) / kCpg;
  if ((size_t)g * L > scratch_cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_chunk_sum<A>), dim3(blocks_for(L), (unsigned)g), dim3(256), 0, st, part, nch, L, kCpg, scratch,
                     gate);
  *out = scratch;
  *nout = g;
  return hipGetLastError();
}
}  // namespace

template <class E>
hipError_t launch_tsq_proj(const E* A1, int ma, const E* B1, int nb, size_t nrow, typename GemmTile<E>::Acc* part,
                           size_t part_cap, int* nch_out, hipStream_t st) {
  return proj_any<E, false>(A1, ma, B1, nb, nrow, part, part_cap, nch_out, st, nullptr);
}

template <class A, class E, class T>
hipError_t launch_tsq_combine(const A* part, int nch, int nq, int p, c2<T>* H, E* Hb, int ldhb, double* scratch,
                              size_t scratch_cap, hipStream_t st) {
  if (nch < 1 || p < 1 || nq < p || ldhb < 2 * nq) return hipErrorInvalidValue;
  const unsigned nb = blocks_for((size_t)nq * p);
  if (nch > 16) {
    const double* g;
    int ng;
    hipError_t e = chunk_groups<A>(part, nch, (size_t)4 * nq * p, scratch, scratch_cap, &g, &ng, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_tsq_combine<double, E, T>), dim3(nb), dim3(256), 0, st, g, ng, nq, p, H, Hb, ldhb);
  } else {
    hipLaunchKernelGGL((k_tsq_combine<A, E, T>), dim3(nb), dim3(256), 0, st, part, nch, nq, p, H, Hb, ldhb);
  }
  return hipGetLastError();
}

template <class E>
hipError_t launch_tsq_update(const E* A2, int mc, size_t ccap, size_t nrow, const E* Hb, int ldhb, int nb,
                             typename GemmTile<E>::Acc* Ws, size_t ldw, hipStream_t st) {
  using Tl = GemmTile<E>;
  if (mc < 1 || nb < 1 || nb > 128 || nrow % 32 || ccap % 32 || (size_t)mc > ccap || ldw < nrow || ldhb < mc ||
      ldhb % Tl::KV)
    return hipErrorInvalidValue;
  const int nt = (nb + Tl::R - 1) / Tl::R;
  // eight waves a block where Hb is large (more rows share each staged chunk), else four
  const unsigned g4 = (unsigned)((nrow / Tl::R + 3) / 4), g8 = (unsigned)((nrow / Tl::R + 7) / 8);
  constexpr int NTMAX = 128 / Tl::R;
#define DIE_UPD(NT_)                                                                                                \
  case NT_:                                                                                                         \
    if constexpr (NT_ <= NTMAX) {                                                                                   \
      if constexpr (NT_ * Tl::R > 64)                                                                               \
        hipLaunchKernelGGL((k_tsq_update<E, NT_, 8>), dim3(g8), dim3(512), 0, st, A2, mc, ccap, nrow, Hb, ldhb, nb, \
                           Ws, ldw);                                                                                \
      else                                                                                                          \
        hipLaunchKernelGGL((k_tsq_update<E, NT_, 4>), dim3(g4), dim3(256), 0, st, A2, mc, ccap, nrow, Hb, ldhb, nb, \
                           Ws, ldw);                                                                                \
      break;                                                                                                        \
    } else {                                                                                                        \
      return hipErrorInvalidValue;                                                                                  \
    }
  switch (nt) {
    DIE_UPD(1)
    DIE_UPD(2)
    DIE_UPD(3)
    DIE_UPD(4)
    DIE_UPD(5)
    DIE_UPD(6)
    DIE_UPD(7)
    DIE_UPD(8)
    default:
      return hipErrorInvalidValue;
  }
#undef DIE_UPD
  return hipGetLastError();
}

template <class A>
hipError_t launch_gram_planar(const A* Xs, size_t nrow, int p, A* part, size_t part_cap, double* scratch,
                              size_t scratch_cap, double2* G, hipStream_t st, const int* gate) {
  if (p < 1 || p > 64) return hipErrorInvalidValue;
  int nch = 0;
  hipError_t e = proj_any<A, true>(Xs, 2 * p, Xs, 2 * p, nrow, part, part_cap, &nch, st, gate);
  if (e != hipSuccess) return e;
  const unsigned nb = blocks_for((size_t)p * p);
  if (nch > 16) {
    const double* g;
    int ng;
    e = chunk_groups<A>(part, nch, (size_t)4 * p * p, scratch, scratch_cap, &g, &ng, st, gate);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_gram_combine<double>), dim3(nb), dim3(256), 0, st, g, ng, p, G, gate);
  } else {
    hipLaunchKernelGGL((k_gram_combine<A>), dim3(nb), dim3(256), 0, st, part, nch, p, G, gate);
  }
  return hipGetLastError();
}

namespace {
template <class T, bool PLANAR>
hipError_t cplx_rmul(const void* X, size_t ldx, int s, const c2<T>* S, int lds, int q, size_t n, c2<T>* Y, size_t ldy,
                     hipStream_t st, const int* ctl, c2<T>* Yalt) {
  if (s < 1 || q < 1 || q > 64 || lds < s || (!PLANAR && ldx < n) || ldy < n || X == (const void*)Y ||
      (ctl && (!Yalt || X == (const void*)Yalt)))
    return hipErrorInvalidValue;
  if (n == 0) return hipSuccess;
  constexpr int R = Mf1<T>::R;
  const int nt = (q + R - 1) / R;
  const unsigned grid = (unsigned)((n + 4 * R - 1) / (4 * R));
  switch (nt) {
    case 1:
      hipLaunchKernelGGL((k_cplx_rmul<T, 1, PLANAR>), dim3(grid), dim3(256), 0, st, X, ldx, s, S, lds, q, n, Y, ldy,
                         ctl, Yalt);
      break;
    case 2:
      hipLaunchKernelGGL((k_cplx_rmul<T, 2, PLANAR>), dim3(grid), dim3(256), 0, st, X, ldx, s, S, lds, q, n, Y, ldy,
                         ctl, Yalt);
      break;
    case 3:
      if constexpr (R == 16) {
        hipLaunchKernelGGL((k_cplx_rmul<T, 3, PLANAR>), dim3(grid), dim3(256), 0, st, X, ldx, s, S, lds, q, n, Y, ldy,
                         ctl, Yalt);
        break;
      }
      return hipErrorInvalidValue;
    case 4:
      if constexpr (R == 16) {
        hipLaunchKernelGGL((k_cplx_rmul<T, 4, PLANAR>), dim3(grid), dim3(256), 0, st, X, ldx, s, S, lds, q, n, Y, ldy,
                         ctl, Yalt);
        break;
      }
      return hipErrorInvalidValue;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}
}  // namespace

template <class T>
hipError_t launch_cplx_rmul(const c2<T>* X, size_t ldx, int s, const c2<T>* S, int lds, int q, size_t n, c2<T>* Y,
                            size_t ldy, hipStream_t st, const int* ctl, c2<T>* Yalt) {
  return cplx_rmul<T, false>(X, ldx, s, S, lds, q, n, Y, ldy, st, ctl, Yalt);
}

template <class T>
hipError_t launch_cplx_rmul_planar(const T* Xs, size_t ldw, int s, const c2<T>* S, int lds, int q, size_t n, c2<T>* Y,
                                   size_t ldy, hipStream_t st, const int* ctl, c2<T>* Yalt) {
  if (ldw < n) return hipErrorInvalidValue;
  return cplx_rmul<T, true>(Xs, ldw, s, S, lds, q, n, Y, ldy, st, ctl, Yalt);
}

namespace {
template <int KC>
hipError_t trsm_kc(const double2* R, int ldr, int nc, double2* B, int ldb, int k, hipStream_t st) {
  // the columns' rows in LDS: at most 64 KiB beside the kernel's own 68 KiB
  static bool attr_set[64] = {false};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  if (!attr_set[dev]) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_trsm_upper<KC>),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, 65536);
    if (e != hipSuccess) return e;
    attr_set[dev] = true;
  }
  hipLaunchKernelGGL((k_trsm_upper<KC>), dim3((unsigned)((k + KC - 1) / KC)), dim3(1024),
                     (size_t)KC * nc * sizeof(double2), st, R, ldr, nc, B, ldb, k);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_trsm_upper(const double2* R, int ldr, int nc, double2* B, int ldb, int k, hipStream_t st) {
  if (nc < 1 || nc > kTrsmMaxRows || ldr < nc || ldb < nc || k < 1) return hipErrorInvalidValue;
  // two columns a block where their rows fit in 64 KiB of LDS, else one
  return nc <= kTrsmMaxRows / 2 ? trsm_kc<2>(R, ldr, nc, B, ldb, k, st) : trsm_kc<1>(R, ldr, nc, B, ldb, k, st);
}

template <class T>
hipError_t launch_cadd2(const c2<T>* A, int lda, const c2<T>* B, int ldb, int rows, int cols, c2<T>* C, int ldc,
                        hipStream_t st) {
  if (rows < 1 || cols < 1 || lda < rows || ldb < rows || ldc < rows) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_cadd2<T>), dim3(blocks_for((size_t)rows * cols)), dim3(256), 0, st, A, lda, B, ldb, rows, cols,
                     C, ldc);
  return hipGetLastError();
}

#define DIE_INST_T(T)                                                                                              \
  template hipError_t launch_gram_planar<T>(const T*, size_t, int, T*, size_t, double*, size_t, double2*, hipStream_t, \
                                            const int*);                                                             \
  template hipError_t launch_cplx_rmul_planar<T>(const T*, size_t, int, const c2<T>*, int, int, size_t, c2<T>*,      \
                                                  size_t, hipStream_t, const int*, c2<T>*);                          \
  template hipError_t launch_cplx_rmul<T>(const c2<T>*, size_t, int, const c2<T>*, int, int, size_t, c2<T>*, size_t, \
                                          hipStream_t, const int*, c2<T>*);                                         \
  template hipError_t launch_cadd2<T>(const c2<T>*, int, const c2<T>*, int, int, int, c2<T>*, int, hipStream_t);
DIE_INST_T(float)
DIE_INST_T(double)
#undef DIE_INST_T

#define DIE_INST_E(T, E)                                                                                            \
  template hipError_t launch_tsq_split<T, typename GemmTile<E>::Acc, E>(const c2<T>*, size_t, size_t, int, int, size_t, \
                                                                        size_t, typename GemmTile<E>::Acc*, size_t, E*, \
                                                                        E*, hipStream_t, const int*);                \
  template hipError_t launch_tsq_to_t1<typename GemmTile<E>::Acc, E>(const typename GemmTile<E>::Acc*, size_t, size_t, \
                                                                     int, E*, hipStream_t);                          \
  template hipError_t launch_tsq_proj<E>(const E*, int, const E*, int, size_t, typename GemmTile<E>::Acc*, size_t,    \
                                         int*, hipStream_t);                                                          \
  template hipError_t launch_tsq_combine<typename GemmTile<E>::Acc, E, T>(const typename GemmTile<E>::Acc*, int, int, \
                                                                          int, c2<T>*, E*, int, double*, size_t,      \
                                                                          hipStream_t);                               \
  template hipError_t launch_tsq_update<E>(const E*, int, size_t, size_t, const E*, int, int,                        \
                                           typename GemmTile<E>::Acc*, size_t, hipStream_t);
DIE_INST_E(float, _Float16)
DIE_INST_E(float, float)
DIE_INST_E(double, double)
#undef DIE_INST_E

}  // namespace die
