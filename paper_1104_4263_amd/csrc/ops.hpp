// Internal launch interface between the host runtime and the HIP kernels.
#pragma once
#include "common.hpp"

namespace die {

// ---------------------------------------------------------------- FFT passes
// Twiddle tables exp(-2 pi i j / 4096) for the current device (created on first use).
hipError_t fft_tables(const double2** tw64, const float2** tw32);

// Variants of the three product passes (the `v` argument; see kernels_fft.hip): bit 0 the
// other radix, bit 1 half the tile.  Only transforms of length >= 2^kFftTunedMinLog have
// them (shorter ones, the inverse and the unpadded row transforms always use variant 0).
constexpr int kFftVariants = 4;
constexpr int kFftTunedMinLog = 7;

// The product's FFT intermediate is tiled: one plane per (right-hand side, component) of
// wtile_cols(px) x wtile_rows(ny) values in kWTile x kWTile tiles (one 128-byte line of
// complex64), the tiles of one column strip (kWTile columns) contiguous:
// element (x, y) at ((x / kWTile) rows4 / kWTile + y / kWTile) kWTile^2 + (x % kWTile) kWTile
// + y % kWTile, rows4 = wtile_rows(ny).  The column pass (kWTile columns per block) reads and
// writes one contiguous run per block; the row passes (kWTile rows per block or more) whole
// lines, adjacent ones for adjacent row tiles.
constexpr int kWTile = 4;
__host__ __device__ constexpr int wtile_rows(int ny) { return (ny + kWTile - 1) / kWTile * kWTile; }
__host__ __device__ constexpr int wtile_cols(int px) { return (px + kWTile - 1) / kWTile * kWTile; }
__host__ __device__ constexpr size_t wtile_index(int x, int y, int rows4) {
  return ((size_t)(x / kWTile) * (rows4 / kWTile) + y / kWTile) * (kWTile * kWTile) + (x % kWTile) * kWTile +
         y % kWTile;
}

// Pass 1.  For every set s = r * spr + c (r < nrhs right-hand sides, c < spr components)
// and row y < nrows: W[s][x][y] = FFT_N( pad_N( chi[y][:] * x_in[s][y][:] ) )[x],
// x < N = 2^logn (chi may be NULL).  x_in rows have nx <= N entries; W is the tiled
// intermediate above for the zero-padded product (2 nx <= N, not inverse), else transposed
// ([N][nrows]).  A block handles the spr sets of rb right-hand sides (rb = 0: automatic).
// chi holds one [nrows][nx] plane per object; right-hand side r uses plane r / rpo
// (rpo = 0: every right-hand side uses the first plane).
// chi2 (may be NULL): the contrast of components c >= 2 (H3 of the full TE system, chi_m),
// laid out as chi.
template <class T, class S>
hipError_t launch_rows_fwd(int logn, bool inverse, const c2<S>* x_in, const c2<T>* chi, const c2<T>* chi2, c2<T>* W,
                           int nx, int nrows, int nrhs, int spr, int rb, int rpo, const int* live,
                           hipStream_t st, int v = 0);

// Symbol values per frequency for ncomp field components: the upper triangle of the symmetric
// ncomp x ncomp Green-tensor symbol (1: TM; 3: T11, T12, T22; 6: T11, T12, T22, T13, T23, T33).
__host__ __device__ constexpr int sym_planes(int ncomp) { return ncomp == 1 ? 1 : (ncomp == 2 ? 3 : 6); }

// Pass 2.  For every rhs r and column x < ncols of the tiled W (components c < ncomp):
// FFT_N over y (zero padded), multiply by the symmetric symbol sym[x][ky][sym_planes(ncomp)],
// inverse FFT_N, keep y < nrows; in place.
template <class T>
hipError_t launch_cols_symbol(int logn, int ncomp, c2<T>* W, const c2<T>* sym, int ncols, int nrows, int nrhs,
                              const int* live, hipStream_t st, int v = 0);

// Pass 3.  y_out[s][y][x] = u[s][y][x] - IFFT_N(W[s][:][y])[x] for x < nx (W tiled).
// With planar (a real array in S), y is written planar instead: right-hand side r's element i
// (i = component nrows nx + y nx + x) to planar[r ldp + i] (real) and planar[(pw + r) ldp + i]
// (imaginary), y_out unused.
template <class T, class S>
hipError_t launch_rows_inv_sub(int logn, const c2<T>* W, const c2<S>* u, c2<S>* y_out, int nx,
                               int nrows, int nsets, int sets_per_rhs, const int* live,
                               hipStream_t st, int v = 0, S* planar = nullptr, size_t ldp = 0, int pw = 0);

// Full-length FFT along the contiguous axis of W[nsets][ncols][N], in place.
template <class T>
hipError_t launch_cols_plain(int logn, bool inverse, c2<T>* W, int ncols, int nsets, hipStream_t st);

// out[b][j][i] = in[b][i][j] for in of shape [nb][rows][cols].
template <class T>
hipError_t launch_transpose(const c2<T>* in, c2<T>* out, int rows, int cols, int nb, hipStream_t st);

// sym64[(x * py + ky) * npl + a] = scale * W[a][x][ky]; sym32 the rounded copy.
hipError_t launch_pack_symbol(const double2* W, double2* sym64, float2* sym32, int px, int py, int npl,
                              double scale, hipStream_t st);

// ------------------------------------------------------------- Krylov BLAS-1
constexpr int kBlasThreads = 256;
constexpr int kBlasEpt = 4;
inline int blas_blocks(size_t n) {
  return (int)((n + (size_t)kBlasThreads * kBlasEpt - 1) / ((size_t)kBlasThreads * kBlasEpt));
}

// part[(r * nv + i) * nblk + b] = sum over block b of conj(A_i,r[e]) * B_r[e],
// A_i,r = A + i * a_vs + r * a_rs, B_r = B + r * b_rs, e < n.  nv_r = nv_dev ? nv_dev[r] : nv.
template <class SA, class SB>
hipError_t launch_mdot(const c2<SA>* A, size_t a_vs, size_t a_rs, int nv, const int* nv_dev,
                       const c2<SB>* B, size_t b_rs, size_t n, int nrhs, double2* part,
                       const int* live, hipStream_t st);

// out[r * nv + i] = sign * sum_b part[(r * nv + i) * nblk + b]; if C (nv x nv, row-major,
// shared by all r) is given, out[r] is replaced by C * out[r].
hipError_t launch_reduce(const double2* part, int nv, int nblk, int nrhs, double sign,
                         const double2* C, double2* out, const int* live, hipStream_t st);

// Y_r = beta * Y_r + alpha * X_r + sum_{i < nv_r} coef[r * ldc + i] * A_i,r   (X may be NULL,
// X may alias Y).  MODE 0: nothing else; 1: also part = partial dots conj(A_i) . Y_new (CGS2
// second pass, nv_r vectors); 2: also partn[r * nblk + b] = partial ||Y_new||^2.
template <class SA, class SX, class SY>
hipError_t launch_maxpy(int mode, const c2<SA>* A, size_t a_vs, size_t a_rs, int nv,
                        const int* nv_dev, const double2* coef, int ldc, const c2<SX>* X,
                        size_t x_rs, double alpha, c2<SY>* Y, size_t y_rs, double beta, size_t n,
                        int nrhs, double2* part, double* partn, const int* live, hipStream_t st);

// partn[r * nblk + b] = partial ||X_r||^2.
template <class S>
hipError_t launch_norm2(const c2<S>* X, size_t x_rs, size_t n, int nrhs, double* partn,
                        const int* live, hipStream_t st);

// out[r] = sum_b partn[r * nblk + b]
hipError_t launch_reduce_norm(const double* partn, int nblk, int nrhs, double* out,
                              const int* live, hipStream_t st);

// Y_r = s_r * X_r with s_r = scale[r * sstride] (double), converting precision.  X may alias Y.
template <class SX, class SY>
hipError_t launch_scale(const c2<SX>* X, size_t x_rs, c2<SY>* Y, size_t y_rs, const double* scale,
                        int sstride, size_t n, int nrhs, const int* live, hipStream_t st);

// u[idx[c]] += src[c] for c < k <= 65535: src [k][n] in S, u [*][n] complex128 (block GMRES update).
template <class S>
hipError_t launch_add_cols(const c2<S>* src, size_t n, const int* idx, int k, double2* u, hipStream_t st);

// QR of the block upper Hessenberg H (mr x nc, column-major, leading dimension ld, at most p
// sub-diagonals, nc a multiple of p, p <= kPanelMaxCols) in place, p columns at a time, with the
// same reflectors applied to B (mr x k, leading dimension ldb): on return R is in H[0:nc, 0:nc]
// and Q^H B in B.  U (kPanelMaxRows x p complex) and s (p doubles) are scratch.  Complex FP64.
constexpr int kPanelMaxCols = 64;
constexpr int kPanelMaxRows = 2 * kPanelMaxCols;
hipError_t launch_block_hessenberg_qr(double2* H, int ld, int mr, int nc, int p, double2* B, int ldb, int k,
                                      double2* U, double* s, hipStream_t st);

// Block Gram-Schmidt products on the matrix cores (kernels_gemm.hip).  Element types E:
// binary16, FP32, FP64; R rows per MFMA tile, KV values per 16-byte lane load, KS = (64 / R) KV
// reduction values per tile, Acc the accumulation type.  Tiled layouts of an nrow-row matrix
// (nrow and the column capacity ccap multiples of 32; a T1 buffer holds the columns rounded up
// to a multiple of 32, a T2 buffer ccap):
//   T1 (the projection's operands): element (n, c) at t1(n, c, nrow);
//   T2 (the update's basis operand): element (n, c) at t2(n, c, ccap).
template <class E> struct GemmTileBase;
template <> struct GemmTileBase<_Float16> { static constexpr int R = 32, KV = 8; using Acc = float; };
template <> struct GemmTileBase<float> { static constexpr int R = 32, KV = 4; using Acc = float; };
template <> struct GemmTileBase<double> { static constexpr int R = 16, KV = 2; using Acc = double; };
template <class E> struct GemmTile : GemmTileBase<E> {
  using Base = GemmTileBase<E>;
  static constexpr int R = Base::R, KV = Base::KV, KS = (64 / Base::R) * Base::KV, TILE = 64 * Base::KV;
  __host__ __device__ static constexpr size_t t1(size_t n, size_t c, size_t nrow) {
    return ((c / R) * (nrow / KS) + n / KS) * TILE + ((c % R) + R * ((n % KS) / KV)) * KV + n % KV;
  }
  __host__ __device__ static constexpr size_t t2(size_t n, size_t c, size_t ccap) {
    return ((n / R) * (ccap / KS) + c / KS) * TILE + ((n % R) + R * ((c % KS) / KV)) * KV + c % KV;
  }
};
__host__ __device__ constexpr size_t gemm_pad(size_t x) { return (x + 31) / 32 * 32; }

// Columns [c0, c0 + 2p) of the planar form of X (n x p complex, leading dimension ldx; rows n ..
// nrow - 1 zero): into Ws (planar, leading dimension ldw), A1 (T1) and A2 (T2, capacity ccap);
// any of the three may be null (Ws takes the columns 0 .. 2p - 1; with Ws and A1 both given, c0 = 0).
// gate (device int, only with Ws alone): the launch does nothing while *gate == 0.
template <class T, class A, class E>
hipError_t launch_tsq_split(const c2<T>* X, size_t ldx, size_t n, int p, int c0, size_t nrow, size_t ccap, A* Ws,
                            size_t ldw, E* A1, E* A2, hipStream_t st, const int* gate = nullptr);
// B1 (T1, columns 0 .. nb - 1) from the planar Ws (nrow rows, leading dimension ldw).
template <class A, class E>
hipError_t launch_tsq_to_t1(const A* Ws, size_t ldw, size_t nrow, int nb, E* B1, hipStream_t st);
// part[h][b ma + a] = sum over the rows of chunk h of A(n, a) B(n, b) (A: ma columns, B: nb <= 128
// columns, both T1 with nrow rows); the chunk count (at most part_cap / (ma nb)) goes to *nch.
template <class E>
hipError_t launch_tsq_proj(const E* A1, int ma, const E* B1, int nb, size_t nrow, typename GemmTile<E>::Acc* part,
                           size_t part_cap, int* nch, hipStream_t st);
// H (nq x p complex, leading dimension nq) = Q^H W from the nch chunk products of the planar
// projection (2nq x 2p each), summed in chunk order (more than 16 in two stages through scratch,
// at most scratch_cap doubles), rounded to E; Hb (2nq x 2p in E, leading dimension ldhb) the
// real matrix with which Ws -= Qs Hb is W -= Q H.
constexpr size_t kTsqScratch = (size_t)1 << 22;  // doubles of the two-stage sums that always suffice
template <class A, class E, class T>
hipError_t launch_tsq_combine(const A* part, int nch, int nq, int p, c2<T>* H, E* Hb, int ldhb, double* scratch,
                              size_t scratch_cap, hipStream_t st);
// Ws (nrow rows, nb <= 128 columns, leading dimension ldw) -= Q Hb over the mc columns of Q
// (T2, capacity ccap) and rows of Hb (leading dimension ldhb, a multiple of KV).
template <class E>
hipError_t launch_tsq_update(const E* A2, int mc, size_t ccap, size_t nrow, const E* Hb, int ldhb, int nb,
                             typename GemmTile<E>::Acc* Ws, size_t ldw, hipStream_t st);
// G (p x p, leading dimension p, FP64) = X^H X for the complex block X held planar in Xs (n x 2p,
// rows contiguous, leading dimension nrow, rows past the data zero; the buffer holds 2p rounded
// up to 32 columns), p <= 64: on the matrix cores in A (FP32 or FP64) with the chunk products in
// part (at most part_cap values), summed in FP64 (through scratch as for launch_tsq_combine).
// gate (device int): every launch does nothing while *gate == 0.
template <class A>
hipError_t launch_gram_planar(const A* Xs, size_t nrow, int p, A* part, size_t part_cap, double* scratch,
                              size_t scratch_cap, double2* G, hipStream_t st, const int* gate = nullptr);
// Y (n x q) = X (n x s) S (s x q, leading dimension lds), complex in T on the matrix cores, q <= 64;
// X and Y distinct.  ctl (device ints, with Yalt): nothing happens while ctl[0] == 0, and the result
// goes to Yalt (distinct from X, same leading dimension) while ctl[1] == 0.
template <class T>
hipError_t launch_cplx_rmul(const c2<T>* X, size_t ldx, int s, const c2<T>* S, int lds, int q, size_t n, c2<T>* Y,
                            size_t ldy, hipStream_t st, const int* ctl = nullptr, c2<T>* Yalt = nullptr);
// The same with X held planar in T (Xs: column c's real parts at c ldw, its imaginary parts at
// (s + c) ldw, ldw >= n).
template <class T>
hipError_t launch_cplx_rmul_planar(const T* Xs, size_t ldw, int s, const c2<T>* S, int lds, int q, size_t n, c2<T>* Y,
                                   size_t ldy, hipStream_t st, const int* ctl = nullptr, c2<T>* Yalt = nullptr);
// CholQR factor of a block from its Gram matrix G (p x p, FP64, leading dimension p), p <= 64, by
// one workgroup (no host round trip).  flags (device ints; every path writes each flag it owns):
// [0] pass 1 succeeded, [1] one pass suffices (smallest pivot of the unit-diagonal Gram's
// Cholesky >= single_piv), [2] a second pass is to run, [3] the block is orthonormalised,
// [4] the second factor is to be applied, [5] 1.  pass 1: R1 (FP64, p x p, zero below the
// diagonal) and R1^-1 (into Rinv, in T) from G; flags 0-2 and 5.  pass 2: while flags[2], R2^-1
// into Rinv from the second Gram and H = R2 R1, otherwise H = R1; H into Hb (leading dimension
// ldh, in T, zero below the diagonal); flags 3-4.  A pivot <= rel_tol x the largest diagonal entry
// fails the pass (the block is numerically rank deficient).
constexpr int kCholQRMax = 64;
template <class T>
hipError_t launch_cholqr_factor(const double2* G, int p, double rel_tol, double single_piv, int pass, double2* R1,
                                c2<T>* Rinv, int* flags, c2<T>* Hb, int ldh, hipStream_t st);
// Y (n x p complex, leading dimension ldy) = 0 unless *flag (device int): a block the device CholQR
// could not orthonormalise is cleared, so that work queued behind it reads zeros.
template <class T>
hipError_t launch_zero_unless(c2<T>* Y, size_t ldy, size_t n, int p, const int* flag, hipStream_t st);
// R Y = B in place in B (nc x k, leading dimension ldb) for the upper triangular R (leading
// dimension ldr), nc <= kTrsmMaxRows.
constexpr int kTrsmMaxRows = 4096;
hipError_t launch_trsm_upper(const double2* R, int ldr, int nc, double2* B, int ldb, int k, hipStream_t st);
// C = A + B (rows x cols).
template <class T>
hipError_t launch_cadd2(const c2<T>* A, int lda, const c2<T>* B, int ldb, int rows, int cols, c2<T>* C, int ldc,
                        hipStream_t st);

// Identity columns X[j][e] = (e == col0 + j), j < ncols, complex128 vectors of length n.
hipError_t launch_unit_cols(double2* X, size_t n, size_t col0, int ncols, hipStream_t st);
// Y_r = c[r][0] X0_r + c[r][1] X1_r + c[r][2] X2_r, complex128 vectors of length n per right-hand
// side (coefficients [nrhs][3]); an input may be null (skipped) or alias Y; only live[r] != 0
// (live may be null).
hipError_t launch_comb3(double2* Y, const double2* X0, const double2* X1, const double2* X2, const double2* coef,
                        size_t n, int nrhs, const int* live, hipStream_t st);

// ----------------------------------------------------------------- GMRES state
struct GmresState {
  int j;         // iterations done in the current cycle
  int done;      // cycle finished (target reached, m iterations, breakdown)
  int breakdown; // 1: non-finite value met
  int pad;
  double beta0;  // norm of the cycle's starting residual
  double target; // cycle stops when |g_{j}| <= target
  double resid;  // current residual estimate |g_j|
  double invbeta;// 1 / h_{j+1,j} of the last column (0 if breakdown)
};

// One Arnoldi column per live rhs: h = hsign (h1 + h2) (two CGS passes, [r * ldh + i], i <= j),
// beta = sqrt(sum_b partn[r * nblk + b]); Givens update of the (m+1) x m least-squares
// problem kept in R (column-major, [r][m * (m + 1)]), cs, sn, g; when the cycle ends,
// y = R^-1 g is written to y[r * m + i].  Clears live[r] when the cycle ends.
hipError_t launch_givens(const double2* h1, const double2* h2, int ldh, double hsign, const double* partn,
                         int nblk, GmresState* state, double2* R, double* cs, double2* sn, double2* g,
                         double2* y, int m, int nrhs, int* live, const int* active, hipStream_t st);

// ---- Arnoldi kernels for the GMRES inner loop (reductions finished by the last block)
// counter: nrhs * kCounterStride ints, zero on entry, left zero on exit.
// part: nrhs * gmres_part_elems(n, nv) partials.
constexpr int kDotChunkElems = 2048;
constexpr int kCounterStride = 1024;
inline size_t gmres_part_elems(size_t n, int nv) {
  const size_t dots = (size_t)nv * ((n + kDotChunkElems - 1) / kDotChunkElems) + (size_t)nv;
  const size_t axpy = 2 * ((n + 255) / 256) + 16;  // per-256 partials (+ up to 7 past the end) and group sums
  return dots > axpy ? dots : axpy;
}
// In the two kernels below the operand of right-hand side r is A + i * a_vs + (r / a_rpo) * a_rs
// (a_rpo right-hand sides share one set of vectors, e.g. the deflation basis of an object).
// out[r * nv + i] = sign * sum_e conj(A_i,r[e]) B_r[e]   (times C_(r / a_rpo) = C + (r / a_rpo) *
// c_stride when C is given).
template <class SA, class SB>
hipError_t launch_fdot(const c2<SA>* A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const c2<SB>* B, size_t b_rs,
                       size_t n, int nrhs, double2* part, double sign, const double2* C, size_t c_stride,
                       double2* out, int* counter, const int* live, hipStream_t st);
// W_r = X_r + sum_i coef[r * nv + i] A_i,r  (X NULL: W_r += ...).
template <class SA, class SW>
hipError_t launch_faxpy(const c2<SA>* A, size_t a_vs, size_t a_rs, int a_rpo, int nv, const double2* coef,
                        const c2<SW>* X, c2<SW>* W, size_t w_rs, size_t n, int nrhs, const int* live,
                        hipStream_t st);
// W_r += sum_i h2neg[r * nv + i] A_i,r; beta = ||W_r||; Givens update of column j = nv - 1 with
// h = -(h1neg + h2neg); clears live[r] when the cycle of rhs r ends.
template <class SA, class SW>
hipError_t launch_faxpy_givens(const c2<SA>* A, size_t a_vs, size_t a_rs, int nv, const double2* h2neg,
                               const double2* h1neg, c2<SW>* W, size_t w_rs, size_t n, int nrhs, double2* part,
                               int* counter, GmresState* state, double2* R, double* cs, double2* sn, double2* g,
                               int m, int* live, hipStream_t st);
// y_r = R_r^-1 g_r over the j_r columns of the cycle.
// One-reduction Arnoldi (CGS2 with the second projection delayed by a step): dots of
// Q_0..Q_{nq-1} and V against V and W (W null: zero second target), out[r ostride + 2 i + t]; the per-rhs scalar update of step j (delayed column j-1,
// Givens, stopping, coefficients); the pass that writes q_j and v_{j+1}.
// part: nrhs * gmres_part_elems(n, 2 (nq + 1)); counter as for launch_fdot.
template <class SQ, class SV>
hipError_t launch_dots2(const c2<SQ>* Q, size_t q_vs, int nq, const c2<SV>* V, const c2<SV>* W, size_t rs, size_t n,
                        int nrhs, double2* part, double2* out, int ostride, int* counter, const int* live,
                        hipStream_t st);
hipError_t launch_dcgs_update(const double2* D, int dstride, int j, int m, int nrhs, GmresState* state, double2* Hu,
                              double2* R, double* cs, double2* sn, double2* g, double2* c, double2* coef, int* live,
                              hipStream_t st);
// q_j into basis slot j (Q), v_{j+1} into V in place, reading w from W.
template <class SQ, class SV>
hipError_t launch_dcgs_axpy(c2<SQ>* Q, size_t q_vs, int j, c2<SV>* V, const c2<SV>* W, size_t rs, size_t n, int nrhs,
                            const double2* coef, int ld, const GmresState* state, const int* live, hipStream_t st);
hipError_t launch_lsq(const GmresState* state, const double2* R, const double2* g, double2* y, int m, int nrhs,
                      const int* active, hipStream_t st);

}  // namespace die
