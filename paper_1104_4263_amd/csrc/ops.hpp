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
template <class T, class S>
hipError_t launch_rows_inv_sub(int logn, const c2<T>* W, const c2<S>* u, c2<S>* y_out, int nx,
                               int nrows, int nsets, int sets_per_rhs, const int* live,
                               hipStream_t st, int v = 0);

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

// Planar binary16 GEMM path of the block Arnoldi step (complex64 blocks, n even).
// launch_planar_split: X (n x p complex, leading dimension ldx) to Xs (n x 2p FP32: real parts,
// then imaginary parts; leading dimension ldo) and/or Xh (the same in binary16); either may be null.
hipError_t launch_planar_split(const float2* X, size_t ldx, size_t n, int p, float* Xs, _Float16* Xh, size_t ldo,
                               hipStream_t st);
// launch_planar_merge: Xs (planar FP32, leading dimension lds) back to X (interleaved).
hipError_t launch_planar_merge(const float* Xs, size_t lds, size_t n, int p, float2* X, size_t ldx, hipStream_t st);
// launch_planar_to_half: the binary16 copy of a planar FP32 block (n x 2p, leading dimension ld;
// n and ld even).
hipError_t launch_planar_to_half(const float* Xs, size_t ld, size_t n, int p, _Float16* Xh, hipStream_t st);
// launch_planar_combine: H (nq x p complex, leading dimension nq) = Q^H W from nch chunk products
// C_b = Qs^T Ws (2nq x 2p FP32, leading dimension 2nq, stride 4 nq p), summed in chunk order and
// rounded to binary16; Hb (2nq x 2p binary16, leading dimension 2nq) the real matrix with
// Ws -= Qs Hb equal to W -= Q H.  Qs holds each p-column block of Q planar.
hipError_t launch_planar_combine(const float* C, int nch, int nq, int p, float2* H, _Float16* Hb, hipStream_t st);

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
