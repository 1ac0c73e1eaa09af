// Launchers of the U-Net kernels (kernels_unet.hip) used by the host code in unet.cpp.
// Activations are NHWC bfloat16 (raw 16-bit storage, round to nearest even from float32);
// gradients of activations are NHWC float32; parameters and their gradients float32.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace die {
namespace nn {

using bf16raw = uint16_t;

enum ConvOut { kOutBf16 = 0, kOutF32 = 1, kOutF32Add = 2 };

// out[p][n] (op)= act( sum_k A(p, k) Wm[n][k] + bias[n] ), an implicit GEMM on MFMA
// (bf16 operands, float32 accumulation).  A(p, k) with k = t cin + ci is X at the pixel
// p shifted by tap t (zero outside the image); flip = true uses the opposite shift (the
// backward-data convolution).  X: [B][H][W][cin] bf16, cin % 8 == 0; Wm: [cout][taps cin]
// bf16; taps 9 (3x3, zero padding 1) or 1; bias float32 [cout] or null.
hipError_t launch_conv(const bf16raw* X, int B, int H, int W, int cin, int taps, bool flip, const bf16raw* Wm,
                       const float* bias, bool relu, void* out, int cout, ConvOut mode, hipStream_t st);

// Weight gradient partials: part[s][co][t cin + ci] = sum over the pixels of split s of
// dZ[p][co] X[p + d_t][ci].  W % 8 == 0.  Returns the number of splits through *nsplit
// (the caller sizes part with conv_wgrad_max_floats).
size_t conv_wgrad_max_floats(int cout, int taps, int cin);
// dZ rows have ldz >= cout entries.
hipError_t launch_conv_wgrad(const bf16raw* dZ, int ldz, const bf16raw* X, int B, int H, int W, int cin, int taps,
                             int cout, float* part, int* nsplit, hipStream_t st);
// The same partials and the bias gradient partials bpart[s][co] = sum over the pixels of split
// s of dZ[p][co] in one kernel that stages 32-pixel chunks in LDS; needs W % 32 == 0 and
// ldz % 8 == 0 (conv_wgrad_bias_fused).  bpart holds at least 256 cout floats.
bool conv_wgrad_bias_fused(int W, int ldz, int cout);
hipError_t launch_conv_wgrad_bias(const bf16raw* dZ, int ldz, const bf16raw* X, int B, int H, int W, int cin,
                                  int taps, int cout, float* part, float* bpart, int* nsplit, hipStream_t st);
// Bias gradient partials: part[s][co] = sum over the pixels of split s of dZ[p][co].
hipError_t launch_bias_grad(const bf16raw* dZ, int ldz, long npix, int cout, float* part, int nsplit, hipStream_t st);
// out[j] = sum_s part[s][j] for j < count (fixed order).
hipError_t launch_reduce_splits(const float* part, int nsplit, size_t count, float* out, hipStream_t st);

// dZ = bf16(Y > 0 ? dY : 0) (ReLU layers) or bf16(dY) (Y null).
hipError_t launch_relu_grad(const float* dY, const bf16raw* Y, bf16raw* dZ, size_t count, hipStream_t st);
// 2x2 average pool of [B][H][W][C] -> [B][H/2][W/2][C], and its adjoint accumulated into dX.
hipError_t launch_pool(const bf16raw* X, bf16raw* Y, int B, int H, int W, int C, hipStream_t st);
hipError_t launch_pool_grad_add(const float* dY, float* dX, int B, int H, int W, int C, hipStream_t st);
// cat[b][y][x] = [low[b][y/2][x/2][0:cl], skip[b][y][x][0:cs]] and the adjoint (written).
hipError_t launch_upcat(const bf16raw* low, const bf16raw* skip, bf16raw* cat, int B, int H, int W, int cl, int cs,
                        hipStream_t st);
hipError_t launch_upcat_grad(const float* dcat, float* dlow, float* dskip, int B, int H, int W, int cl, int cs,
                             hipStream_t st);
// float32 -> bf16 (the network input).
hipError_t launch_to_bf16(const float* x, bf16raw* y, size_t count, hipStream_t st);
// Mean-square loss over out, t [npix][4]: loss_part[block] partial sums of (out - t)^2 and
// dZ [npix][8] = bf16(2 (out - t) / count) in channels 0..3, zero in 4..7.
int loss_blocks(size_t count);
hipError_t launch_mse(const float* out, const float* t, size_t count, double* loss_part, bf16raw* dZ,
                      hipStream_t st);
hipError_t launch_sum_doubles(const double* part, int n, double* out, hipStream_t st);
// Adam (bias-corrected) on float32 master weights; refreshes the bf16 copy.
hipError_t launch_adam(float* w, const float* g, float* m, float* v, bf16raw* wbf, size_t n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t st);
hipError_t launch_to_bf16_params(const float* w, bf16raw* wbf, size_t n, hipStream_t st);
// Backward-data weights of one layer: Wbd[ci][t cpad + co] = Wf[co][t cin + ci] (zero for
// co >= cout; cpad >= cout keeps the reduction length a multiple of 8).
hipError_t launch_wbd(const bf16raw* Wf, bf16raw* Wbd, int cout, int cpad, int taps, int cin, hipStream_t st);

// Inputs from the permittivity (or contrast) and the incident field, complex128:
// eps [nobj][ny][nx] (chi = eps - shift), e_in [batch][2][ny][nx]; sample r uses object
// (r0 + r) / rpo (rpo = 0: object 0).  x: [batch][ny][nx][8] float32.
hipError_t launch_pack_inputs(const double2* eps, double shift, int rpo, int r0, const double2* e_in, float* x,
                              int batch, int ny, int nx, hipStream_t st);
// Targets [batch][ny][nx][4] = Re/Im of e_tot - e_in per component.
hipError_t launch_pack_targets(const double2* e_tot, const double2* e_in, float* t, int batch, int ny, int nx,
                               hipStream_t st);
// x0 = e_in + (network output as the scattered field), complex128 [batch][2][ny][nx].
hipError_t launch_unpack_guess(const double2* e_in, const float* y, double2* x0, int batch, int ny, int nx,
                               hipStream_t st);

}  // namespace nn
}  // namespace die
