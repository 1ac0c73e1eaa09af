// U-Net kernels for the learned GMRES warm start (gfx950, wave64).
//
// Convolutions are implicit GEMMs on the matrix cores: v_mfma_f32_32x32x16_bf16, one
// 32 x 32 output tile per wave, bf16 operands gathered straight from NHWC activations
// (8 consecutive channels = one 16-byte load per lane) and from [cout][taps cin]
// weights, float32 accumulation.  Lane l of a wave supplies row (l % 32) of A and
// column (l % 32) of B for the 8 reduction indices 8 (l / 32) .. + 7 of each step of
// 16, and holds C[8 (i / 4) + 4 (l / 32) + i % 4][l % 32] in accumulator i (the
// operand layout of this instruction).  Everything else is element-parallel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "common.hpp"
#include "unet_ops.hpp"

namespace die {
namespace nn {
namespace {

constexpr int NT = 256;

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float floatx16;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// round to nearest even (finite inputs)
__device__ __forceinline__ bf16raw f2bf(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (bf16raw)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16raw h) { return __uint_as_float((uint32_t)h << 16); }

__device__ __forceinline__ bf16x8 as_bf16x8(u32x4 v) { return __builtin_bit_cast(bf16x8, v); }

// pack 8 bf16 values (low index in the low half of the first word)
__device__ __forceinline__ u32x4 pack8(const bf16raw (&h)[8]) {
  u32x4 v;
  v.x = (uint32_t)h[0] | ((uint32_t)h[1] << 16);
  v.y = (uint32_t)h[2] | ((uint32_t)h[3] << 16);
  v.z = (uint32_t)h[4] | ((uint32_t)h[5] << 16);
  v.w = (uint32_t)h[6] | ((uint32_t)h[7] << 16);
  return v;
}

inline unsigned blocks_for(size_t n, size_t per) { return (unsigned)std::min<size_t>((n + per - 1) / per, 65535u * 8); }

// ------------------------------------------------------------------ convolution (forward / backward data)
template <bool FLIP, bool RELU, int OUT>
__global__ void __launch_bounds__(NT)
k_conv(const bf16raw* __restrict__ X, int B, int H, int W, int cin, int taps, const bf16raw* __restrict__ Wm,
       const float* __restrict__ bias, void* __restrict__ out, int cout) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 5;
  const long M = (long)B * H * W;
  const int K = taps * cin, N = cout;
  const long m0 = ((long)blockIdx.x * 4 + wave) * 32;
  if (m0 >= M) return;  // wave-uniform; the kernel has no block barrier
  const int n0 = blockIdx.y * 32;
  const long m = m0 + (lane & 31);
  const bool mvalid = m < M;
  int px = 0, py = 0;
  long pb = 0;
  if (mvalid) {
    px = (int)(m % W);
    const long q = m / W;
    py = (int)(q % H);
    pb = q / H;
  }
  const int n = n0 + (lane & 31);
  const bool nvalid = n < N;
  const bf16raw* wrow = Wm + (size_t)(nvalid ? n : 0) * K;
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (int k0 = 0; k0 < K; k0 += 16) {
    const int k = k0 + 8 * g;
    u32x4 av = {0u, 0u, 0u, 0u}, bv = {0u, 0u, 0u, 0u};
    if (k < K) {
      const int t = k / cin, ci = k - t * cin;
      int dy = 0, dx = 0;
      if (taps == 9) {
        dy = t / 3 - 1;
        dx = t % 3 - 1;
        if (FLIP) {
          dy = -dy;
          dx = -dx;
        }
      }
      const int yy = py + dy, xx = px + dx;
      if (mvalid && yy >= 0 && yy < H && xx >= 0 && xx < W)
        av = *reinterpret_cast<const u32x4*>(X + (((size_t)pb * H + yy) * W + xx) * cin + ci);
      if (nvalid) bv = *reinterpret_cast<const u32x4*>(wrow + k);
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv), acc, 0, 0, 0);
  }
  if (!nvalid) return;
  const float bn = bias ? bias[n] : 0.f;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const long mm = m0 + (i / 4) * 8 + g * 4 + (i % 4);
    if (mm < M) {
      float v = acc[i] + bn;
      if (RELU) v = fmaxf(v, 0.f);
      const size_t o = (size_t)mm * N + n;
      if (OUT == kOutBf16) static_cast<bf16raw*>(out)[o] = f2bf(v);
      else if (OUT == kOutF32) static_cast<float*>(out)[o] = v;
      else static_cast<float*>(out)[o] += v;
    }
  }
}

// 3x3 convolutions with their operands staged in LDS (W % 32 == 0, cin % 16 == 0, cout a multiple
// of 32 NCO).  Block: 4 image rows x 32 pixels x 32 NCO output channels, wave w on row w.  For each
// chunk of 16 input channels the input patch (6 rows x 34 pixels with the halo, zero outside the
// image) and the weights of the chunk (9 taps x 32 NCO channels x 16) are staged once; every tap's
// A operand is then a 16-byte LDS read of the patch shifted by that tap (so each staged input
// value serves nine MFMAs of the wave and the rows above and below), and each B operand is shared
// by the four waves.  The next chunk's global loads are in flight while the current one is
// multiplied.
constexpr int kCvRows = 4, kCvPx = 32, kCvCi = 16;
constexpr int kCvPr = kCvRows + 2, kCvPq = kCvPx + 2;  // patch rows and pixels with the halo

template <bool FLIP, bool RELU, int OUT, int NCO>
__global__ void __launch_bounds__(NT)
k_conv_lds(const bf16raw* __restrict__ X, int H, int W, int cin, const bf16raw* __restrict__ Wm,
           const float* __restrict__ bias, void* __restrict__ out, int cout) {
  constexpr int NB = 32 * NCO;
  constexpr int AITEMS = kCvPr * kCvPq * 2;   // 16-byte loads of the patch (two per pixel)
  constexpr int BITEMS = 9 * NB * 2;          // 16-byte loads of the chunk's weights
  constexpr int IA = (AITEMS + NT - 1) / NT, IB = (BITEMS + NT - 1) / NT;
  __shared__ __attribute__((aligned(16))) bf16raw sA[kCvPr * kCvPq * kCvCi];
  __shared__ __attribute__((aligned(16))) bf16raw sB[9 * NB * kCvCi];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5, r32 = lane & 31;
  const int tiles_x = W / kCvPx, tiles_y = (H + kCvRows - 1) / kCvRows;
  const int tx = blockIdx.x % tiles_x, rest = blockIdx.x / tiles_x;
  const int ty = rest % tiles_y, b = rest / tiles_y;
  const int x0 = tx * kCvPx, y0 = ty * kCvRows, n0 = blockIdx.y * NB;
  const int K = 9 * cin;
  u32x4 ra[IA], rb[IB];
  auto load = [&](int c0) {
#pragma unroll
    for (int k = 0; k < IA; ++k) {
      const int i = tid + k * NT;
      const int half = i & 1, pq = (i >> 1) % kCvPq, pr = (i >> 1) / kCvPq;
      const int yy = y0 - 1 + pr, xx = x0 - 1 + pq;
      ra[k] = u32x4{0u, 0u, 0u, 0u};
      if (i < AITEMS && yy >= 0 && yy < H && xx >= 0 && xx < W)
        ra[k] = *reinterpret_cast<const u32x4*>(X + (((size_t)b * H + yy) * W + xx) * cin + c0 + 8 * half);
    }
#pragma unroll
    for (int k = 0; k < IB; ++k) {
      const int i = tid + k * NT;
      const int half = i & 1, nn = (i >> 1) % NB, t = (i >> 1) / NB;
      rb[k] = u32x4{0u, 0u, 0u, 0u};
      if (i < BITEMS) rb[k] = *reinterpret_cast<const u32x4*>(Wm + (size_t)(n0 + nn) * K + t * cin + c0 + 8 * half);
    }
  };
  auto put = [&]() {
#pragma unroll
    for (int k = 0; k < IA; ++k) {
      const int i = tid + k * NT;
      if (i < AITEMS) *reinterpret_cast<u32x4*>(&sA[(i >> 1) * kCvCi + 8 * (i & 1)]) = ra[k];
    }
#pragma unroll
    for (int k = 0; k < IB; ++k) {
      const int i = tid + k * NT;
      if (i < BITEMS) *reinterpret_cast<u32x4*>(&sB[(i >> 1) * kCvCi + 8 * (i & 1)]) = rb[k];
    }
  };
  floatx16 acc[NCO];
#pragma unroll
  for (int c = 0; c < NCO; ++c)
#pragma unroll
    for (int i = 0; i < 16; ++i) acc[c][i] = 0.f;
  load(0);
  for (int c0 = 0; c0 < cin; c0 += kCvCi) {
    lds_sync();  // the previous chunk's LDS reads are done
    put();
    lds_sync();
    if (c0 + kCvCi < cin) load(c0 + kCvCi);
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      int dy = t / 3 - 1, dx = t % 3 - 1;
      if (FLIP) {
        dy = -dy;
        dx = -dx;
      }
      const u32x4 av = *reinterpret_cast<const u32x4*>(
          &sA[((wave + 1 + dy) * kCvPq + r32 + 1 + dx) * kCvCi + 8 * g]);
#pragma unroll
      for (int c = 0; c < NCO; ++c) {
        const u32x4 bv = *reinterpret_cast<const u32x4*>(&sB[(t * NB + 32 * c + r32) * kCvCi + 8 * g]);
        acc[c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(av), as_bf16x8(bv), acc[c], 0, 0, 0);
      }
    }
  }
  const int y = y0 + wave;
  if (y >= H) return;
#pragma unroll
  for (int c = 0; c < NCO; ++c) {
    const int n = n0 + 32 * c + r32;
    const float bn = bias ? bias[n] : 0.f;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int px = x0 + (i / 4) * 8 + g * 4 + (i % 4);
      float v = acc[c][i] + bn;
      if (RELU) v = fmaxf(v, 0.f);
      const size_t o = (((size_t)b * H + y) * W + px) * cout + n;
      if (OUT == kOutBf16) static_cast<bf16raw*>(out)[o] = f2bf(v);
      else if (OUT == kOutF32) static_cast<float*>(out)[o] = v;
      else static_cast<float*>(out)[o] += v;
    }
  }
}

// ------------------------------------------------------------------ weight gradient
// Tile: rows co0..co0+31 (A = dZ^T), columns n0..n0+31 of (t, ci) (B = shifted X), one
// split of the pixels per blockIdx.z, 8 consecutive pixels of one image row per lane
// group (W % 8 == 0, split starts are multiples of 16).
__global__ void __launch_bounds__(NT)
k_conv_wgrad(const bf16raw* __restrict__ dZ, int ldz, const bf16raw* __restrict__ X, int B, int H, int W, int cin,
             int taps, int cout, long pps, float* __restrict__ part) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 5;
  const int N = taps * cin;
  const int n0 = (blockIdx.x * 4 + wave) * 32;
  if (n0 >= N) return;  // wave-uniform
  const int co0 = blockIdx.y * 32;
  const long M = (long)B * H * W;
  const long pbeg = (long)blockIdx.z * pps, pend = std::min(M, pbeg + pps);
  const int co = co0 + (lane & 31), n = n0 + (lane & 31);
  const bool covalid = co < cout, nvalid = n < N;
  const int t = nvalid ? n / cin : 0, ci = nvalid ? n - t * cin : 0;
  const int dy = taps == 9 ? t / 3 - 1 : 0, dx = taps == 9 ? t % 3 - 1 : 0;
  floatx16 acc;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = 0.f;
  for (long p0 = pbeg; p0 < pend; p0 += 16) {
    const long pg = p0 + 8 * g;  // first of this lane group's 8 pixels (same image row)
    bf16raw ha[8], hb[8];
#pragma unroll
    for (int i = 0; i < 8; ++i) ha[i] = hb[i] = 0;
    if (pg < pend) {
      const int x0 = (int)(pg % W);
      const long q = pg / W;
      const int y = (int)(q % H);
      const long b = q / H;
      const int yy = y + dy;
      const bool yin = yy >= 0 && yy < H;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        if (pg + i < pend) {
          if (covalid) ha[i] = dZ[(size_t)(pg + i) * ldz + co];
          const int xx = x0 + i + dx;
          if (nvalid && yin && xx >= 0 && xx < W) hb[i] = X[(((size_t)b * H + yy) * W + xx) * cin + ci];
        }
      }
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(pack8(ha)), as_bf16x8(pack8(hb)), acc, 0, 0, 0);
  }
  if (!nvalid) return;
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    const int r = co0 + (i / 4) * 8 + g * 4 + (i % 4);
    if (r < cout) part[((size_t)blockIdx.z * cout + r) * N + n] = acc[i];
  }
}

// Weight and bias gradients with the pixel chunks staged in LDS (W % 32 == 0).
// Block: 64 output channels (two 32-row tiles) x 32 input channels x every tap over one split of
// the pixels, one wave per tap.  Each chunk of 32 consecutive pixels (one image row) is stored
// transposed: dZ as [co][pixel] and, for each tap, the input shifted by that tap as [ci][pixel],
// so that each MFMA operand (8 consecutive pixels of one channel) is one 16-byte LDS read.  The
// next chunk's global loads are in flight while the current one is multiplied.  Blocks of the
// first input-channel tile also sum dZ over the pixels (the bias gradient).
constexpr int kWgPx = 32;         // pixels per chunk
constexpr int kWgLd = kWgPx + 8;  // LDS row stride in bf16 (80 bytes: the 16-byte reads of 8 rows hit distinct banks)

template <int NTAPS>
__global__ void __launch_bounds__(64 * NTAPS)
k_conv_wgrad_lds(const bf16raw* __restrict__ dZ, int ldz, const bf16raw* __restrict__ X, int H, int W, int cin,
                 int cout, long M, long pps, float* __restrict__ part, float* __restrict__ bpart) {
  constexpr int NTH = 64 * NTAPS;
  constexpr int NR = NTAPS == 9 ? 3 : 1;       // input rows per chunk (dy = -1, 0, 1)
  constexpr int NQ = NTAPS == 9 ? 34 : 32;     // input pixels per row (dx halo)
  constexpr int QOFF = NTAPS == 9 ? 1 : 0;
  constexpr int ZITEMS = 64 / 8 * kWgPx;       // 16-byte loads of the dZ chunk
  constexpr int XITEMS = NR * NQ * 4;          // 16-byte loads of the input rows (4 groups of 8 channels)
  constexpr int IZ = (ZITEMS + NTH - 1) / NTH, IX = (XITEMS + NTH - 1) / NTH;
  __shared__ __attribute__((aligned(16))) bf16raw sZ[2][64 * kWgLd];
  __shared__ __attribute__((aligned(16))) bf16raw sX[2][NTAPS * 32 * kWgLd];
  __shared__ float sB[4][64];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, g = lane >> 5, r32 = lane & 31;
  const int c0 = blockIdx.x * 32, co0 = blockIdx.y * 64;
  const long pbeg = (long)blockIdx.z * pps, pend = min(M, pbeg + pps);
  const bool do_bias = bpart != nullptr && blockIdx.x == 0;
  const long HW = (long)H * W;

  u32x4 rz[IZ], rx[IX];
  auto load = [&](long p0) {
    const long bimg = p0 / HW;
    const int y = (int)((p0 / W) % H), x0 = (int)(p0 % W);
#pragma unroll
    for (int k = 0; k < IZ; ++k) {
      const int i = tid + k * NTH;
      const int px = i & (kWgPx - 1), co = co0 + 8 * (i / kWgPx);
      rz[k] = u32x4{0u, 0u, 0u, 0u};
      if (i < ZITEMS && co < cout) rz[k] = *reinterpret_cast<const u32x4*>(dZ + (size_t)(p0 + px) * ldz + co);
    }
#pragma unroll
    for (int k = 0; k < IX; ++k) {
      const int i = tid + k * NTH;
      const int grp = i & 3, rest = i >> 2, qi = rest % NQ, r = rest / NQ;
      const int yy = y + r - (NR == 3 ? 1 : 0), xx = x0 + qi - QOFF, ci = c0 + 8 * grp;
      rx[k] = u32x4{0u, 0u, 0u, 0u};
      if (i < XITEMS && yy >= 0 && yy < H && xx >= 0 && xx < W && ci < cin)
        rx[k] = *reinterpret_cast<const u32x4*>(X + ((size_t)bimg * HW + (size_t)yy * W + xx) * cin + ci);
    }
  };
  auto put = [&](int buf) {
#pragma unroll
    for (int k = 0; k < IZ; ++k) {
      const int i = tid + k * NTH;
      if (i >= ZITEMS) continue;
      const int px = i & (kWgPx - 1), row = 8 * (i / kWgPx);
      const uint32_t w4[4] = {rz[k].x, rz[k].y, rz[k].z, rz[k].w};
#pragma unroll
      for (int e = 0; e < 8; ++e) sZ[buf][(row + e) * kWgLd + px] = (bf16raw)(w4[e >> 1] >> (16 * (e & 1)));
    }
#pragma unroll
    for (int k = 0; k < IX; ++k) {
      const int i = tid + k * NTH;
      if (i >= XITEMS) continue;
      const int grp = i & 3, rest = i >> 2, qi = rest % NQ, r = rest / NQ, q = qi - QOFF;
      const uint32_t w4[4] = {rx[k].x, rx[k].y, rx[k].z, rx[k].w};
#pragma unroll
      for (int dx = -QOFF; dx <= QOFF; ++dx) {
        const int j = q - dx;  // position of input pixel q in the copy shifted by dx
        if (j < 0 || j >= kWgPx) continue;
        const int t = NTAPS == 9 ? r * 3 + dx + 1 : 0;
#pragma unroll
        for (int e = 0; e < 8; ++e)
          sX[buf][(t * 32 + 8 * grp + e) * kWgLd + j] = (bf16raw)(w4[e >> 1] >> (16 * (e & 1)));
      }
    }
  };

  floatx16 acc0, acc1;
#pragma unroll
  for (int i = 0; i < 16; ++i) acc0[i] = acc1[i] = 0.f;
  float bsum = 0.f;
  if (pbeg < pend) {
    load(pbeg);
    put(0);
  }
  lds_sync();
  int buf = 0;
  for (long p0 = pbeg; p0 < pend; p0 += kWgPx, buf ^= 1) {
    const bool more = p0 + kWgPx < pend;
    if (more) load(p0 + kWgPx);
#pragma unroll
    for (int s = 0; s < kWgPx / 16; ++s) {
      const int k0 = 16 * s + 8 * g;
      const u32x4 a0 = *reinterpret_cast<const u32x4*>(&sZ[buf][r32 * kWgLd + k0]);
      const u32x4 a1 = *reinterpret_cast<const u32x4*>(&sZ[buf][(32 + r32) * kWgLd + k0]);
      const u32x4 bv = *reinterpret_cast<const u32x4*>(&sX[buf][(wave * 32 + r32) * kWgLd + k0]);
      acc0 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a0), as_bf16x8(bv), acc0, 0, 0, 0);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(as_bf16x8(a1), as_bf16x8(bv), acc1, 0, 0, 0);
    }
    if (do_bias) {
      // row tid % 64, pixels 8 (tid / 64) .. + 7 (threads beyond 256 idle; 64-thread blocks loop)
      for (int qq = tid >> 6; qq < 4; qq += NTH / 64) {
        const u32x4 v = *reinterpret_cast<const u32x4*>(&sZ[buf][(tid & 63) * kWgLd + 8 * qq]);
        const uint32_t w4[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int e = 0; e < 8; ++e) bsum += bf2f((bf16raw)(w4[e >> 1] >> (16 * (e & 1))));
      }
    }
    if (more) put(buf ^ 1);
    lds_sync();
  }
  const int N = NTAPS * cin, col = c0 + r32;
  if (col < cin) {
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int row = co0 + (i / 4) * 8 + g * 4 + (i % 4);
      if (row < cout) part[((size_t)blockIdx.z * cout + row) * N + wave * cin + col] = acc0[i];
      if (row + 32 < cout) part[((size_t)blockIdx.z * cout + row + 32) * N + wave * cin + col] = acc1[i];
    }
  }
  if (do_bias) {
    if (tid < 256) sB[tid >> 6][tid & 63] = bsum;
    if (NTH == 64)
      for (int qq = 1; qq < 4; ++qq) sB[qq][tid] = 0.f;
    lds_sync();
    if (tid < 64 && co0 + tid < cout)
      bpart[(size_t)blockIdx.z * cout + co0 + tid] = (sB[0][tid] + sB[1][tid]) + (sB[2][tid] + sB[3][tid]);
  }
}

__global__ void __launch_bounds__(NT)
k_bias_grad(const bf16raw* __restrict__ dZ, int ldz, long npix, int cout, long pps, float* __restrict__ part) {
  const long pbeg = (long)blockIdx.x * pps, pend = std::min(npix, pbeg + pps);
  for (int c = threadIdx.x; c < cout; c += NT) {
    float s = 0.f;
    for (long p = pbeg; p < pend; ++p) s += bf2f(dZ[(size_t)p * ldz + c]);
    part[(size_t)blockIdx.x * cout + c] = s;
  }
}

// Block: 32 consecutive outputs x 8 groups of splits (group q sums splits q, q + 8, ... in
// order), then the 8 group sums in order.
constexpr int kRedJ = 32, kRedG = NT / kRedJ;
__global__ void __launch_bounds__(NT)
k_reduce_splits(const float* __restrict__ part, int nsplit, size_t count, float* __restrict__ out) {
  __shared__ float red[kRedG][kRedJ];
  const int jj = threadIdx.x % kRedJ, q = threadIdx.x / kRedJ;
  const size_t j = (size_t)blockIdx.x * kRedJ + jj;
  float s = 0.f;
  if (j < count)
    for (int k = q; k < nsplit; k += kRedG) s += part[(size_t)k * count + j];
  red[q][jj] = s;
  lds_sync();
  if (q == 0 && j < count) {
    float t = red[0][jj];
    for (int k = 1; k < kRedG; ++k) t += red[k][jj];
    out[j] = t;
  }
}

// ------------------------------------------------------------------ element-wise kernels
__global__ void __launch_bounds__(NT)
k_relu_grad(const float* __restrict__ dY, const bf16raw* __restrict__ Y, bf16raw* __restrict__ dZ, size_t count) {
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const float d = dY[j];
    dZ[j] = f2bf(Y && !(bf2f(Y[j]) > 0.f) ? 0.f : d);
  }
}

__global__ void __launch_bounds__(NT)
k_pool(const bf16raw* __restrict__ X, bf16raw* __restrict__ Y, int B, int H, int W, int C) {
  const int Ho = H / 2, Wo = W / 2;
  const size_t count = (size_t)B * Ho * Wo * C;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const int c = (int)(j % C);
    size_t q = j / C;
    const int x = (int)(q % Wo);
    q /= Wo;
    const int y = (int)(q % Ho);
    const size_t b = q / Ho;
    const size_t r0 = ((b * H + 2 * y) * W + 2 * x) * C + c, r1 = r0 + (size_t)W * C;
    const float s = (bf2f(X[r0]) + bf2f(X[r0 + C])) + (bf2f(X[r1]) + bf2f(X[r1 + C]));
    Y[j] = f2bf(0.25f * s);
  }
}

__global__ void __launch_bounds__(NT)
k_pool_grad_add(const float* __restrict__ dY, float* __restrict__ dX, int B, int H, int W, int C) {
  const size_t count = (size_t)B * H * W * C;
  const int Wo = W / 2, Ho = H / 2;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const int c = (int)(j % C);
    size_t q = j / C;
    const int x = (int)(q % W);
    q /= W;
    const int y = (int)(q % H);
    const size_t b = q / H;
    dX[j] += 0.25f * dY[((b * Ho + y / 2) * Wo + x / 2) * C + c];
  }
}

// Eight channels (16 bytes) per thread; cl and cs are multiples of 8.
__global__ void __launch_bounds__(NT)
k_upcat(const bf16raw* __restrict__ low, const bf16raw* __restrict__ skip, bf16raw* __restrict__ cat, int B, int H,
        int W, int cl, int cs) {
  const int C8 = (cl + cs) / 8, cl8 = cl / 8;
  const size_t count = (size_t)B * H * W * C8;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const int c8 = (int)(j % C8);
    const size_t pix = j / C8;
    const int x = (int)(pix % W);
    size_t q = pix / W;
    const int y = (int)(q % H);
    const size_t b = q / H;
    const bf16raw* src = c8 < cl8 ? low + ((b * (H / 2) + y / 2) * (W / 2) + x / 2) * cl + 8 * c8
                                  : skip + pix * cs + 8 * (c8 - cl8);
    reinterpret_cast<u32x4*>(cat)[j] = *reinterpret_cast<const u32x4*>(src);
  }
}

// dlow (written): each low-resolution pixel sums its 2x2 block; dskip (written): a copy.
__global__ void __launch_bounds__(NT)
k_upcat_grad(const float* __restrict__ dcat, float* __restrict__ dlow, float* __restrict__ dskip, int B, int H, int W,
             int cl, int cs) {
  const int C = cl + cs, Ho = H / 2, Wo = W / 2;
  const size_t nlow = (size_t)B * Ho * Wo * cl, nskip = (size_t)B * H * W * cs;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < nlow + nskip; j += (size_t)gridDim.x * NT) {
    if (j < nlow) {
      const int c = (int)(j % cl);
      size_t q = j / cl;
      const int x = (int)(q % Wo);
      q /= Wo;
      const int y = (int)(q % Ho);
      const size_t b = q / Ho;
      const size_t r0 = ((b * H + 2 * y) * W + 2 * x) * C + c, r1 = r0 + (size_t)W * C;
      dlow[j] = (dcat[r0] + dcat[r0 + C]) + (dcat[r1] + dcat[r1 + C]);
    } else {
      const size_t k = j - nlow;
      dskip[k] = dcat[(k / cs) * C + cl + (k % cs)];
    }
  }
}

__global__ void __launch_bounds__(NT) k_to_bf16(const float* __restrict__ x, bf16raw* __restrict__ y, size_t count) {
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) y[j] = f2bf(x[j]);
}

constexpr int kLossPer = NT * 16;

__global__ void __launch_bounds__(NT)
k_mse(const float* __restrict__ out, const float* __restrict__ t, size_t count, double* __restrict__ part,
      bf16raw* __restrict__ dZ) {
  __shared__ double red[NT];
  double s = 0.0;
  const float sc = 2.0f / (float)count;
  const size_t base = (size_t)blockIdx.x * kLossPer;
  for (int k = 0; k < kLossPer / NT; ++k) {
    const size_t j = base + (size_t)k * NT + threadIdx.x;
    if (j < count) {
      const float d = out[j] - t[j];
      s += (double)d * (double)d;
      const size_t o = (j / 4) * 8 + (j % 4);  // 8-channel rows, channels 4..7 zero
      dZ[o] = f2bf(sc * d);
      dZ[o + 4] = 0;
    }
  }
  red[threadIdx.x] = s;
  lds_sync();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    lds_sync();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(NT) k_sum_doubles(const double* __restrict__ part, int n, double* __restrict__ out) {
  __shared__ double red[NT];
  double s = 0.0;
  for (int j = threadIdx.x; j < n; j += NT) s += part[j];
  red[threadIdx.x] = s;
  lds_sync();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    lds_sync();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}

__global__ void __launch_bounds__(NT)
k_adam(float* __restrict__ w, const float* __restrict__ g, float* __restrict__ m, float* __restrict__ v,
       bf16raw* __restrict__ wbf, size_t n, float lr, float beta1, float beta2, float eps, float c1, float c2) {
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < n; j += (size_t)gridDim.x * NT) {
    const float gj = g[j];
    const float mj = beta1 * m[j] + (1.0f - beta1) * gj;
    const float vj = beta2 * v[j] + (1.0f - beta2) * gj * gj;
    m[j] = mj;
    v[j] = vj;
    const float wj = w[j] - lr * (mj * c1) / (sqrtf(vj * c2) + eps);
    w[j] = wj;
    wbf[j] = f2bf(wj);
  }
}

__global__ void __launch_bounds__(NT) k_to_bf16_params(const float* __restrict__ w, bf16raw* __restrict__ wbf, size_t n) {
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < n; j += (size_t)gridDim.x * NT) wbf[j] = f2bf(w[j]);
}

__global__ void __launch_bounds__(NT)
k_wbd(const bf16raw* __restrict__ Wf, bf16raw* __restrict__ Wbd, int cout, int cpad, int taps, int cin) {
  const size_t count = (size_t)cpad * taps * cin;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    // j indexes Wbd[ci][t cpad + co]; rows co >= cout are zero
    const int co = (int)(j % cpad);
    size_t q = j / cpad;
    const int t = (int)(q % taps);
    const int ci = (int)(q / taps);
    Wbd[j] = co < cout ? Wf[((size_t)co * taps + t) * cin + ci] : (bf16raw)0;
  }
}

__global__ void __launch_bounds__(NT)
k_pack_inputs(const double2* __restrict__ eps, double shift, int rpo, int r0, const double2* __restrict__ e_in,
              float* __restrict__ x, int batch, int ny, int nx) {
  const size_t ncell = (size_t)ny * nx, count = (size_t)batch * ncell;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const size_t r = j / ncell, c = j % ncell;
    const size_t obj = rpo > 0 ? (r0 + r) / rpo : 0;
    const double2 ev = eps[obj * ncell + c];
    const double2 e1 = e_in[(2 * r) * ncell + c], e2 = e_in[(2 * r + 1) * ncell + c];
    float* o = x + j * 8;
    o[0] = (float)(ev.x - shift);
    o[1] = (float)ev.y;
    o[2] = (float)e1.x;
    o[3] = (float)e1.y;
    o[4] = (float)e2.x;
    o[5] = (float)e2.y;
    o[6] = 0.f;
    o[7] = 0.f;
  }
}

__global__ void __launch_bounds__(NT)
k_pack_targets(const double2* __restrict__ e_tot, const double2* __restrict__ e_in, float* __restrict__ t, int batch,
               int ny, int nx) {
  const size_t ncell = (size_t)ny * nx, count = (size_t)batch * ncell;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const size_t r = j / ncell, c = j % ncell;
    const size_t i1 = (2 * r) * ncell + c, i2 = (2 * r + 1) * ncell + c;
    float* o = t + j * 4;
    o[0] = (float)(e_tot[i1].x - e_in[i1].x);
    o[1] = (float)(e_tot[i1].y - e_in[i1].y);
    o[2] = (float)(e_tot[i2].x - e_in[i2].x);
    o[3] = (float)(e_tot[i2].y - e_in[i2].y);
  }
}

__global__ void __launch_bounds__(NT)
k_unpack_guess(const double2* __restrict__ e_in, const float* __restrict__ y, double2* __restrict__ x0, int batch,
               int ny, int nx) {
  const size_t ncell = (size_t)ny * nx, count = (size_t)batch * ncell;
  for (size_t j = (size_t)blockIdx.x * NT + threadIdx.x; j < count; j += (size_t)gridDim.x * NT) {
    const size_t r = j / ncell, c = j % ncell;
    const size_t i1 = (2 * r) * ncell + c, i2 = (2 * r + 1) * ncell + c;
    const float* o = y + j * 4;
    x0[i1] = make_double2(e_in[i1].x + (double)o[0], e_in[i1].y + (double)o[1]);
    x0[i2] = make_double2(e_in[i2].x + (double)o[2], e_in[i2].y + (double)o[3]);
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_conv(const bf16raw* X, int B, int H, int W, int cin, int taps, bool flip, const bf16raw* Wm,
                       const float* bias, bool relu, void* out, int cout, ConvOut mode, hipStream_t st) {
  if (cin % 8 || (taps != 1 && taps != 9) || B < 1 || H < 1 || W < 1 || cout < 1) return hipErrorInvalidValue;
  if (taps == 9 && W % kCvPx == 0 && cin % kCvCi == 0 && cout % 32 == 0) {
    const int nco = cout % 64 == 0 ? 2 : 1;
    const long tiles = (long)B * ((H + kCvRows - 1) / kCvRows) * (W / kCvPx);
    dim3 g((unsigned)tiles, (unsigned)(cout / (32 * nco)));
#define DIE_CONV_LDS(F, R, O)                                                                                  \
  do {                                                                                                         \
    if (nco == 2) hipLaunchKernelGGL((k_conv_lds<F, R, O, 2>), g, dim3(NT), 0, st, X, H, W, cin, Wm, bias, out, cout); \
    else hipLaunchKernelGGL((k_conv_lds<F, R, O, 1>), g, dim3(NT), 0, st, X, H, W, cin, Wm, bias, out, cout);    \
  } while (0)
    if (!flip && relu && mode == kOutBf16) DIE_CONV_LDS(false, true, kOutBf16);
    else if (!flip && !relu && mode == kOutF32) DIE_CONV_LDS(false, false, kOutF32);
    else if (flip && !relu && mode == kOutF32) DIE_CONV_LDS(true, false, kOutF32);
    else if (flip && !relu && mode == kOutF32Add) DIE_CONV_LDS(true, false, kOutF32Add);
    else return hipErrorInvalidValue;
#undef DIE_CONV_LDS
    return hipGetLastError();
  }
  const long M = (long)B * H * W;
  dim3 grid((unsigned)((M + 127) / 128), (unsigned)((cout + 31) / 32));
#define DIE_CONV(F, R, O) \
  hipLaunchKernelGGL((k_conv<F, R, O>), grid, dim3(NT), 0, st, X, B, H, W, cin, taps, Wm, bias, out, cout)
  if (!flip && relu && mode == kOutBf16) DIE_CONV(false, true, kOutBf16);
  else if (!flip && !relu && mode == kOutF32) DIE_CONV(false, false, kOutF32);
  else if (flip && !relu && mode == kOutF32) DIE_CONV(true, false, kOutF32);
  else if (flip && !relu && mode == kOutF32Add) DIE_CONV(true, false, kOutF32Add);
  else return hipErrorInvalidValue;
#undef DIE_CONV
  return hipGetLastError();
}

// at most this many (tile x split) blocks per weight-gradient launch
constexpr long kWgradBlocks = 2048;

static void wgrad_shape(long M, int cout, int N, long* pps, int* nsplit) {
  const long tiles = (long)((cout + 31) / 32) * ((N + 31) / 32);
  long ns = std::max<long>(1, kWgradBlocks / std::max<long>(tiles, 1));
  long per = (M + ns - 1) / ns;
  per = (per + 15) / 16 * 16;
  *pps = std::max<long>(per, 16);
  *nsplit = (int)((M + *pps - 1) / *pps);
}

// Splits of the LDS-staged gradient kernel: about 1024 blocks, at most 256 splits and at most
// kWgLdsPartFloats partial values (one split per 32-pixel chunk at most).
constexpr long kWgLdsPartFloats = 8l << 20;
static long wgrad_lds_splits(int cout, int taps, int cin) {
  const long tiles = (long)((cin + 31) / 32) * ((cout + 63) / 64);
  long s = std::max<long>(1, 1024 / tiles);
  s = std::min<long>(s, 256);
  return std::max<long>(1, std::min<long>(s, kWgLdsPartFloats / ((long)cout * taps * cin)));
}

size_t conv_wgrad_max_floats(int cout, int taps, int cin) {
  const int N = taps * cin;
  const long tiles = (long)((cout + 31) / 32) * ((N + 31) / 32);
  const long ns = std::max<long>(1, kWgradBlocks / std::max<long>(tiles, 1));
  return (size_t)std::max(ns, wgrad_lds_splits(cout, taps, cin)) * cout * N;
}

bool conv_wgrad_bias_fused(int W, int ldz, int cout) { return W % kWgPx == 0 && ldz % 8 == 0 && ldz >= cout; }

hipError_t launch_conv_wgrad_bias(const bf16raw* dZ, int ldz, const bf16raw* X, int B, int H, int W, int cin,
                                  int taps, int cout, float* part, float* bpart, int* nsplit, hipStream_t st) {
  if (!conv_wgrad_bias_fused(W, ldz, cout) || (taps != 1 && taps != 9) || cin < 8 || cin % 8 || cout < 1 || B < 1 ||
      H < 1)
    return hipErrorInvalidValue;
  const long M = (long)B * H * W;
  const long chunks = M / kWgPx;
  const long s = std::min(wgrad_lds_splits(cout, taps, cin), chunks);
  const long pps = (chunks + s - 1) / s * kWgPx;
  *nsplit = (int)((M + pps - 1) / pps);
  dim3 grid((unsigned)((cin + 31) / 32), (unsigned)((cout + 63) / 64), (unsigned)*nsplit);
  if (taps == 9)
    hipLaunchKernelGGL(k_conv_wgrad_lds<9>, grid, dim3(64 * 9), 0, st, dZ, ldz, X, H, W, cin, cout, M, pps, part,
                       bpart);
  else
    hipLaunchKernelGGL(k_conv_wgrad_lds<1>, grid, dim3(64), 0, st, dZ, ldz, X, H, W, cin, cout, M, pps, part, bpart);
  return hipGetLastError();
}

hipError_t launch_conv_wgrad(const bf16raw* dZ, int ldz, const bf16raw* X, int B, int H, int W, int cin, int taps,
                             int cout, float* part, int* nsplit, hipStream_t st) {
  if (W % 8 || (taps != 1 && taps != 9) || cin < 1 || cout < 1 || ldz < cout) return hipErrorInvalidValue;
  const int N = taps * cin;
  long pps;
  wgrad_shape((long)B * H * W, cout, N, &pps, nsplit);
  dim3 grid((unsigned)((N + 127) / 128), (unsigned)((cout + 31) / 32), (unsigned)*nsplit);
  hipLaunchKernelGGL(k_conv_wgrad, grid, dim3(NT), 0, st, dZ, ldz, X, B, H, W, cin, taps, cout, pps, part);
  return hipGetLastError();
}

hipError_t launch_bias_grad(const bf16raw* dZ, int ldz, long npix, int cout, float* part, int nsplit, hipStream_t st) {
  if (nsplit < 1 || ldz < cout) return hipErrorInvalidValue;
  const long pps = (npix + nsplit - 1) / nsplit;
  hipLaunchKernelGGL(k_bias_grad, dim3((unsigned)nsplit), dim3(NT), 0, st, dZ, ldz, npix, cout, pps, part);
  return hipGetLastError();
}

hipError_t launch_reduce_splits(const float* part, int nsplit, size_t count, float* out, hipStream_t st) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_reduce_splits, dim3((unsigned)((count + kRedJ - 1) / kRedJ)), dim3(NT), 0, st, part, nsplit,
                     count, out);
  return hipGetLastError();
}

hipError_t launch_relu_grad(const float* dY, const bf16raw* Y, bf16raw* dZ, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_relu_grad, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, dY, Y, dZ, count);
  return hipGetLastError();
}

hipError_t launch_pool(const bf16raw* X, bf16raw* Y, int B, int H, int W, int C, hipStream_t st) {
  if (H % 2 || W % 2) return hipErrorInvalidValue;
  const size_t count = (size_t)B * (H / 2) * (W / 2) * C;
  hipLaunchKernelGGL(k_pool, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, X, Y, B, H, W, C);
  return hipGetLastError();
}

hipError_t launch_pool_grad_add(const float* dY, float* dX, int B, int H, int W, int C, hipStream_t st) {
  if (H % 2 || W % 2) return hipErrorInvalidValue;
  const size_t count = (size_t)B * H * W * C;
  hipLaunchKernelGGL(k_pool_grad_add, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, dY, dX, B, H, W, C);
  return hipGetLastError();
}

hipError_t launch_upcat(const bf16raw* low, const bf16raw* skip, bf16raw* cat, int B, int H, int W, int cl, int cs,
                        hipStream_t st) {
  if (H % 2 || W % 2 || cl % 8 || cs % 8) return hipErrorInvalidValue;
  const size_t count = (size_t)B * H * W * ((cl + cs) / 8);
  hipLaunchKernelGGL(k_upcat, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, low, skip, cat, B, H, W, cl, cs);
  return hipGetLastError();
}

hipError_t launch_upcat_grad(const float* dcat, float* dlow, float* dskip, int B, int H, int W, int cl, int cs,
                             hipStream_t st) {
  if (H % 2 || W % 2) return hipErrorInvalidValue;
  const size_t count = (size_t)B * (H / 2) * (W / 2) * cl + (size_t)B * H * W * cs;
  hipLaunchKernelGGL(k_upcat_grad, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, dcat, dlow, dskip, B, H, W, cl,
                     cs);
  return hipGetLastError();
}

hipError_t launch_to_bf16(const float* x, bf16raw* y, size_t count, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, x, y, count);
  return hipGetLastError();
}

int loss_blocks(size_t count) { return (int)((count + kLossPer - 1) / kLossPer); }

hipError_t launch_mse(const float* out, const float* t, size_t count, double* loss_part, bf16raw* dZ,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_mse, dim3((unsigned)loss_blocks(count)), dim3(NT), 0, st, out, t, count, loss_part, dZ);
  return hipGetLastError();
}

hipError_t launch_sum_doubles(const double* part, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_sum_doubles, dim3(1), dim3(NT), 0, st, part, n, out);
  return hipGetLastError();
}

hipError_t launch_adam(float* w, const float* g, float* m, float* v, bf16raw* wbf, size_t n, float lr, float beta1,
                       float beta2, float eps, float c1, float c2, hipStream_t st) {
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, st, w, g, m, v, wbf, n, lr, beta1, beta2, eps,
                     c1, c2);
  return hipGetLastError();
}

hipError_t launch_to_bf16_params(const float* w, bf16raw* wbf, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_to_bf16_params, dim3(blocks_for(n, NT * 4)), dim3(NT), 0, st, w, wbf, n);
  return hipGetLastError();
}

hipError_t launch_wbd(const bf16raw* Wf, bf16raw* Wbd, int cout, int cpad, int taps, int cin, hipStream_t st) {
  if (cpad < cout) return hipErrorInvalidValue;
  const size_t count = (size_t)cpad * taps * cin;
  hipLaunchKernelGGL(k_wbd, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, Wf, Wbd, cout, cpad, taps, cin);
  return hipGetLastError();
}

hipError_t launch_pack_inputs(const double2* eps, double shift, int rpo, int r0, const double2* e_in, float* x,
                              int batch, int ny, int nx, hipStream_t st) {
  const size_t count = (size_t)batch * ny * nx;
  hipLaunchKernelGGL(k_pack_inputs, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, eps, shift, rpo, r0, e_in, x,
                     batch, ny, nx);
  return hipGetLastError();
}

hipError_t launch_pack_targets(const double2* e_tot, const double2* e_in, float* t, int batch, int ny, int nx,
                               hipStream_t st) {
  const size_t count = (size_t)batch * ny * nx;
  hipLaunchKernelGGL(k_pack_targets, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, e_tot, e_in, t, batch, ny, nx);
  return hipGetLastError();
}

hipError_t launch_unpack_guess(const double2* e_in, const float* y, double2* x0, int batch, int ny, int nx,
                               hipStream_t st) {
  const size_t count = (size_t)batch * ny * nx;
  hipLaunchKernelGGL(k_unpack_guess, dim3(blocks_for(count, NT * 4)), dim3(NT), 0, st, e_in, y, x0, batch, ny, nx);
  return hipGetLastError();
}

}  // namespace nn
}  // namespace die
