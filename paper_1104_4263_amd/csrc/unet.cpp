// Host runtime of the learned warm start: the U-Net of include/die_te_learn.h, its
// forward and backward passes, Adam, and the guess builder used by die_te_warm_start.
// Every numerical step runs in kernels_unet.hip; this file owns the buffers and the
// order of the launches.
#include "die_te_learn.h"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "host.hpp"
#include "unet_internal.hpp"
#include "unet_ops.hpp"

using die_host::DBuf;
using die_host::fail;
using namespace die::nn;

namespace {

struct Layer {
  int cin, cout, taps, cpad;  // cpad: cout rounded up to a multiple of 8 (gradient rows)
  size_t woff, boff;
  DBuf wbd;  // bf16 [cin][taps cpad], backward-data weights
};

struct Level {
  int H, W, w;
  DBuf encA, encB, pool, cat, decA, decB;           // bf16 activations
  DBuf gEncA, gEncB, gPool, gCat, gDecA, gDecB;     // float32 gradients
};

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double uniform01(uint64_t& s) { return ((double)(splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0); }

}  // namespace

struct die_te_unet {
  int dev = 0, L = 0, C = 0, H = 0, W = 0, maxB = 0;
  size_t np = 0;
  long long step = 0;
  std::vector<Layer> layers;
  std::vector<Level> lv;
  DBuf master, grad, m, v, wbf;  // parameters (float32, bf16 copy)
  DBuf xin, out, dz, wpart, bpart, lpart, loss;
  DBuf xf, yf;  // staging for guesses
};

namespace {

int layer_index(const die_te_unet* n, bool enc, int l, bool second) {
  if (enc) return 2 * l + (second ? 1 : 0);
  return 2 * n->L + 2 * (n->L - 2 - l) + (second ? 1 : 0);
}

int refresh_bf16(die_te_unet* n, hipStream_t st) {
  DIE_HIP(launch_to_bf16_params(n->master.as<float>(), n->wbf.as<bf16raw>(), n->np, st));
  for (auto& ly : n->layers)
    DIE_HIP(launch_wbd(n->wbf.as<bf16raw>() + ly.woff, ly.wbd.as<bf16raw>(), ly.cout, ly.cpad, ly.taps, ly.cin, st));
  return DIE_OK;
}

int forward(die_te_unet* n, const float* x, int B, hipStream_t st) {
  DIE_HIP(launch_to_bf16(x, n->xin.as<bf16raw>(), (size_t)B * n->H * n->W * 8, st));
  const bf16raw* wbf = n->wbf.as<bf16raw>();
  const float* prm = n->master.as<float>();
  const bf16raw* in = n->xin.as<bf16raw>();
  int cin = 8;
  for (int l = 0; l < n->L; ++l) {
    Level& v = n->lv[l];
    const Layer& a = n->layers[layer_index(n, true, l, false)];
    const Layer& b = n->layers[layer_index(n, true, l, true)];
    DIE_HIP(launch_conv(in, B, v.H, v.W, cin, 9, false, wbf + a.woff, prm + a.boff, true, v.encA.p, v.w, kOutBf16, st));
    DIE_HIP(launch_conv(v.encA.as<bf16raw>(), B, v.H, v.W, v.w, 9, false, wbf + b.woff, prm + b.boff, true, v.encB.p,
                        v.w, kOutBf16, st));
    if (l < n->L - 1) {
      DIE_HIP(launch_pool(v.encB.as<bf16raw>(), v.pool.as<bf16raw>(), B, v.H, v.W, v.w, st));
      in = v.pool.as<bf16raw>();
      cin = v.w;
    }
  }
  const bf16raw* h = n->lv[n->L - 1].encB.as<bf16raw>();
  int hw = n->lv[n->L - 1].w;
  for (int l = n->L - 2; l >= 0; --l) {
    Level& v = n->lv[l];
    const Layer& a = n->layers[layer_index(n, false, l, false)];
    const Layer& b = n->layers[layer_index(n, false, l, true)];
    DIE_HIP(launch_upcat(h, v.encB.as<bf16raw>(), v.cat.as<bf16raw>(), B, v.H, v.W, hw, v.w, st));
    DIE_HIP(launch_conv(v.cat.as<bf16raw>(), B, v.H, v.W, hw + v.w, 9, false, wbf + a.woff, prm + a.boff, true,
                        v.decA.p, v.w, kOutBf16, st));
    DIE_HIP(launch_conv(v.decA.as<bf16raw>(), B, v.H, v.W, v.w, 9, false, wbf + b.woff, prm + b.boff, true, v.decB.p,
                        v.w, kOutBf16, st));
    h = v.decB.as<bf16raw>();
    hw = v.w;
  }
  const Layer& hd = n->layers.back();
  DIE_HIP(launch_conv(h, B, n->H, n->W, hw, 1, false, wbf + hd.woff, prm + hd.boff, false, n->out.p, 4, kOutF32, st));
  return DIE_OK;
}

// Parameter gradient of one layer from dz ([pixels][ldz] bf16) and its input X; when gx is
// given also the input gradient (float32, written or added).
int layer_backward(die_te_unet* n, const Layer& ly, const bf16raw* dz, int ldz, const bf16raw* X, int B, int H, int W,
                   float* gx, ConvOut mode, hipStream_t st) {
  int ns = 0;
  float* g = n->grad.as<float>();
  if (conv_wgrad_bias_fused(W, ldz, ly.cout)) {
    DIE_HIP(launch_conv_wgrad_bias(dz, ldz, X, B, H, W, ly.cin, ly.taps, ly.cout, n->wpart.as<float>(),
                                   n->bpart.as<float>(), &ns, st));
    DIE_HIP(launch_reduce_splits(n->wpart.as<float>(), ns, (size_t)ly.cout * ly.taps * ly.cin, g + ly.woff, st));
    DIE_HIP(launch_reduce_splits(n->bpart.as<float>(), ns, (size_t)ly.cout, g + ly.boff, st));
  } else {
    DIE_HIP(launch_conv_wgrad(dz, ldz, X, B, H, W, ly.cin, ly.taps, ly.cout, n->wpart.as<float>(), &ns, st));
    DIE_HIP(launch_reduce_splits(n->wpart.as<float>(), ns, (size_t)ly.cout * ly.taps * ly.cin, g + ly.woff, st));
    const long npix = (long)B * H * W;
    const int nsb = (int)std::min<long>(256, std::max<long>(1, npix / 256));
    DIE_HIP(launch_bias_grad(dz, ldz, npix, ly.cout, n->bpart.as<float>(), nsb, st));
    DIE_HIP(launch_reduce_splits(n->bpart.as<float>(), nsb, (size_t)ly.cout, g + ly.boff, st));
  }
  if (gx)
    DIE_HIP(launch_conv(dz, B, H, W, ldz, ly.taps, true, ly.wbd.as<bf16raw>(), nullptr, false, gx, ly.cin, mode, st));
  return DIE_OK;
}

int backward(die_te_unet* n, const float* target, int B, double* loss, hipStream_t st) {
  const size_t nout = (size_t)B * n->H * n->W * 4;
  const int nlb = loss_blocks(nout);
  bf16raw* dz = n->dz.as<bf16raw>();
  DIE_HIP(launch_mse(n->out.as<float>(), target, nout, n->lpart.as<double>(), dz, st));
  DIE_HIP(launch_sum_doubles(n->lpart.as<double>(), nlb, n->loss.as<double>(), st));
  const int L = n->L;
  Level& top = n->lv[0];
  const bf16raw* hin = L > 1 ? top.decB.as<bf16raw>() : top.encB.as<bf16raw>();
  float* ghin = L > 1 ? top.gDecB.as<float>() : top.gEncB.as<float>();
  DIE_TRY(layer_backward(n, n->layers.back(), dz, 8, hin, B, n->H, n->W, ghin, kOutF32, st));
  // decoder, in reverse of the forward order
  for (int l = 0; l <= L - 2; ++l) {
    Level& v = n->lv[l];
    const Layer& a = n->layers[layer_index(n, false, l, false)];
    const Layer& b = n->layers[layer_index(n, false, l, true)];
    const size_t cnt = (size_t)B * v.H * v.W * v.w;
    DIE_HIP(launch_relu_grad(v.gDecB.as<float>(), v.decB.as<bf16raw>(), dz, cnt, st));
    DIE_TRY(layer_backward(n, b, dz, v.w, v.decA.as<bf16raw>(), B, v.H, v.W, v.gDecA.as<float>(), kOutF32, st));
    DIE_HIP(launch_relu_grad(v.gDecA.as<float>(), v.decA.as<bf16raw>(), dz, cnt, st));
    DIE_TRY(layer_backward(n, a, dz, v.w, v.cat.as<bf16raw>(), B, v.H, v.W, v.gCat.as<float>(), kOutF32, st));
    const int cl = n->lv[l + 1].w;
    float* glow = (l + 1 <= L - 2) ? n->lv[l + 1].gDecB.as<float>() : n->lv[L - 1].gEncB.as<float>();
    DIE_HIP(launch_upcat_grad(v.gCat.as<float>(), glow, v.gEncB.as<float>(), B, v.H, v.W, cl, v.w, st));
  }
  // encoder, deepest level first
  for (int l = L - 1; l >= 0; --l) {
    Level& v = n->lv[l];
    const Layer& a = n->layers[layer_index(n, true, l, false)];
    const Layer& b = n->layers[layer_index(n, true, l, true)];
    const size_t cnt = (size_t)B * v.H * v.W * v.w;
    DIE_HIP(launch_relu_grad(v.gEncB.as<float>(), v.encB.as<bf16raw>(), dz, cnt, st));
    DIE_TRY(layer_backward(n, b, dz, v.w, v.encA.as<bf16raw>(), B, v.H, v.W, v.gEncA.as<float>(), kOutF32, st));
    DIE_HIP(launch_relu_grad(v.gEncA.as<float>(), v.encA.as<bf16raw>(), dz, cnt, st));
    if (l == 0) {
      DIE_TRY(layer_backward(n, a, dz, v.w, n->xin.as<bf16raw>(), B, v.H, v.W, nullptr, kOutF32, st));
    } else {
      Level& u = n->lv[l - 1];
      DIE_TRY(layer_backward(n, a, dz, v.w, u.pool.as<bf16raw>(), B, v.H, v.W, u.gPool.as<float>(), kOutF32, st));
      DIE_HIP(launch_pool_grad_add(u.gPool.as<float>(), u.gEncB.as<float>(), B, u.H, u.W, u.w, st));
    }
  }
  if (loss) {
    double sum = 0.0;
    DIE_HIP(hipMemcpyAsync(&sum, n->loss.p, sizeof(double), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    *loss = sum / (double)nout;  // mean over all outputs
  }
  return DIE_OK;
}

int check_net(const die_te_unet* n) {
  if (!n) return fail(DIE_E_INVALID, "null network");
  return DIE_OK;
}

int check_batch(const die_te_unet* n, int B) {
  if (B < 1 || B > n->maxB) return fail(DIE_E_INVALID, "batch must be in [1, max_batch]");
  return DIE_OK;
}

}  // namespace

namespace die_host {

int unet_guess(die_te_unet* n, const double2* chi, int rpo, const double2* e_in, double2* x0, int nrhs, int ny,
               int nx, hipStream_t st) {
  if (ny != n->H || nx != n->W) return fail(DIE_E_INVALID, "the network's H x W differs from the grid's ny x nx");
  const size_t ncell = (size_t)ny * nx;
  for (int r0 = 0; r0 < nrhs; r0 += n->maxB) {
    const int nb = std::min(n->maxB, nrhs - r0);
    const double2* e = e_in + (size_t)r0 * 2 * ncell;
    DIE_HIP(launch_pack_inputs(chi, 0.0, rpo, r0, e, n->xf.as<float>(), nb, ny, nx, st));
    DIE_TRY(forward(n, n->xf.as<float>(), nb, st));
    DIE_HIP(launch_unpack_guess(e, n->out.as<float>(), x0 + (size_t)r0 * 2 * ncell, nb, ny, nx, st));
  }
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}

}  // namespace die_host

extern "C" {

int die_te_unet_create(die_te_unet** out, int levels, int base, int height, int width, int max_batch,
                       unsigned long long seed, void* stream) {
  die_host::last_error().clear();
  if (!out) return fail(DIE_E_INVALID, "null argument");
  *out = nullptr;
  if (levels < 1 || levels > 8) return fail(DIE_E_INVALID, "levels must be in [1, 8]");
  if (base < 8 || base % 8 || base > 1024) return fail(DIE_E_INVALID, "base must be a multiple of 8 in [8, 1024]");
  const int div = 8 << (levels - 1);
  if (height < div || width < div || height % div || width % div || height > 8192 || width > 8192)
    return fail(DIE_E_INVALID, "height and width must be multiples of 8 * 2^(levels-1), at most 8192");
  if (max_batch < 1 || max_batch > 4096) return fail(DIE_E_INVALID, "max_batch must be in [1, 4096]");
  hipStream_t st = (hipStream_t)stream;
  auto* n = new (std::nothrow) die_te_unet();
  if (!n) return fail(DIE_E_NOMEM, "host allocation failed");
  auto guard = [&](int rc) {
    if (rc < 0) delete n;
    return rc;
  };
  if (hipGetDevice(&n->dev) != hipSuccess) return guard(fail(DIE_E_HIP, "hipGetDevice failed"));
  n->L = levels;
  n->C = base;
  n->H = height;
  n->W = width;
  n->maxB = max_batch;
  // layers in parameter order
  std::vector<int> w(levels);
  for (int l = 0; l < levels; ++l) w[l] = base << l;
  auto add = [&](int cin, int cout, int taps) {
    Layer ly;
    ly.cin = cin;
    ly.cout = cout;
    ly.taps = taps;
    ly.cpad = (cout + 7) / 8 * 8;
    ly.woff = n->np;
    n->np += (size_t)cout * taps * cin;
    ly.boff = n->np;
    n->np += cout;
    n->layers.push_back(std::move(ly));
  };
  for (int l = 0; l < levels; ++l) {
    add(l == 0 ? 8 : w[l - 1], w[l], 9);
    add(w[l], w[l], 9);
  }
  for (int l = levels - 2; l >= 0; --l) {
    add(w[l + 1] + w[l], w[l], 9);
    add(w[l], w[l], 9);
  }
  add(w[0], 4, 1);
  int rc;
  const size_t B = (size_t)max_batch;
  // buffers
  size_t dzmax = B * height * width * 8, wpmax = 0, bpmax = 0;
  for (auto& ly : n->layers) {
    if ((rc = ly.wbd.alloc((size_t)ly.cin * ly.taps * ly.cpad * sizeof(bf16raw))) < 0) return guard(rc);
    wpmax = std::max(wpmax, conv_wgrad_max_floats(ly.cout, ly.taps, ly.cin));
    bpmax = std::max(bpmax, (size_t)256 * ly.cout);
  }
  n->lv.resize(levels);
  for (int l = 0; l < levels; ++l) {
    Level& v = n->lv[l];
    v.H = height >> l;
    v.W = width >> l;
    v.w = w[l];
    const size_t pix = B * v.H * v.W;
    dzmax = std::max(dzmax, pix * v.w);
    if ((rc = v.encA.alloc(pix * v.w * 2)) < 0 || (rc = v.encB.alloc(pix * v.w * 2)) < 0 ||
        (rc = v.gEncA.alloc(pix * v.w * 4)) < 0 || (rc = v.gEncB.alloc(pix * v.w * 4)) < 0)
      return guard(rc);
    if (l < levels - 1) {
      const size_t cw = (size_t)w[l + 1] + w[l];
      if ((rc = v.pool.alloc(pix / 4 * v.w * 2)) < 0 || (rc = v.gPool.alloc(pix / 4 * v.w * 4)) < 0 ||
          (rc = v.cat.alloc(pix * cw * 2)) < 0 || (rc = v.gCat.alloc(pix * cw * 4)) < 0 ||
          (rc = v.decA.alloc(pix * v.w * 2)) < 0 || (rc = v.decB.alloc(pix * v.w * 2)) < 0 ||
          (rc = v.gDecA.alloc(pix * v.w * 4)) < 0 || (rc = v.gDecB.alloc(pix * v.w * 4)) < 0)
        return guard(rc);
    }
  }
  const size_t npx = B * height * width;
  if ((rc = n->master.alloc(n->np * 4)) < 0 || (rc = n->grad.alloc(n->np * 4)) < 0 ||
      (rc = n->m.alloc(n->np * 4)) < 0 || (rc = n->v.alloc(n->np * 4)) < 0 || (rc = n->wbf.alloc(n->np * 2)) < 0 ||
      (rc = n->xin.alloc(npx * 8 * 2)) < 0 || (rc = n->out.alloc(npx * 4 * 4)) < 0 ||
      (rc = n->dz.alloc(dzmax * 2)) < 0 || (rc = n->wpart.alloc(wpmax * 4)) < 0 ||
      (rc = n->bpart.alloc(bpmax * 4)) < 0 || (rc = n->lpart.alloc((size_t)loss_blocks(npx * 4) * 8)) < 0 ||
      (rc = n->loss.alloc(8)) < 0 || (rc = n->xf.alloc(npx * 8 * 4)) < 0)
    return guard(rc);
  // He-normal weights, zero biases
  std::vector<float> p(n->np, 0.0f);
  uint64_t s = seed ^ 0xA0761D6478BD642Full;
  for (auto& ly : n->layers) {
    const double sd = std::sqrt(2.0 / (double)(ly.taps * ly.cin));
    const size_t cnt = (size_t)ly.cout * ly.taps * ly.cin;
    for (size_t j = 0; j < cnt; j += 2) {
      const double u1 = uniform01(s), u2 = uniform01(s);
      const double r = std::sqrt(-2.0 * std::log(u1));
      p[ly.woff + j] = (float)(sd * r * std::cos(2.0 * M_PI * u2));
      if (j + 1 < cnt) p[ly.woff + j + 1] = (float)(sd * r * std::sin(2.0 * M_PI * u2));
    }
  }
  if (hipMemcpyAsync(n->master.p, p.data(), n->np * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemsetAsync(n->m.p, 0, n->np * 4, st) != hipSuccess || hipMemsetAsync(n->v.p, 0, n->np * 4, st) != hipSuccess ||
      hipMemsetAsync(n->grad.p, 0, n->np * 4, st) != hipSuccess)
    return guard(fail(DIE_E_HIP, "initialising the parameters failed"));
  if ((rc = refresh_bf16(n, st)) < 0) return guard(rc);
  if (hipStreamSynchronize(st) != hipSuccess) return guard(fail(DIE_E_HIP, "synchronising failed"));
  *out = n;
  return DIE_OK;
}

int die_te_unet_num_params(const die_te_unet* n, long long* np) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  if (!np) return fail(DIE_E_INVALID, "null output");
  *np = (long long)n->np;
  return DIE_OK;
}

int die_te_unet_get_params(die_te_unet* n, float* params, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  if (!params) return fail(DIE_E_INVALID, "null params");
  hipStream_t st = (hipStream_t)stream;
  DIE_HIP(hipMemcpyAsync(params, n->master.p, n->np * 4, hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}

int die_te_unet_set_params(die_te_unet* n, const float* params, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  if (!params) return fail(DIE_E_INVALID, "null params");
  for (size_t j = 0; j < n->np; ++j)
    if (!std::isfinite(params[j])) return fail(DIE_E_INVALID, "params contain non-finite values");
  hipStream_t st = (hipStream_t)stream;
  DIE_HIP(hipMemcpyAsync(n->master.p, params, n->np * 4, hipMemcpyHostToDevice, st));
  DIE_HIP(hipMemsetAsync(n->m.p, 0, n->np * 4, st));
  DIE_HIP(hipMemsetAsync(n->v.p, 0, n->np * 4, st));
  n->step = 0;
  DIE_TRY(refresh_bf16(n, st));
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}

int die_te_unet_get_grads(die_te_unet* n, float* grads, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  if (!grads) return fail(DIE_E_INVALID, "null grads");
  hipStream_t st = (hipStream_t)stream;
  DIE_HIP(hipMemcpyAsync(grads, n->grad.p, n->np * 4, hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}

int die_te_unet_forward(die_te_unet* n, const float* x, float* y, int batch, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  DIE_TRY(check_batch(n, batch));
  if (!x || !y) return fail(DIE_E_INVALID, "null x or y");
  hipStream_t st = (hipStream_t)stream;
  DIE_TRY(forward(n, x, batch, st));
  DIE_HIP(hipMemcpyAsync(y, n->out.p, (size_t)batch * n->H * n->W * 4 * sizeof(float), hipMemcpyDeviceToDevice, st));
  return DIE_OK;
}

int die_te_unet_loss_grad(die_te_unet* n, const float* x, const float* target, int batch, double* loss,
                          void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  DIE_TRY(check_batch(n, batch));
  if (!x || !target) return fail(DIE_E_INVALID, "null x or target");
  hipStream_t st = (hipStream_t)stream;
  DIE_TRY(forward(n, x, batch, st));
  double l = 0.0;
  DIE_TRY(backward(n, target, batch, &l, st));
  if (!std::isfinite(l)) return fail(DIE_E_BREAKDOWN, "the loss is not finite");
  if (loss) *loss = l;
  return DIE_OK;
}

int die_te_unet_adam(die_te_unet* n, float lr, float beta1, float beta2, float eps, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_net(n));
  if (!(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
    return fail(DIE_E_INVALID, "need lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
  hipStream_t st = (hipStream_t)stream;
  n->step += 1;
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, (double)n->step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, (double)n->step)));
  DIE_HIP(launch_adam(n->master.as<float>(), n->grad.as<float>(), n->m.as<float>(), n->v.as<float>(),
                      n->wbf.as<bf16raw>(), n->np, lr, beta1, beta2, eps, c1, c2, st));
  for (auto& ly : n->layers)
    DIE_HIP(launch_wbd(n->wbf.as<bf16raw>() + ly.woff, ly.wbd.as<bf16raw>(), ly.cout, ly.cpad, ly.taps, ly.cin, st));
  return DIE_OK;
}

int die_te_unet_train_step(die_te_unet* n, const float* x, const float* target, int batch, float lr, double* loss,
                           void* stream) {
  DIE_TRY(die_te_unet_loss_grad(n, x, target, batch, loss, stream));
  return die_te_unet_adam(n, lr, 0.9f, 0.999f, 1e-8f, stream);
}

int die_te_unet_pack_inputs(const void* eps_r, int nobj, const void* e_in, float* x, int batch, int ny, int nx,
                            void* stream) {
  die_host::last_error().clear();
  if (!eps_r || !e_in || !x) return fail(DIE_E_INVALID, "null argument");
  if (batch < 1 || nobj < 1 || batch % nobj || ny < 1 || nx < 1)
    return fail(DIE_E_INVALID, "need batch >= 1 a multiple of nobj >= 1, and ny, nx >= 1");
  DIE_HIP(launch_pack_inputs((const double2*)eps_r, 1.0, batch / nobj, 0, (const double2*)e_in, x, batch, ny, nx,
                             (hipStream_t)stream));
  return DIE_OK;
}

int die_te_unet_pack_targets(const void* e_tot, const void* e_in, float* t, int batch, int ny, int nx, void* stream) {
  die_host::last_error().clear();
  if (!e_tot || !e_in || !t) return fail(DIE_E_INVALID, "null argument");
  if (batch < 1 || ny < 1 || nx < 1) return fail(DIE_E_INVALID, "need batch, ny, nx >= 1");
  DIE_HIP(launch_pack_targets((const double2*)e_tot, (const double2*)e_in, t, batch, ny, nx, (hipStream_t)stream));
  return DIE_OK;
}

int die_te_unet_destroy(die_te_unet* n) {
  die_host::last_error().clear();
  if (!n) return DIE_OK;
  (void)hipDeviceSynchronize();
  delete n;
  return DIE_OK;
}

}  // extern "C"
