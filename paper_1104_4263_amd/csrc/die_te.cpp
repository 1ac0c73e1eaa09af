// Host runtime of the TE DIE solver: the C ABI declared in include/die_te.h.
//
// Everything numerical runs in the HIP kernels of kernels_fft.hip and
// kernels_krylov.hip; this file owns device memory, validates arguments,
// evaluates the Green tensor once on the host (FP64) and orchestrates the
// Krylov methods (restarted GMRES, Section 4; Arnoldi/Krylov-Schur eigensolver
// for the deflation basis, Section 4 eq. DeflatingPrecondtioner).
#include "die_te.h"
#include "die_te_learn.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <thread>
#include <vector>


#include "dense.hpp"
#include "green.hpp"
#include "host.hpp"
#include "ops.hpp"
#include "scratch.hpp"
#include "unet_internal.hpp"

using die::c2;
using cd = std::complex<double>;

namespace die_host {
std::string& last_error() {
  thread_local std::string msg;
  return msg;
}
}  // namespace die_host

namespace {

using die_host::DBuf;
using die_host::fail;

// Work buffers of the block solver, kept in the context between calls (defined with the solver).
struct BlockWork;

bool is_pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }
int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}
int auto_pad(int n) {
  int p = 2;
  while (p < 2 * n - 1) p <<= 1;
  return p;
}
// Largest order of the dense eigenvalue problem die_te_spectrum solves on the host.
constexpr int kSpectrumMaxOrder = 4096;

}  // namespace

struct die_te_ctx {
  int dev = 0;
  int nx = 0, ny = 0, px = 0, py = 0, lpx = 0, lpy = 0;
  double h = 0, k = 0;
  size_t ncell = 0, nvec = 0;
  int nobj = 1;  // objects sharing this grid (and therefore the symbol)
  int ncomp = 2;  // field components: 2 = TE (E1, E2), 1 = TM (E3), 3 = TE with H3 (E1, E2, H3)
  DBuf chi64, chir64, chi32, chir32, sym64, sym32;
  DBuf chim64, chimr64, chim32, chimr32;  // ncomp 3: magnetic contrast chi_m and its regularizer
  DBuf work;  // FFT intermediate [nrhs][2][px][ny]
  int regularize = 0;
  // deflation
  int r = 0;
  DBuf V;     // [nobj][r][nvec] complex128, orthonormal per object
  DBuf Cdev;  // [nobj][r][r] row-major complex128, C = T^-1 - I
  std::vector<cd> Chost, ritz;  // [nobj][r][r], [nobj][r]
  std::vector<double> radius;   // automatic deflation: each object's deflation radius
  int eigs_restarts = 0, eigs_converged = 0;
  // diagnostic timing: event pairs recorded around launches of each kind
  bool prof_on = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_ev[4];
  size_t prof_used[4] = {0, 0, 0, 0};
  unsigned long long prof_seen[4] = {0, 0, 0, 0};
  double prof_bytes[4] = {0, 0, 0, 0};  // algorithmic bytes (flops for the GEMM kind) of the bracketed launches
  double prof_mem[4] = {0, 0, 0, 0};    // algorithmic HBM bytes of the bracketed launches (every kind)
  double prof_ms[4] = {0, 0, 0, 0};     // elapsed ms of the bracketed launches already read back
  size_t prof_resolved[4] = {0, 0, 0, 0};  // event pairs read back so far
  int prof_every = 1;
  int prof_nlive = -1;  // right-hand sides live in the current launches (-1: all of them)
  // FFT pass variants of the products: forced (>= 0) or tuned per [FP64, FP32][batch class][pass]
  int fft_force = -1;
  std::shared_ptr<BlockWork> bw;  // block GMRES work buffers, reused by later calls
  int fftv[2][3][3] = {{{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}}, {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}}};
  ~die_te_ctx() {
    for (auto& v : prof_ev)
      for (auto& pr : v) {
        (void)hipEventDestroy(pr.first);
        (void)hipEventDestroy(pr.second);
      }
  }
};

namespace {

// Brackets the launches of one kind with events on the launch stream while profiling is on.
struct ProfScope {
  die_te_ctx* c;
  int kind;
  hipStream_t st;
  hipEvent_t end = nullptr;
  // bytes: the algorithmic HBM bytes of the bracketed launch (the compulsory reads and writes
  // of its operands), credited to the kind only when the launch is bracketed; for a GEMM,
  // bytes holds its flops and mem its operand bytes (mem < 0: mem = bytes).
  ProfScope(die_te_ctx* cc, int k, hipStream_t s, double bytes, double mem = -1.0) : c(cc), kind(k), st(s) {
    if (!c->prof_on) return;
    if (c->prof_seen[kind]++ % c->prof_every) return;  // sample one launch in prof_every
    auto& v = c->prof_ev[kind];
    size_t& u = c->prof_used[kind];
    if (u == v.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
      v.emplace_back(a, b);
    }
    (void)hipEventRecord(v[u].first, st);
    end = v[u].second;
    ++u;
    c->prof_bytes[kind] += bytes;
    c->prof_mem[kind] += mem < 0.0 ? bytes : mem;
  }
  ~ProfScope() {
    if (end) (void)hipEventRecord(end, st);
  }
};

int live_count(const die_te_ctx* c, int nrhs) { return c->prof_nlive >= 0 ? std::min(c->prof_nlive, nrhs) : nrhs; }

// Read back the elapsed time of every bracketed launch not read yet (waits for their events).
// Called before a stream that the library created is destroyed, and by die_te_profile_read.
int prof_resolve(die_te_ctx* c) {
  for (int kind = 0; kind < 4; ++kind) {
    for (size_t i = c->prof_resolved[kind]; i < c->prof_used[kind]; ++i) {
      auto& pr = c->prof_ev[kind][i];
      DIE_HIP(hipEventSynchronize(pr.second));
      float ms = 0.0f;
      DIE_HIP(hipEventElapsedTime(&ms, pr.first, pr.second));
      c->prof_ms[kind] += ms;
    }
    c->prof_resolved[kind] = c->prof_used[kind];
  }
  return DIE_OK;
}

// Algorithmic bytes of one product on R live right-hand sides (the three passes):
// pass 1 reads u (2RN) and chi, writes the row transforms (2R ny px);
// pass 2 reads them and the symbol (3 px py), writes the column products (2R ny px);
// pass 3 reads those and u, writes y (2RN).
double product_bytes(const die_te_ctx* c, int R, int nchi, size_t es) {
  const double N = (double)c->ncell, rows = (double)c->ny * c->px, P = (double)c->px * c->py;
  const double nc = c->ncomp, nplanes = die::sym_planes(c->ncomp), ncontrast = c->ncomp == 3 ? 2.0 : 1.0;
  return es * (nc * R * N + ncontrast * nchi * N + nc * R * rows + nc * R * rows + nplanes * P + nc * R * rows +
               nc * R * rows + nc * R * N + nc * R * N);
}

// ------------------------------------------------------------------ operator products
template <class T> const c2<T>* chi_of(const die_te_ctx* c, bool reg);
template <> const double2* chi_of<double>(const die_te_ctx* c, bool reg) {
  return reg ? c->chir64.as<double2>() : c->chi64.as<double2>();
}
template <> const float2* chi_of<float>(const die_te_ctx* c, bool reg) {
  return reg ? c->chir32.as<float2>() : c->chi32.as<float2>();
}
// The contrast of components from the third on (chi_m of the full TE system), null otherwise.
template <class T> const c2<T>* chi2_of(const die_te_ctx* c, bool reg);
template <> const double2* chi2_of<double>(const die_te_ctx* c, bool reg) {
  if (c->ncomp != 3) return nullptr;
  return reg ? c->chimr64.as<double2>() : c->chim64.as<double2>();
}
template <> const float2* chi2_of<float>(const die_te_ctx* c, bool reg) {
  if (c->ncomp != 3) return nullptr;
  return reg ? c->chimr32.as<float2>() : c->chim32.as<float2>();
}
template <class T> const c2<T>* sym_of(const die_te_ctx* c);
template <> const double2* sym_of<double>(const die_te_ctx* c) { return c->sym64.as<double2>(); }
template <> const float2* sym_of<float>(const die_te_ctx* c) { return c->sym32.as<float2>(); }

// Bytes of the product's FFT intermediate for nrhs fields of es-byte complex values (the
// tiled layout of the three passes: wtile_cols(px) x wtile_rows(ny) per component).
size_t work_bytes(const die_te_ctx* c, size_t nrhs, size_t es) {
  return nrhs * (size_t)c->ncomp * die::wtile_cols(c->px) * die::wtile_rows(c->ny) * es;
}

int ensure_work(die_te_ctx* c, size_t bytes, hipStream_t st) {
  if (c->work.p && c->work.bytes >= bytes) return DIE_OK;
  if (c->work.p) DIE_HIP(hipStreamSynchronize(st));
  return c->work.alloc(bytes);
}

// ------------------------------------------------------------------ FFT pass autotuner
// The radix of each product pass is chosen once per (device, precision, grid shape) for the
// whole process, because it changes the rounding and every context and batch size must agree;
// the tile of each pass is chosen per batch-size class (it moves no arithmetic).  Both by
// timing the variants of the pass on the grid with min(nrhs, 64) fields.
struct TuneKey {
  int dev, prec, lpx, lpy, nx, ny, ncomp;
  bool operator<(const TuneKey& o) const {
    return std::tie(dev, prec, lpx, lpy, nx, ny, ncomp) < std::tie(o.dev, o.prec, o.lpx, o.lpy, o.nx, o.ny, o.ncomp);
  }
};
struct TuneEntry {
  int radix[3] = {-1, -1, -1};                                   // per pass: 0 default radix, 1 the other
  int tile[3][3] = {{-1, -1, -1}, {-1, -1, -1}, {-1, -1, -1}};   // [batch class][pass]: 0 full, 1 half tile
};
std::mutex g_tune_mu;
std::map<TuneKey, TuneEntry> g_tune;

int batch_class(int nrhs) { return nrhs <= 2 ? 0 : (nrhs <= 32 ? 1 : 2); }

template <class T> const c2<T>* chi_of(const die_te_ctx* c, bool reg);
template <class T> const c2<T>* sym_of(const die_te_ctx* c);

// Launch pass `pass` (0 rows, 1 columns + symbol, 2 inverse rows) of a product on R fields.
// planar: pass 3 writes y planar (real parts of right-hand side r at planar[r ldp], imaginary parts at
// planar[(R + r) ldp]) instead of into y.
template <class T>
hipError_t launch_pass(die_te_ctx* c, int pass, int v, const c2<T>* x, c2<T>* y, c2<T>* W, int R, const int* live,
                       hipStream_t st, int rpo, const c2<T>* chi, const c2<T>* chi2, T* planar = nullptr,
                       size_t ldp = 0) {
  const int nc = c->ncomp;
  if (pass == 0)
    return die::launch_rows_fwd<T, T>(c->lpx, false, x, chi, chi2, W, c->nx, c->ny, R, nc, 0, rpo, live, st, v);
  if (pass == 1) return die::launch_cols_symbol<T>(c->lpy, nc, W, sym_of<T>(c), c->px, c->ny, R, live, st, v);
  return die::launch_rows_inv_sub<T, T>(c->lpx, W, x, y, c->nx, c->ny, nc * R, nc, live, st, v, planar, ldp, R);
}

// The variants of the three passes for products of nrhs fields; tunes them first if needed
// (synchronises st; never while st is being captured: the default variants are used then).
template <class T>
int fft_plan(die_te_ctx* c, int nrhs, hipStream_t st, const int** out) {
  const int prec = std::is_same<T, double>::value ? 0 : 1, bc = batch_class(nrhs);
  int* pv = c->fftv[prec][bc];
  *out = pv;
  if (pv[0] >= 0) return DIE_OK;
  if (c->fft_force >= 0) {
    pv[0] = pv[1] = pv[2] = c->fft_force;
    return DIE_OK;
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  DIE_HIP(hipStreamIsCapturing(st, &cap));
  static const int kDefault[3] = {0, 0, 0};
  if (cap != hipStreamCaptureStatusNone) {
    *out = kDefault;
    return DIE_OK;
  }
  const bool tuned_len[3] = {c->lpx >= die::kFftTunedMinLog, c->lpy >= die::kFftTunedMinLog,
                             c->lpx >= die::kFftTunedMinLog};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  TuneEntry& te = g_tune[TuneKey{c->dev, prec, c->lpx, c->lpy, c->nx, c->ny, c->ncomp}];
  if (te.tile[bc][0] < 0) {
    const int R = std::min(nrhs, 64);
    const size_t vbytes = (size_t)R * c->nvec * sizeof(c2<T>);
    DBuf xb, yb;
    DIE_TRY(xb.alloc(vbytes));
    DIE_TRY(yb.alloc(vbytes));
    DIE_HIP(hipMemsetAsync(xb.p, 0, vbytes, st));
    DIE_TRY(ensure_work(c, work_bytes(c, R, sizeof(c2<T>)), st));
    c2<T>* W = c->work.as<c2<T>>();
    const c2<T>* chi = chi_of<T>(c, false);
    const c2<T>* chi2 = chi2_of<T>(c, false);
    hipEvent_t e0, e1;
    DIE_HIP(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(DIE_E_HIP, "hipEventCreate failed");
    }
    struct Ev {
      hipEvent_t a, b;
      ~Ev() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
      }
    } ev{e0, e1};
    auto time_pass = [&](int pass, int v, float* ms) -> int {
      for (int k = 0; k < 2; ++k)
        DIE_HIP(launch_pass<T>(c, pass, v, xb.as<c2<T>>(), yb.as<c2<T>>(), W, R, nullptr, st, 0, chi, chi2));
      DIE_HIP(hipEventRecord(ev.a, st));
      for (int k = 0; k < 3; ++k)
        DIE_HIP(launch_pass<T>(c, pass, v, xb.as<c2<T>>(), yb.as<c2<T>>(), W, R, nullptr, st, 0, chi, chi2));
      DIE_HIP(hipEventRecord(ev.b, st));
      DIE_HIP(hipEventSynchronize(ev.b));
      DIE_HIP(hipEventElapsedTime(ms, ev.a, ev.b));
      return DIE_OK;
    };
    for (int pass = 0; pass < 3; ++pass) {
      if (!tuned_len[pass]) {
        te.radix[pass] = 0;
        te.tile[bc][pass] = 0;
        continue;
      }
      if (te.radix[pass] < 0) {
        float t0, t1;
        DIE_TRY(time_pass(pass, 0, &t0));
        DIE_TRY(time_pass(pass, 1, &t1));
        te.radix[pass] = t1 < t0 ? 1 : 0;
      }
      float tf, th;
      DIE_TRY(time_pass(pass, te.radix[pass], &tf));
      DIE_TRY(time_pass(pass, te.radix[pass] | 2, &th));
      // the half tile reads each 128-byte line of the tiled intermediate in two blocks: taken only
      // when clearly faster (its extra traffic costs the other streams' kernels)
      te.tile[bc][pass] = th < 0.97f * tf ? 1 : 0;
    }
    DIE_HIP(hipStreamSynchronize(st));  // xb, yb are freed on return
  }
  for (int pass = 0; pass < 3; ++pass) pv[pass] = te.radix[pass] | (te.tile[bc][pass] << 1);
  return DIE_OK;
}

// y = A(chi) x (reg = false) or A(chi') x (reg = true) for nrhs fields.
// Right-hand side r uses object obj0 + r / rpo (rpo = 0: every right-hand side uses object obj0).
template <class T>
int apply_op(die_te_ctx* c, const c2<T>* x, c2<T>* y, int nrhs, bool reg, const int* live, hipStream_t st,
             int rpo, int obj0 = 0, T* planar = nullptr, size_t ldp = 0) {
  const int* v = nullptr;
  DIE_TRY(fft_plan<T>(c, nrhs, st, &v));
  DIE_TRY(ensure_work(c, work_bytes(c, nrhs, sizeof(c2<T>)), st));
  c2<T>* W = c->work.as<c2<T>>();
  const int nchi = rpo > 0 ? (nrhs + rpo - 1) / rpo : 1;
  ProfScope prof(c, DIE_PROF_PRODUCT, st, product_bytes(c, live_count(c, nrhs), nchi, sizeof(c2<T>)));
  const c2<T>* chi = chi_of<T>(c, reg) + (size_t)obj0 * c->ncell;
  const c2<T>* chi2 = chi2_of<T>(c, reg);
  if (chi2) chi2 += (size_t)obj0 * c->ncell;
  for (int pass = 0; pass < 3; ++pass)
    DIE_HIP(launch_pass<T>(c, pass, v[pass], x, y, W, nrhs, live, st, rpo, chi, chi2, planar, ldp));
  return DIE_OK;
}

// Solved operator M = A_R A (regularized) or A: out = M in, tmp is a scratch field set.
template <class T>
// (planar: out is written planar instead, as launch_pass describes)
int apply_M(die_te_ctx* c, bool reg, const c2<T>* in, c2<T>* tmp, c2<T>* out, int nrhs, const int* live,
            hipStream_t st, int rpo, int obj0 = 0, T* planar = nullptr, size_t ldp = 0) {
  if (reg) {
    DIE_TRY(apply_op<T>(c, in, tmp, nrhs, false, live, st, rpo, obj0));
    DIE_TRY(apply_op<T>(c, tmp, out, nrhs, true, live, st, rpo, obj0, planar, ldp));
  } else {
    DIE_TRY(apply_op<T>(c, in, out, nrhs, false, live, st, rpo, obj0, planar, ldp));
  }
  return DIE_OK;
}

// Deflation projector y = P^-1 x = x + V (C (V^* x)) on basis-precision vectors (V in FP64).
// counter: nrhs zeroed ints (left zeroed).
// (rpo right-hand sides per object: each uses its object's V and C)
template <class T>
int apply_pinv(die_te_ctx* c, const c2<T>* x, c2<T>* y, int nrhs, double2* part, double2* coef, int* counter,
               const int* live, hipStream_t st, int rpo, int obj0 = 0) {
  // right-hand side r uses object obj0 + r / rpo, which must exist
  if (rpo < 1 || obj0 < 0 || obj0 + (nrhs - 1) / rpo >= c->nobj)
    return fail(DIE_E_INVALID, "deflation: right-hand sides map past the last object");
  const size_t n = c->nvec;
  const size_t vstride = (size_t)c->r * n, cstride = (size_t)c->r * c->r;
  const double2* V = c->V.as<double2>() + (size_t)obj0 * vstride;
  const double2* C = c->Cdev.as<double2>() + (size_t)obj0 * cstride;
  DIE_HIP((die::launch_fdot<double, T>(V, n, vstride, rpo, c->r, x, n, n, nrhs, part, 1.0, C, cstride, coef, counter,
                                       live, st)));
  DIE_HIP((die::launch_faxpy<double, T>(V, n, vstride, rpo, c->r, coef, x, y, n, n, nrhs, live, st)));
  return DIE_OK;
}

// One CGS2 Arnoldi step on w against Q[0..nq) (Q[i] of rhs r at Q + (i * nrhs + r) n):
// leaves w orthogonalised, h1neg/h2neg = -(projection coefficients) ([r * ldh + i]),
// partn = partial ||w||^2.
template <class T>
int cgs2(const c2<T>* Q, int nq, int nrhs, size_t n, c2<T>* w, double2* part, double2* h1neg, double2* h2neg,
         int ldh, double* partn, const int* live, hipStream_t st) {
  const int nblk = die::blas_blocks(n);
  const size_t vs = (size_t)nrhs * n;
  DIE_HIP((die::launch_mdot<T, T>(Q, vs, n, nq, nullptr, w, n, n, nrhs, part, live, st)));
  DIE_HIP(die::launch_reduce(part, nq, nblk, nrhs, -1.0, nullptr, h1neg, live, st));
  // the reduce writes [r * nq + i]; ldh must equal nq for the coefficient reads below
  (void)ldh;
  DIE_HIP((die::launch_maxpy<T, T, T>(1, Q, vs, n, nq, nullptr, h1neg, nq, w, n, 1.0, w, n, 0.0, n, nrhs, part,
                                      nullptr, live, st)));
  DIE_HIP(die::launch_reduce(part, nq, nblk, nrhs, -1.0, nullptr, h2neg, live, st));
  DIE_HIP((die::launch_maxpy<T, T, T>(2, Q, vs, n, nq, nullptr, h2neg, nq, w, n, 1.0, w, n, 0.0, n, nrhs, nullptr,
                                      partn, live, st)));
  return DIE_OK;
}

// ------------------------------------------------------------------ eigensolver
uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Deflation data of the r largest-magnitude eigenpairs of object `obj`'s operator into slot
// `slot` of c->V / c->Cdev / c->Chost / c->ritz (each slot sized for c->r >= r vectors; an
// object whose Krylov space closes early, or that wants fewer than c->r, fills fewer and the
// rest of its slot stays zero, which leaves P^-1 unchanged).
int run_eigs(die_te_ctx* c, int obj, int slot, int r, double tol, int mk, int maxrst, unsigned long long seed,
             hipStream_t st) {
  const int ld = c->r;  // vectors per slot
  const size_t n = c->nvec;
  const bool reg = c->regularize != 0;
  const int nblk = die::blas_blocks(n);
  if (mk <= 0) mk = std::max(2 * r + 8, 24);
  if ((size_t)mk > n - 1) mk = (int)(n - 1);
  if (mk < r + 1) return fail(DIE_E_INVALID, "deflate_k too large for the Krylov dimension");
  if (maxrst <= 0) maxrst = 300;
  if (tol <= 0) tol = 1e-4;
  DBuf Q, Qn, Tm, Wv, part, partn, hA, hB, nrm, Zd;
  DIE_TRY(Q.alloc((size_t)(mk + 1) * n * sizeof(double2)));
  DIE_TRY(Qn.alloc((size_t)mk * n * sizeof(double2)));
  DIE_TRY(Tm.alloc(n * sizeof(double2)));
  DIE_TRY(part.alloc((size_t)(mk + 1) * nblk * sizeof(double2)));
  DIE_TRY(partn.alloc((size_t)nblk * sizeof(double)));
  DIE_TRY(hA.alloc((size_t)(mk + 1) * sizeof(double2)));
  DIE_TRY(hB.alloc((size_t)(mk + 1) * sizeof(double2)));
  DIE_TRY(nrm.alloc(sizeof(double)));
  DIE_TRY(Zd.alloc((size_t)mk * mk * sizeof(double2)));
  double2* q = Q.as<double2>();
  // seeded start vector
  {
    std::vector<double2> v(n);
    uint64_t s = seed ^ 0x5DEECE66Dull;
    for (size_t e = 0; e < n; ++e) {
      const double a = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
      const double b = (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0) - 0.5;
      v[e] = make_double2(a, b);
    }
    DIE_HIP(hipMemcpyAsync(q, v.data(), n * sizeof(double2), hipMemcpyHostToDevice, st));
    DIE_HIP((die::launch_norm2<double>(q, n, n, 1, partn.as<double>(), nullptr, st)));
    DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, 1, nrm.as<double>(), nullptr, st));
    double nn = 0;
    DIE_HIP(hipMemcpyAsync(&nn, nrm.p, sizeof(double), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    std::vector<double> sc(1, 1.0 / std::sqrt(nn));
    DBuf scd;
    DIE_TRY(scd.alloc(sizeof(double)));
    DIE_HIP(hipMemcpyAsync(scd.p, sc.data(), sizeof(double), hipMemcpyHostToDevice, st));
    DIE_HIP((die::launch_scale<double, double>(q, n, q, n, scd.as<double>(), 1, n, 1, nullptr, st)));
    DIE_HIP(hipStreamSynchronize(st));
  }
  die::la::Mat H(mk + 1, mk);
  int k0 = 0, mk_eff = mk;
  die::la::Mat S, Z;
  std::vector<double> resid;
  int rst = 0;
  bool converged = false;
  DBuf scd;
  DIE_TRY(scd.alloc(sizeof(double)));
  for (rst = 0; rst <= maxrst; ++rst) {
    mk_eff = mk;
    for (int j = k0; j < mk; ++j) {
      double2* w = q + (size_t)(j + 1) * n;
      DIE_TRY(apply_M<double>(c, reg, q + (size_t)j * n, Tm.as<double2>(), w, 1, nullptr, st, 0, obj));
      DIE_TRY(cgs2<double>(q, j + 1, 1, n, w, part.as<double2>(), hA.as<double2>(), hB.as<double2>(), j + 1,
                           partn.as<double>(), nullptr, st));
      DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, 1, nrm.as<double>(), nullptr, st));
      std::vector<double2> ha(j + 1), hb(j + 1);
      double nn = 0;
      DIE_HIP(hipMemcpyAsync(ha.data(), hA.p, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, st));
      DIE_HIP(hipMemcpyAsync(hb.data(), hB.p, (j + 1) * sizeof(double2), hipMemcpyDeviceToHost, st));
      DIE_HIP(hipMemcpyAsync(&nn, nrm.p, sizeof(double), hipMemcpyDeviceToHost, st));
      DIE_HIP(hipStreamSynchronize(st));
      double hn = 0;
      for (int i = 0; i <= j; ++i) {
        H(i, j) = -cd(ha[i].x + hb[i].x, ha[i].y + hb[i].y);
        hn += std::norm(H(i, j));
      }
      const double beta = std::sqrt(nn);
      if (!std::isfinite(beta)) return fail(DIE_E_BREAKDOWN, "eigensolver: non-finite Arnoldi coefficient");
      H(j + 1, j) = beta;
      if (beta <= 1e-13 * std::sqrt(hn)) {  // invariant subspace: the Ritz values are exact
        mk_eff = j + 1;
        break;
      }
      const double inv = 1.0 / beta;
      DIE_HIP(hipMemcpyAsync(scd.p, &inv, sizeof(double), hipMemcpyHostToDevice, st));
      DIE_HIP((die::launch_scale<double, double>(w, n, w, n, scd.as<double>(), 1, n, 1, nullptr, st)));
      DIE_HIP(hipStreamSynchronize(st));
    }
    // Schur form of the projected matrix, wanted (largest |theta|) first
    S = die::la::Mat(mk_eff, mk_eff);
    for (int j = 0; j < mk_eff; ++j)
      for (int i = 0; i < mk_eff; ++i) S(i, j) = H(i, j);
    Z = die::la::Mat::eye(mk_eff);
    die::la::hessenberg(S, Z);
    if (!die::la::schur(S, Z)) return fail(DIE_E_BREAKDOWN, "eigensolver: QR iteration did not converge");
    std::vector<int> idx(mk_eff);
    for (int i = 0; i < mk_eff; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](int a, int b) { return std::abs(S(a, a)) > std::abs(S(b, b)); });
    const int rr = std::min(r, mk_eff);
    std::vector<char> want(mk_eff, 0);
    for (int i = 0; i < rr; ++i) want[idx[i]] = 1;
    die::la::reorder(S, Z, want);
    const cd beta_last = H(mk_eff, mk_eff - 1);
    std::vector<cd> b(mk_eff);
    for (int l = 0; l < mk_eff; ++l) b[l] = beta_last * Z(mk_eff - 1, l);
    die::la::Mat Y = die::la::tri_eigvecs(S);
    resid.assign(rr, 0.0);
    int nconv = 0;
    for (int i = 0; i < rr; ++i) {
      cd s = 0;
      for (int l = 0; l <= i; ++l) s += b[l] * Y(l, i);
      resid[i] = std::abs(s);
      if (resid[i] <= tol * std::abs(S(i, i))) ++nconv;
    }
    c->eigs_converged = nconv;
    if (nconv >= rr || mk_eff < mk || rst == maxrst) {
      converged = nconv >= rr;
      break;
    }
    // Krylov-Schur restart: keep kk leading Schur vectors
    const int kk = std::min(mk - 1, r + (mk - r) / 2);
    std::vector<double2> zh((size_t)mk_eff * kk);
    for (int l = 0; l < kk; ++l)
      for (int i = 0; i < mk_eff; ++i) zh[(size_t)l * mk_eff + i] = make_double2(Z(i, l).real(), Z(i, l).imag());
    DIE_HIP(hipMemcpyAsync(Zd.p, zh.data(), zh.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    DIE_HIP((die::launch_maxpy<double, double, double>(0, q, n, 0, mk_eff, nullptr, Zd.as<double2>(), mk_eff,
                                                       (const double2*)nullptr, 0, 0.0, Qn.as<double2>(), n, 0.0,
                                                       n, kk, nullptr, nullptr, nullptr, st)));
    DIE_HIP(hipMemcpyAsync(q, Qn.p, (size_t)kk * n * sizeof(double2), hipMemcpyDeviceToDevice, st));
    DIE_HIP(hipMemcpyAsync(q + (size_t)kk * n, q + (size_t)mk_eff * n, n * sizeof(double2), hipMemcpyDeviceToDevice,
                           st));
    DIE_HIP(hipStreamSynchronize(st));
    die::la::Mat Hn(mk + 1, mk);
    for (int j = 0; j < kk; ++j) {
      for (int i = 0; i <= j; ++i) Hn(i, j) = S(i, j);
      Hn(kk, j) = b[j];
    }
    H = Hn;
    k0 = kk;
  }
  c->eigs_restarts = rst;
  const int rr = std::min(r, mk_eff);
  // deflation basis V = Q Z[:, :rr]
  double2* Vo = c->V.as<double2>() + (size_t)slot * ld * n;
  {
    std::vector<double2> zh((size_t)mk_eff * rr);
    for (int l = 0; l < rr; ++l)
      for (int i = 0; i < mk_eff; ++i) zh[(size_t)l * mk_eff + i] = make_double2(Z(i, l).real(), Z(i, l).imag());
    DIE_HIP(hipMemcpyAsync(Zd.p, zh.data(), zh.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    DIE_HIP((die::launch_maxpy<double, double, double>(0, q, n, 0, mk_eff, nullptr, Zd.as<double2>(), mk_eff,
                                                       (const double2*)nullptr, 0, 0.0, Vo, n, 0.0,
                                                       n, rr, nullptr, nullptr, nullptr, st)));
  }
  // T = V^* M V from rr products of M (batched), C = T^-1 - I
  DBuf MV, MT, partT, Td;
  DIE_TRY(MV.alloc((size_t)rr * n * sizeof(double2)));
  DIE_TRY(MT.alloc((size_t)rr * n * sizeof(double2)));
  DIE_TRY(partT.alloc((size_t)rr * rr * nblk * sizeof(double2)));
  DIE_TRY(Td.alloc((size_t)rr * rr * sizeof(double2)));
  DIE_TRY(apply_M<double>(c, reg, Vo, MT.as<double2>(), MV.as<double2>(), rr, nullptr, st, 0, obj));
  DIE_HIP((die::launch_mdot<double, double>(Vo, n, 0, rr, nullptr, MV.as<double2>(), n, n, rr,
                                            partT.as<double2>(), nullptr, st)));
  DIE_HIP(die::launch_reduce(partT.as<double2>(), rr, nblk, rr, 1.0, nullptr, Td.as<double2>(), nullptr, st));
  std::vector<double2> th((size_t)rr * rr);
  DIE_HIP(hipMemcpyAsync(th.data(), Td.p, th.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  die::la::Mat T(rr, rr), Ti;
  for (int l = 0; l < rr; ++l)
    for (int i = 0; i < rr; ++i) T(i, l) = cd(th[(size_t)l * rr + i].x, th[(size_t)l * rr + i].y);
  if (!die::la::inverse(T, Ti)) return fail(DIE_E_BREAKDOWN, "deflation: T = V^* M V is singular");
  std::vector<double2> ch((size_t)ld * ld, make_double2(0.0, 0.0));
  cd* Ch = c->Chost.data() + (size_t)slot * ld * ld;
  for (int i = 0; i < rr; ++i)
    for (int l = 0; l < rr; ++l) {
      cd v = Ti(i, l) - (i == l ? 1.0 : 0.0);
      Ch[(size_t)i * ld + l] = v;
      ch[(size_t)i * ld + l] = make_double2(v.real(), v.imag());
    }
  DIE_HIP(hipMemcpyAsync(c->Cdev.as<double2>() + (size_t)slot * ld * ld, ch.data(), ch.size() * sizeof(double2),
                         hipMemcpyHostToDevice, st));
  for (int i = 0; i < rr; ++i) c->ritz[(size_t)slot * ld + i] = S(i, i);
  DIE_HIP(hipStreamSynchronize(st));
  (void)converged;
  return DIE_OK;
}

// ------------------------------------------------------------------ GMRES
// T: precision of the cycle's products and vectors; TB: storage of the Krylov basis in the
// one-reduction path (T, or binary16 for the compressed basis).
// Optional HIP graph of one restart cycle's inner iterations, captured on a stream of its own
// (the caller's may be the legacy default stream, which cannot be captured) and launched on
// the solve's stream.
struct CycleGraph {
  hipStream_t cs = nullptr;
  hipGraphExec_t exec = nullptr;
  CycleGraph() = default;
  CycleGraph(const CycleGraph&) = delete;
  CycleGraph& operator=(const CycleGraph&) = delete;
  ~CycleGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (cs) (void)hipStreamDestroy(cs);
  }
  // issue(stream) queues the launches to capture
  template <class F> int capture(F&& issue) {
    DIE_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    DIE_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    const int rc = issue(cs);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(cs, &graph);
    if (rc < 0) {
      if (graph) (void)hipGraphDestroy(graph);
      return rc;
    }
    DIE_HIP(e);
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (ei != hipSuccess) exec = nullptr;
    DIE_HIP(ei);
    return DIE_OK;
  }
};

// Copy the kept best iterate back into u for every right-hand side that ended without
// convergence or breakdown at a true residual above its best one (synchronises st).
int restore_best(double2* u, const double2* ubest, size_t n, int nrhs, const std::vector<int>& conv,
                 const std::vector<int>& brk, const std::vector<double>& best, std::vector<double>& relres,
                 std::vector<int>& bm, int* dmask, const double* one, hipStream_t st) {
  int nb = 0;
  for (int r = 0; r < nrhs; ++r) {
    bm[r] = !conv[r] && !brk[r] && best[r] < relres[r];
    if (bm[r]) {
      relres[r] = best[r];
      ++nb;
    }
  }
  if (!nb) return DIE_OK;
  DIE_HIP(hipMemcpyAsync(dmask, bm.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
  DIE_HIP((die::launch_scale<double, double>(ubest, n, u, n, one, 0, n, nrhs, dmask, st)));
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}

template <class T, class TB = T>
int gmres_solve(die_te_ctx* c, const double2* b, double2* u, int nrhs, const die_te_solve_opts& o,
                die_te_solve_info* info, hipStream_t st) {
  const size_t n = c->nvec;
  const int m = o.restart;
  const int nblk = die::blas_blocks(n);
  const bool reg = c->regularize != 0;
  const bool defl = c->r > 0;
  const int rpo = nrhs / c->nobj;  // right-hand sides per object (validated by the caller)
  const double tol = o.tol > 0 ? o.tol : 1e-8;
  const double margin = reg ? (o.reg_margin > 0 ? o.reg_margin : 0.1) : 1.0;
  const double floor_eta = std::is_same<T, float>::value ? 2e-6 : 0.0;
  const size_t vbytes = (size_t)nrhs * n * sizeof(c2<T>);
  const size_t dbytes = (size_t)nrhs * n * sizeof(double2);
  const int nvmax = std::max(m + 1, c->r);
  DBuf Q, Zb, Tb, Wb, Rs, Sd, part, partn, h1, h2, hd, Rm, cs, sn, g, y, state, live, active, nrm, cnt;
  DBuf Qb, Vf, Wf;  // one-reduction path: basis q_0..q_{m-1} (TB), current v and w (T)
  const bool dcgs = o.orth == 1;
  if (dcgs) {
    DIE_TRY(Qb.alloc((size_t)m * nrhs * n * sizeof(c2<TB>)));
    DIE_TRY(Vf.alloc(vbytes));
    DIE_TRY(Wf.alloc(vbytes));
  } else {
    DIE_TRY(Q.alloc((size_t)(m + 1) * vbytes));
  }
  if (defl) DIE_TRY(Zb.alloc(vbytes));
  if (reg) DIE_TRY(Tb.alloc(vbytes));
  DIE_TRY(Wb.alloc(vbytes));
  DIE_TRY(Rs.alloc(dbytes));
  if (reg) DIE_TRY(Sd.alloc(dbytes));
  DIE_TRY(part.alloc((size_t)nrhs * std::max((size_t)nvmax * nblk, die::gmres_part_elems(n, nvmax)) *
                     sizeof(double2)));
  DIE_TRY(partn.alloc((size_t)nrhs * nblk * sizeof(double)));
  DIE_TRY(h1.alloc((size_t)nrhs * (m + 1) * sizeof(double2)));
  DIE_TRY(h2.alloc((size_t)nrhs * (m + 1) * sizeof(double2)));
  DIE_TRY(hd.alloc((size_t)nrhs * std::max(c->r, 1) * sizeof(double2)));
  DIE_TRY(Rm.alloc((size_t)nrhs * (m + 1) * m * sizeof(double2)));
  DIE_TRY(cs.alloc((size_t)nrhs * m * sizeof(double)));
  DIE_TRY(sn.alloc((size_t)nrhs * m * sizeof(double2)));
  DIE_TRY(g.alloc((size_t)nrhs * (m + 1) * sizeof(double2)));
  DIE_TRY(y.alloc((size_t)nrhs * m * sizeof(double2)));
  DIE_TRY(state.alloc((size_t)nrhs * sizeof(die::GmresState)));
  DIE_TRY(live.alloc((size_t)nrhs * sizeof(int)));
  DIE_TRY(active.alloc((size_t)nrhs * sizeof(int)));
  DIE_TRY(nrm.alloc((size_t)nrhs * sizeof(double)));
  DIE_TRY(cnt.alloc((size_t)nrhs * die::kCounterStride * sizeof(int)));
  DIE_HIP(hipMemsetAsync(cnt.p, 0, (size_t)nrhs * die::kCounterStride * sizeof(int), st));
  int* dcnt = cnt.as<int>();
  {  // pick the FFT pass variants now, never inside a captured cycle
    const int* pv = nullptr;
    DIE_TRY(fft_plan<T>(c, nrhs, st, &pv));
    DIE_TRY(fft_plan<double>(c, nrhs, st, &pv));
  }
  DIE_TRY(ensure_work(c, work_bytes(c, nrhs, std::max(sizeof(c2<T>), sizeof(double2))), st));
  // one-reduction Arnoldi: raw dots, unrotated Hessenberg, first projections, axpy coefficients
  const int dstride = 2 * (m + 2);
  DBuf Dd, Hu, cprev, coef, part2;
  if (dcgs) {
    DIE_TRY(Dd.alloc((size_t)nrhs * dstride * sizeof(double2)));
    DIE_TRY(Hu.alloc((size_t)nrhs * (m + 1) * m * sizeof(double2)));
    DIE_TRY(cprev.alloc((size_t)nrhs * (m + 1) * sizeof(double2)));
    DIE_TRY(coef.alloc((size_t)nrhs * 2 * (m + 1) * sizeof(double2)));
    DIE_TRY(part2.alloc((size_t)nrhs * die::gmres_part_elems(n, 2 * (m + 2)) * sizeof(double2)));
  }

  c2<T>* q = Q.as<c2<T>>();
  c2<TB>* qb = Qb.as<c2<TB>>();
  c2<T>* vf = Vf.as<c2<T>>();
  c2<T>* wf = Wf.as<c2<T>>();
  const size_t vs = (size_t)nrhs * n;  // stride between basis vectors j
  double2* res = Rs.as<double2>();
  std::vector<double> bnorm(nrhs), rnorm(nrhs), hn(nrhs);
  std::vector<int> act(nrhs, 1), iters(nrhs, 0), pa(nrhs, 0), par(nrhs, 0), cycles(nrhs, 0), conv(nrhs, 0),
      brk(nrhs, 0);
  std::vector<double> relres(nrhs, 1.0);
  // best iterate so far per right-hand side (returned when the tolerance is not reached: the
  // regularized cycles minimise ||A_R r||, so ||r|| need not decrease from cycle to cycle)
  DBuf Ubest, bmask, oned;
  DIE_TRY(Ubest.alloc(dbytes));
  DIE_TRY(bmask.alloc((size_t)nrhs * sizeof(int)));
  DIE_TRY(oned.alloc(sizeof(double)));
  const double one = 1.0;
  DIE_HIP(hipMemcpyAsync(oned.p, &one, sizeof(double), hipMemcpyHostToDevice, st));
  std::vector<double> best(nrhs, std::numeric_limits<double>::infinity());
  std::vector<int> bm(nrhs, 0);
  bool first_check = true;

  if (!o.x0_given) DIE_HIP(hipMemsetAsync(u, 0, dbytes, st));
  DIE_HIP((die::launch_norm2<double>(b, n, n, nrhs, partn.as<double>(), nullptr, st)));
  DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), nullptr, st));
  DIE_HIP(hipMemcpyAsync(hn.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  for (int r = 0; r < nrhs; ++r) {
    bnorm[r] = std::sqrt(hn[r]);
    if (!std::isfinite(bnorm[r])) return fail(DIE_E_INVALID, "e_in contains non-finite values");
  }

  std::vector<die::GmresState> hst(nrhs);
  std::vector<int> jn(nrhs);
  DBuf jd;
  DIE_TRY(jd.alloc(nrhs * sizeof(int)));
  std::vector<double2> hg((size_t)nrhs * (m + 1));
  std::vector<double> inv0(nrhs);
  DBuf sc;
  DIE_TRY(sc.alloc((size_t)nrhs * sizeof(double)));
  struct LiveReset {
    die_te_ctx* c;
    ~LiveReset() { c->prof_nlive = -1; }
  } live_reset{c};
  auto nlive = [&]() {
    int k = 0;
    for (int r = 0; r < nrhs; ++r) k += act[r] != 0;
    return k;
  };
  CycleGraph gx;
  const bool use_graph = o.graph != 0 && !c->prof_on;
  for (;;) {
    // ---- FP64 true residual res = b - A u
    c->prof_nlive = nlive();
    DIE_HIP(hipMemcpyAsync(active.p, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    const int* dact = active.as<int>();
    DIE_TRY(apply_op<double>(c, u, res, nrhs, false, dact, st, rpo));
    DIE_HIP((die::launch_maxpy<double, double, double>(2, (const double2*)nullptr, 0, 0, 0, nullptr, nullptr, 0, b, n,
                                                       1.0, res, n, -1.0, n, nrhs, nullptr, partn.as<double>(), dact,
                                                       st)));
    DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), dact, st));
    DIE_HIP(hipMemcpyAsync(hn.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    int nact = 0, nfb = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      pa[r] += 1;
      rnorm[r] = std::sqrt(hn[r]);
      relres[r] = bnorm[r] > 0 ? rnorm[r] / bnorm[r] : 0.0;
      if (first_check && o.x0_given && !(std::isfinite(rnorm[r]) && rnorm[r] < bnorm[r])) {
        // a given guess that is non-finite or no better than zero is replaced by zero
        DIE_HIP(hipMemsetAsync(u + (size_t)r * n, 0, n * sizeof(double2), st));
        ++nfb;
      } else if (!std::isfinite(rnorm[r])) {
        brk[r] = 1;
        act[r] = 0;
      } else if (relres[r] <= tol || bnorm[r] == 0.0) {
        conv[r] = 1;
        act[r] = 0;
      } else if (iters[r] >= o.max_iters) {
        act[r] = 0;
      } else {
        ++nact;
      }
    }
    first_check = false;
    if (nfb) continue;  // residuals of the zeroed guesses
    if (nact == 0) break;
    // the iterate about to be corrected is kept when it is the best one so far
    {
      int nb = 0;
      for (int r = 0; r < nrhs; ++r) {
        bm[r] = act[r] && relres[r] < best[r];
        if (bm[r]) {
          best[r] = relres[r];
          ++nb;
        }
      }
      if (nb) {
        DIE_HIP(hipMemcpyAsync(bmask.p, bm.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
        DIE_HIP((die::launch_scale<double, double>(u, n, Ubest.as<double2>(), n, oned.as<double>(), 0, n, nrhs,
                                                   bmask.as<int>(), st)));
      }
    }
    DIE_HIP(hipMemcpyAsync(active.p, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    // ---- cycle right-hand side s = A_R res (or res), beta0, q0 = s / beta0
    const double2* s = res;
    if (reg) {
      DIE_TRY(apply_op<double>(c, res, Sd.as<double2>(), nrhs, true, dact, st, rpo));
      s = Sd.as<double2>();
      for (int r = 0; r < nrhs; ++r) par[r] += act[r];
    }
    DIE_HIP((die::launch_norm2<double>(s, n, n, nrhs, partn.as<double>(), dact, st)));
    DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), dact, st));
    DIE_HIP(hipMemcpyAsync(hn.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    std::fill(hg.begin(), hg.end(), make_double2(0.0, 0.0));
    for (int r = 0; r < nrhs; ++r) {
      die::GmresState S{};
      S.j = 0;
      S.done = act[r] ? 0 : 1;
      const double beta0 = std::sqrt(hn[r]);
      S.beta0 = beta0;
      double eta = act[r] ? tol * bnorm[r] / rnorm[r] * margin : 1.0;
      eta = std::min(1.0, std::max(eta, floor_eta));
      S.target = eta * beta0;
      hst[r] = S;
      hg[(size_t)r * (m + 1)] = make_double2(beta0, 0.0);
      inv0[r] = beta0 > 0 ? 1.0 / beta0 : 0.0;
      if (act[r] && !(beta0 > 0 && std::isfinite(beta0))) {
        // regularized residual vanished or is non-finite: nothing this cycle can do
        act[r] = 0;
        if (!std::isfinite(beta0)) brk[r] = 1;
      }
    }
    c->prof_nlive = nlive();
    DIE_HIP(hipMemcpyAsync(state.p, hst.data(), nrhs * sizeof(die::GmresState), hipMemcpyHostToDevice, st));
    DIE_HIP(hipMemcpyAsync(g.p, hg.data(), hg.size() * sizeof(double2), hipMemcpyHostToDevice, st));
    DIE_HIP(hipMemcpyAsync(sc.p, inv0.data(), nrhs * sizeof(double), hipMemcpyHostToDevice, st));
    DIE_HIP(hipMemcpyAsync(active.p, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    DIE_HIP(hipMemcpyAsync(live.p, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    int* dlive = live.as<int>();
    DIE_HIP((die::launch_scale<double, T>(s, n, dcgs ? vf : q, n, sc.as<double>(), 1, n, nrhs, dact, st)));
    // ---- Arnoldi / GMRES iterations of this cycle (every launch argument is the same in every
    // cycle: the per-rhs state, flags and counters live on the device)
    auto iterate = [&](hipStream_t st) -> int {
      for (int j = 0; dcgs && j <= m; ++j) {
        // one-reduction step j: product on v, one dots pass, scalar update, one pass writing
        // q_j into the basis and the next v
        c2<T>* v = vf;
        c2<T>* w = j < m ? wf : nullptr;
        if (w) {
          const c2<T>* zin = v;
          if (defl) {
            DIE_TRY(apply_pinv<T>(c, v, Zb.as<c2<T>>(), nrhs, part.as<double2>(), hd.as<double2>(), dcnt, dlive, st,
                                  rpo));
            zin = Zb.as<c2<T>>();
          }
          DIE_TRY(apply_M<T>(c, reg, zin, reg ? Tb.as<c2<T>>() : nullptr, w, nrhs, dlive, st, rpo));
        }
        // algorithmic bytes: j basis vectors in TB, v and w in T
        const double nl = (double)live_count(c, nrhs) * n;
        const double bb = nl * sizeof(c2<TB>), vb = nl * sizeof(c2<T>);
        {
          ProfScope prof(c, DIE_PROF_DOTS, st, bb * j + vb * (w ? 2 : 1));
          DIE_HIP((die::launch_dots2<TB, T>(qb, vs, j, v, w, n, n, nrhs, part2.as<double2>(), Dd.as<double2>(), dstride,
                                            dcnt, dlive, st)));
        }
        DIE_HIP(die::launch_dcgs_update(Dd.as<double2>(), dstride, j, m, nrhs, state.as<die::GmresState>(),
                                        Hu.as<double2>(), Rm.as<double2>(), cs.as<double>(), sn.as<double2>(),
                                        g.as<double2>(), cprev.as<double2>(), coef.as<double2>(), dlive, st));
        if (j < m) {
          ProfScope prof(c, DIE_PROF_AXPY, st, bb * (j + 1) + vb * 3);
          DIE_HIP((die::launch_dcgs_axpy<TB, T>(qb, vs, j, vf, wf, n, n, nrhs, coef.as<double2>(), m + 1,
                                                state.as<die::GmresState>(), dlive, st)));
        }
      }
      for (int j = 0; !dcgs && j < m; ++j) {
        const c2<T>* qj = q + (size_t)j * vs;
        const c2<T>* z = qj;
        if (defl) {
          DIE_TRY(apply_pinv<T>(c, qj, Zb.as<c2<T>>(), nrhs, part.as<double2>(), hd.as<double2>(), dcnt, dlive, st, rpo));
          z = Zb.as<c2<T>>();
        }
        c2<T>* w = q + (size_t)(j + 1) * vs;
        DIE_TRY(apply_M<T>(c, reg, z, reg ? Tb.as<c2<T>>() : nullptr, w, nrhs, dlive, st, rpo));
        // CGS2 against Q[0..j], FP64 Givens update, normalisation
        const int nq = j + 1;
        // per live right-hand side: dots read nq basis vectors and w; the multi-axpys also write w
        const double vb = (double)live_count(c, nrhs) * n * sizeof(c2<T>);
        {
          ProfScope prof(c, DIE_PROF_DOTS, st, vb * (nq + 1));
          DIE_HIP((die::launch_fdot<T, T>(q, vs, n, 1, nq, w, n, n, nrhs, part.as<double2>(), -1.0, nullptr, 0,
                                          h1.as<double2>(), dcnt, dlive, st)));
        }
        {
          ProfScope prof(c, DIE_PROF_AXPY, st, vb * (nq + 2));
          DIE_HIP((die::launch_faxpy<T, T>(q, vs, n, 1, nq, h1.as<double2>(), (const c2<T>*)nullptr, w, n, n, nrhs,
                                           dlive, st)));
        }
        {
          ProfScope prof(c, DIE_PROF_DOTS, st, vb * (nq + 1));
          DIE_HIP((die::launch_fdot<T, T>(q, vs, n, 1, nq, w, n, n, nrhs, part.as<double2>(), -1.0, nullptr, 0,
                                          h2.as<double2>(), dcnt, dlive, st)));
        }
        {
          ProfScope prof(c, DIE_PROF_AXPY, st, vb * (nq + 2));
          DIE_HIP((die::launch_faxpy_givens<T, T>(q, vs, n, nq, h2.as<double2>(), h1.as<double2>(), w, n, n, nrhs,
                                                  part.as<double2>(), dcnt, state.as<die::GmresState>(),
                                                  Rm.as<double2>(), cs.as<double>(), sn.as<double2>(), g.as<double2>(),
                                                  m, dlive, st)));
        }
        DIE_HIP((die::launch_scale<T, T>(w, n, w, n, &state.as<die::GmresState>()->invbeta,
                                         (int)(sizeof(die::GmresState) / sizeof(double)), n, nrhs, dlive, st)));
      }
      return DIE_OK;
    };
    if (use_graph) {
      if (!gx.exec) DIE_TRY(gx.capture(iterate));  // captured once, replayed every cycle
      DIE_HIP(hipGraphLaunch(gx.exec, st));
    } else {
      DIE_TRY(iterate(st));
    }
    // ---- least squares y = R^-1 g, then u += P^-1 (Q y)
    DIE_HIP(die::launch_lsq(state.as<die::GmresState>(), Rm.as<double2>(), g.as<double2>(), y.as<double2>(), m, nrhs,
                            dact, st));
    DIE_HIP(hipMemcpyAsync(hst.data(), state.p, nrhs * sizeof(die::GmresState), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) jn[r] = act[r] ? hst[r].j : 0;
    DIE_HIP(hipMemcpyAsync(jd.p, jn.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    c2<T>* t = Wb.as<c2<T>>();
    if (dcgs)
      DIE_HIP((die::launch_maxpy<TB, T, T>(0, qb, vs, n, m, jd.as<int>(), y.as<double2>(), m, (const c2<T>*)nullptr,
                                           0, 0.0, t, n, 0.0, n, nrhs, nullptr, nullptr, dact, st)));
    else
      DIE_HIP((die::launch_maxpy<T, T, T>(0, q, vs, n, m, jd.as<int>(), y.as<double2>(), m, (const c2<T>*)nullptr, 0,
                                          0.0, t, n, 0.0, n, nrhs, nullptr, nullptr, dact, st)));
    if (defl) {
      // t += V (C (V^* t)) with each object's V and C, then u += t below
      DIE_TRY(apply_pinv<T>(c, t, t, nrhs, part.as<double2>(), hd.as<double2>(), dcnt, dact, st, rpo));
    }
    {
      DIE_HIP((die::launch_maxpy<double, T, double>(0, (const double2*)nullptr, 0, 0, 0, nullptr, nullptr, 0, t, n, 1.0,
                                                    u, n, 1.0, n, nrhs, nullptr, nullptr, dact, st)));
    }
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      iters[r] += hst[r].j;
      cycles[r] += 1;
      // the one-reduction step that detects the end has already applied its product
      const int prods = dcgs ? std::min(hst[r].j + 1, m) : hst[r].j;
      pa[r] += prods;
      if (reg) par[r] += prods;
      if (hst[r].breakdown) {
        brk[r] = 1;
        act[r] = 0;
      }
    }
  }
  // right-hand sides that stopped short of the tolerance get their best iterate back
  DIE_TRY(restore_best(u, Ubest.as<double2>(), n, nrhs, conv, brk, best, relres, bm, bmask.as<int>(),
                       oned.as<double>(), st));
  int rc = DIE_OK;
  for (int r = 0; r < nrhs; ++r) {
    if (brk[r]) rc = std::min(rc, (int)DIE_E_BREAKDOWN);
    else if (!conv[r] && rc == DIE_OK) rc = DIE_NOT_CONVERGED;
    if (info) {
      info[r].status = brk[r] ? DIE_E_BREAKDOWN : (conv[r] ? DIE_OK : DIE_NOT_CONVERGED);
      info[r].iters = iters[r];
      info[r].products_A = pa[r];
      info[r].products_AR = par[r];
      info[r].cycles = cycles[r];
      info[r].rel_res_true = relres[r];
      info[r].finish_iters = 0;
    }
  }
  if (rc == DIE_E_BREAKDOWN) return fail(DIE_E_BREAKDOWN, "GMRES met a non-finite value");
  return rc;
}

// ------------------------------------------------------------ other Krylov solvers
// Per right-hand side dots out[r] = (X_r, Y_r) = sum conj(X_r) Y_r (FP64, fixed order), on the device.
int rhs_dots(const double2* X, const double2* Y, size_t n, int nrhs, double2* part, double2* out, const int* live,
             hipStream_t st) {
  DIE_HIP((die::launch_mdot<double, double>(X, 0, n, 1, nullptr, Y, n, n, nrhs, part, live, st)));
  DIE_HIP(die::launch_reduce(part, 1, die::blas_blocks(n), nrhs, 1.0, nullptr, out, live, st));
  return DIE_OK;
}
template <class V> int fetch(const DBuf& d, std::vector<V>& h, hipStream_t st) {
  DIE_HIP(hipMemcpyAsync(h.data(), d.p, h.size() * sizeof(V), hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}
template <class V> int put(DBuf& d, const std::vector<V>& h, hipStream_t st) {
  DIE_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(V), hipMemcpyHostToDevice, st));
  DIE_HIP(hipStreamSynchronize(st));  // the host vector may change before the copy would run
  return DIE_OK;
}

// Bi-CGSTAB (method 1, van der Vorst's stabilised bi-conjugate gradients), restarted GCR(m)
// (method 2, generalized conjugate residuals, restart = m) and IDR(s) (method 3, Sonneveld and van
// Gijzen's induced dimension reduction, s = restart, a random orthonormal shadow space of s
// vectors drawn from a fixed seed) on the system GMRES solves,
// M P^-1 v = A_R r with M = A_R A (regularized) or A and u += P^-1 v, in FP64: the Conclusions
// of the paper note that any short-memory Krylov solver applies to this preconditioned system and
// name these.  Every right-hand side runs its own recurrence in the shared launches; the
// recurrence scalars are formed on the host.  A right-hand side whose recurrence residual reaches
// its target (the tolerance scaled to the solved system, as for GMRES cycles), breaks down or
// stagnates has its FP64 true residual b - A u evaluated; below the tolerance it has converged,
// else its recurrence restarts from that residual.  iters counts applications of M.
int alt_solve(die_te_ctx* c, const double2* b, double2* u, int nrhs, const die_te_solve_opts& o,
              die_te_solve_info* info, hipStream_t st) {
  using cdv = std::complex<double>;
  const size_t n = c->nvec;
  const int m = o.restart;  // GCR: directions kept before a restart; IDR: the shadow dimension s
  const bool gcr = o.method == 2, idr = o.method == 3;
  const int nblk = die::blas_blocks(n);
  const bool reg = c->regularize != 0;
  const bool defl = c->r > 0;
  const int rpo = nrhs / c->nobj;
  const double tol = o.tol > 0 ? o.tol : 1e-8;
  const double margin = reg ? (o.reg_margin > 0 ? o.reg_margin : 0.1) : 1.0;
  const size_t dbytes = (size_t)nrhs * n * sizeof(double2);
  DBuf Rr, Rh, Pv, Vv, Sv, Tv, Ph, Sh, Tmp, Res, Pd, Qd, part, partn, nrm, dv, cf, livb, pcnt, pcoef, ppart, scl;
  DBuf Ubest, bmask, one;  // the best iterate so far per right-hand side (returned when not converged)
  DIE_TRY(Ubest.alloc(dbytes));
  DIE_TRY(bmask.alloc((size_t)nrhs * sizeof(int)));
  DIE_TRY(one.alloc(sizeof(double)));
  {
    const double v1 = 1.0;
    DIE_HIP(hipMemcpyAsync(one.p, &v1, sizeof(double), hipMemcpyHostToDevice, st));
  }
  DIE_TRY(Rr.alloc(dbytes));
  DIE_TRY(Tmp.alloc(dbytes));
  DIE_TRY(Res.alloc(dbytes));
  DBuf Sd, VVd, Zd, Wd;  // IDR: shadow space (s x n, shared), v, P^-1 v, a temporary
  if (gcr || idr) {  // GCR: directions and images; IDR: dU and dR (s columns per right-hand side)
    DIE_TRY(Pd.alloc((size_t)m * dbytes));
    DIE_TRY(Qd.alloc((size_t)m * dbytes));
  }
  if (idr) {
    DIE_TRY(Sd.alloc((size_t)m * n * sizeof(double2)));
    DIE_TRY(VVd.alloc(dbytes));
    DIE_TRY(Zd.alloc(dbytes));
    DIE_TRY(Wd.alloc(dbytes));
    DIE_TRY(Tv.alloc(dbytes));
    // the shadow space: s vectors of normal deviates (SplitMix64 and Box-Muller, seed fixed), made
    // orthonormal by modified Gram-Schmidt on the host
    std::vector<cd> Sh((size_t)m * n);
    unsigned long long state = 0x1D5A11CEULL;
    auto next = [&]() {
      unsigned long long z = (state += 0x9E3779B97F4A7C15ULL);
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
      z ^= z >> 31;
      return ((double)(z >> 11) + 0.5) * (1.0 / 9007199254740992.0);
    };
    for (auto& v : Sh) {
      const double u1 = next(), u2 = next(), rr = std::sqrt(-2.0 * std::log(u1));
      v = cd(rr * std::cos(2.0 * M_PI * u2), rr * std::sin(2.0 * M_PI * u2));
    }
    for (int i = 0; i < m; ++i) {
      cd* vi = Sh.data() + (size_t)i * n;
      for (int j = 0; j < i; ++j) {
        const cd* vj = Sh.data() + (size_t)j * n;
        cd h = 0.0;
        for (size_t e = 0; e < n; ++e) h += std::conj(vj[e]) * vi[e];
        for (size_t e = 0; e < n; ++e) vi[e] -= h * vj[e];
      }
      double nv = 0.0;
      for (size_t e = 0; e < n; ++e) nv += std::norm(vi[e]);
      nv = std::sqrt(nv);
      for (size_t e = 0; e < n; ++e) vi[e] /= nv;
    }
    DIE_HIP(hipMemcpyAsync(Sd.p, Sh.data(), Sh.size() * sizeof(cd), hipMemcpyHostToDevice, st));
    DIE_HIP(hipStreamSynchronize(st));
  }
  if (!gcr && !idr) {
    DIE_TRY(Rh.alloc(dbytes));
    DIE_TRY(Pv.alloc(dbytes));
    DIE_TRY(Vv.alloc(dbytes));
    DIE_TRY(Sv.alloc(dbytes));
    DIE_TRY(Tv.alloc(dbytes));
    if (defl) {
      DIE_TRY(Ph.alloc(dbytes));
      DIE_TRY(Sh.alloc(dbytes));
    }
  }
  const int nvd = (gcr || idr) ? m : 1;
  DIE_TRY(part.alloc((size_t)nrhs * nvd * nblk * sizeof(double2)));
  DIE_TRY(partn.alloc((size_t)nrhs * nblk * sizeof(double)));
  DIE_TRY(nrm.alloc((size_t)nrhs * sizeof(double)));
  DIE_TRY(dv.alloc((size_t)nrhs * 2 * nvd * sizeof(double2)));
  DIE_TRY(cf.alloc((size_t)nrhs * 3 * sizeof(double2)));
  DIE_TRY(livb.alloc((size_t)nrhs * sizeof(int)));
  DIE_TRY(scl.alloc((size_t)nrhs * sizeof(double)));
  if (defl) {
    DIE_TRY(ppart.alloc((size_t)nrhs * std::max((size_t)c->r * nblk, die::gmres_part_elems(n, c->r)) *
                        sizeof(double2)));
    DIE_TRY(pcoef.alloc((size_t)nrhs * c->r * sizeof(double2)));
    DIE_TRY(pcnt.alloc((size_t)nrhs * die::kCounterStride * sizeof(int)));
    DIE_HIP(hipMemsetAsync(pcnt.p, 0, (size_t)nrhs * die::kCounterStride * sizeof(int), st));
  }
  {
    const int* pv = nullptr;
    DIE_TRY(fft_plan<double>(c, nrhs, st, &pv));
  }
  DIE_TRY(ensure_work(c, work_bytes(c, nrhs, sizeof(double2)), st));
  const int* live = livb.as<int>();
  double2* R = Rr.as<double2>();
  double2* TMP = Tmp.as<double2>();
  // z = P^-1 x (or x itself), y = M z
  auto pinv = [&](const double2* x, double2* z) -> int {
    return apply_pinv<double>(c, x, z, nrhs, ppart.as<double2>(), pcoef.as<double2>(), pcnt.as<int>(), live, st, rpo);
  };
  auto opM = [&](const double2* z, double2* y) -> int {
    return apply_M<double>(c, reg, z, reg ? TMP : nullptr, y, nrhs, live, st, rpo);
  };
  auto norms = [&](const double2* x, std::vector<double>& out) -> int {
    DIE_HIP((die::launch_norm2<double>(x, n, n, nrhs, partn.as<double>(), live, st)));
    DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), live, st));
    std::vector<double> h(nrhs);
    DIE_TRY(fetch(nrm, h, st));
    for (int r = 0; r < nrhs; ++r) out[r] = std::sqrt(h[r]);
    return DIE_OK;
  };
  auto dotsv = [&](const double2* X, const double2* Y, std::vector<cdv>& out) -> int {
    DIE_TRY(rhs_dots(X, Y, n, nrhs, part.as<double2>(), dv.as<double2>(), live, st));
    std::vector<double2> h(nrhs);
    DIE_HIP(hipMemcpyAsync(h.data(), dv.p, nrhs * sizeof(double2), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    for (int r = 0; r < nrhs; ++r) out[r] = cdv(h[r].x, h[r].y);
    return DIE_OK;
  };
  std::vector<int> act(nrhs, 1), lv(nrhs, 0), conv(nrhs, 0), brk(nrhs, 0), iters(nrhs, 0), pa(nrhs, 0), par(nrhs, 0),
      cyc(nrhs, 0), kslot(nrhs, 0), check(nrhs, 1);
  std::vector<double> bnorm(nrhs), relres(nrhs, 1.0), target(nrhs, 0.0), rn(nrhs), best(nrhs, 1e300);
  std::vector<cdv> rho(nrhs, 1.0), alpha(nrhs, 1.0), omega(nrhs, 1.0), d1(nrhs), d2(nrhs);
  // IDR: per right-hand side the phase (0 .. s-1 the first minimal-residual steps, s + k step k of
  // a group of s + 1), the oldest difference column, S^H dR (s x s, column-major) and S^H r
  std::vector<int> phase(nrhs, 0), oldest(nrhs, 0);
  std::vector<cdv> SdR(idr ? (size_t)nrhs * m * m : 0), Sr(idr ? (size_t)nrhs * m : 0);
  auto set_live = [&](const std::vector<int>& mask) -> int {
    lv = mask;
    return put(livb, lv, st);
  };
  if (!o.x0_given) DIE_HIP(hipMemsetAsync(u, 0, dbytes, st));
  DIE_TRY(set_live(std::vector<int>(nrhs, 1)));
  DIE_TRY(norms(b, bnorm));
  for (int r = 0; r < nrhs; ++r)
    if (!std::isfinite(bnorm[r])) return fail(DIE_E_INVALID, "e_in contains non-finite values");
  bool first = true;
  for (;;) {
    // ---- FP64 true residuals of the right-hand sides due a check; restart their recurrences
    std::vector<int> chk(nrhs, 0);
    int nchk = 0;
    for (int r = 0; r < nrhs; ++r)
      if (act[r] && check[r]) {
        chk[r] = 1;
        ++nchk;
      }
    if (nchk) {
      DIE_TRY(set_live(chk));
      DIE_TRY(apply_op<double>(c, u, Res.as<double2>(), nrhs, false, live, st, rpo));
      DIE_HIP((die::launch_maxpy<double, double, double>(0, (const double2*)nullptr, 0, 0, 0, nullptr, nullptr, 0, b, n,
                                                         1.0, Res.as<double2>(), n, -1.0, n, nrhs, nullptr, nullptr,
                                                         live, st)));
      std::vector<double> tr(nrhs);
      DIE_TRY(norms(Res.as<double2>(), tr));
      std::vector<int> imp(nrhs, 0);  // iterates better than the best so far
      int nimp = 0;
      int nfb = 0;
      for (int r = 0; r < nrhs; ++r) {
        if (!chk[r]) continue;
        pa[r] += 1;
        ++cyc[r];
        const double rel = bnorm[r] > 0 ? tr[r] / bnorm[r] : 0.0;
        if (first && o.x0_given && !(std::isfinite(tr[r]) && tr[r] < bnorm[r])) {
          // a given guess that is non-finite or no better than zero is replaced by zero
          DIE_HIP(hipMemsetAsync(u + (size_t)r * n, 0, n * sizeof(double2), st));
          ++nfb;
          continue;
        }
        relres[r] = rel;
        if (std::isfinite(rel) && rel < best[r]) {
          best[r] = rel;
          imp[r] = 1;
          ++nimp;
        }
        if (!std::isfinite(tr[r])) {
          brk[r] = 1;
          act[r] = 0;
        } else if (rel <= tol || bnorm[r] == 0.0) {
          conv[r] = 1;
          act[r] = 0;
        } else if (iters[r] >= o.max_iters) {
          act[r] = 0;
        }
        if (!act[r]) chk[r] = 0;
      }
      first = false;
      if (nfb) continue;  // residuals of the zeroed guesses
      if (nimp) {
        DIE_TRY(put(bmask, imp, st));
        DIE_HIP((die::launch_scale<double, double>(u, n, Ubest.as<double2>(), n, one.as<double>(), 0, n, nrhs,
                                                   bmask.as<int>(), st)));
      }
      int nre = 0;
      for (int r = 0; r < nrhs; ++r) nre += chk[r];
      if (nre) {
        // the recurrence restarts: R = A_R res (or res), and the method's own state
        DIE_TRY(set_live(chk));
        if (reg) {
          DIE_TRY(apply_op<double>(c, Res.as<double2>(), R, nrhs, true, live, st, rpo));
        } else {
          DIE_HIP(hipMemcpyAsync(R, Res.as<double2>(), dbytes, hipMemcpyDeviceToDevice, st));
        }
        std::vector<double> sn(nrhs);
        DIE_TRY(norms(R, sn));
        for (int r = 0; r < nrhs; ++r) {
          if (!chk[r]) continue;
          if (reg) par[r] += 1;
          const double tres = relres[r] * bnorm[r];
          target[r] = tres > 0 ? margin * tol * bnorm[r] * sn[r] / tres : 0.0;
          rn[r] = sn[r];
          check[r] = 0;
          kslot[r] = 0;
          phase[r] = 0;
          oldest[r] = 0;
          rho[r] = alpha[r] = omega[r] = 1.0;
          if (!(sn[r] > 0) || !std::isfinite(sn[r])) {  // the regularized residual vanished
            act[r] = 0;
          }
        }
        if (!gcr && !idr) {  // r^ = R, p = v = 0
          DIE_HIP(hipMemcpyAsync(Rh.p, R, dbytes, hipMemcpyDeviceToDevice, st));
          std::vector<double2> z3((size_t)nrhs * 3, make_double2(0.0, 0.0));
          DIE_TRY(put(cf, z3, st));
          DIE_HIP(die::launch_comb3(Pv.as<double2>(), nullptr, nullptr, nullptr, cf.as<double2>(), n, nrhs, live, st));
          DIE_HIP(die::launch_comb3(Vv.as<double2>(), nullptr, nullptr, nullptr, cf.as<double2>(), n, nrhs, live, st));
        }
      }
    }
    // ---- one step of every right-hand side still iterating
    std::vector<int> run(nrhs, 0);
    int nrun = 0;
    for (int r = 0; r < nrhs; ++r)
      if (act[r] && !check[r]) {
        run[r] = 1;
        ++nrun;
      }
    if (nrun == 0) {
      bool any = false;
      for (int r = 0; r < nrhs; ++r) any = any || (act[r] && check[r]);
      if (!any) break;
      continue;
    }
    DIE_TRY(set_live(run));
    const double tiny = 1e-300;
    if (idr) {
      // the right-hand sides in the lowest phase take one step; the others wait for them
      int ph = INT32_MAX;
      for (int r = 0; r < nrhs; ++r)
        if (run[r]) ph = std::min(ph, phase[r]);
      for (int r = 0; r < nrhs; ++r) run[r] = run[r] && phase[r] == ph;
      DIE_TRY(set_live(run));
      const size_t vs = (size_t)nrhs * n;
      double2* dU = Pd.as<double2>();
      double2* dR = Qd.as<double2>();
      double2* Vp = VVd.as<double2>();
      double2* Zp = Zd.as<double2>();
      double2* Wp = Wd.as<double2>();
      double2* Tp = Tv.as<double2>();
      const double2* Sp = Sd.as<double2>();
      std::vector<double2> co((size_t)nrhs * 3, make_double2(0.0, 0.0)), cu((size_t)nrhs * 3, make_double2(0.0, 0.0));
      auto c3 = [](cdv a) { return make_double2(a.real(), a.imag()); };
      // dm = S^H x into column `col` of S^H dR (and, with add_r, into S^H r)
      auto shadow_dots = [&](const double2* x, bool is_dr, const std::vector<int>& col) -> int {
        DIE_HIP((die::launch_mdot<double, double>(Sp, n, 0, m, nullptr, x, n, n, nrhs, part.as<double2>(), live, st)));
        DIE_HIP(die::launch_reduce(part.as<double2>(), m, nblk, nrhs, 1.0, nullptr, dv.as<double2>(), live, st));
        std::vector<double2> h((size_t)nrhs * m);
        DIE_HIP(hipMemcpyAsync(h.data(), dv.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
        DIE_HIP(hipStreamSynchronize(st));
        for (int r = 0; r < nrhs; ++r) {
          if (!run[r]) continue;
          for (int i = 0; i < m; ++i) {
            const cdv d(h[(size_t)r * m + i].x, h[(size_t)r * m + i].y);
            if (is_dr) {
              SdR[((size_t)r * m + col[r]) * m + i] = d;
              Sr[(size_t)r * m + i] += d;  // r was updated by this dR
            } else {
              Sr[(size_t)r * m + i] = d;
            }
          }
        }
        return DIE_OK;
      };
      if (ph < m) {
        // minimal-residual step ph: z = P^-1 r, v = M z, omega = (v, r) / (v, v),
        // dU_ph = omega z, dR_ph = -omega v, u += dU_ph, r += dR_ph
        const double2* z = R;
        if (defl) {
          DIE_TRY(pinv(R, Zp));
          z = Zp;
        }
        DIE_TRY(opM(z, Vp));
        DIE_TRY(dotsv(Vp, R, d1));
        DIE_TRY(dotsv(Vp, Vp, d2));
        for (int r = 0; r < nrhs; ++r) {
          if (!run[r]) continue;
          iters[r] += 1;
          pa[r] += 1;
          if (reg) par[r] += 1;
          if (!(d2[r].real() > tiny)) {
            check[r] = 1;
            continue;
          }
          omega[r] = d1[r] / d2[r];
          co[3 * r] = c3(omega[r]);
          cu[3 * r] = c3(-omega[r]);
        }
        for (int r = 0; r < nrhs; ++r) run[r] = run[r] && !check[r];
        DIE_TRY(set_live(run));
        double2* dUk = dU + (size_t)ph * vs;
        double2* dRk = dR + (size_t)ph * vs;
        DIE_TRY(put(cf, co, st));
        DIE_HIP(die::launch_comb3(dUk, z, nullptr, nullptr, cf.as<double2>(), n, nrhs, live, st));
        DIE_TRY(put(cf, cu, st));
        DIE_HIP(die::launch_comb3(dRk, Vp, nullptr, nullptr, cf.as<double2>(), n, nrhs, live, st));
        std::vector<double2> one3((size_t)nrhs * 3, make_double2(1.0, 0.0));
        DIE_TRY(put(cf, one3, st));
        DIE_HIP(die::launch_comb3(u, u, dUk, nullptr, cf.as<double2>(), n, nrhs, live, st));
        DIE_HIP(die::launch_comb3(R, R, dRk, nullptr, cf.as<double2>(), n, nrhs, live, st));
        std::vector<int> col(nrhs, ph);
        // the column of S^H dR; S^H r itself once the s steps are done
        DIE_HIP((die::launch_mdot<double, double>(Sp, n, 0, m, nullptr, dRk, n, n, nrhs, part.as<double2>(), live,
                                                  st)));
        DIE_HIP(die::launch_reduce(part.as<double2>(), m, nblk, nrhs, 1.0, nullptr, dv.as<double2>(), live, st));
        {
          std::vector<double2> h((size_t)nrhs * m);
          DIE_HIP(hipMemcpyAsync(h.data(), dv.p, h.size() * sizeof(double2), hipMemcpyDeviceToHost, st));
          DIE_HIP(hipStreamSynchronize(st));
          for (int r = 0; r < nrhs; ++r)
            if (run[r])
              for (int i = 0; i < m; ++i)
                SdR[((size_t)r * m + ph) * m + i] = cdv(h[(size_t)r * m + i].x, h[(size_t)r * m + i].y);
        }
        if (ph == m - 1) DIE_TRY(shadow_dots(R, false, col));
        for (int r = 0; r < nrhs; ++r)
          if (run[r]) phase[r] = ph + 1;
      } else {
        const int k = ph - m;  // step k of the group
        // c = (S^H dR)^-1 S^H r per right-hand side (host, s x s)
        std::vector<double2> negc((size_t)nrhs * m, make_double2(0.0, 0.0));
        for (int r = 0; r < nrhs; ++r) {
          if (!run[r]) continue;
          die::la::Mat Mm(m, m), Mi;
          for (int j = 0; j < m; ++j)
            for (int i = 0; i < m; ++i) Mm(i, j) = SdR[((size_t)r * m + j) * m + i];
          if (!die::la::inverse(Mm, Mi)) {
            check[r] = 1;
            continue;
          }
          for (int i = 0; i < m; ++i) {
            cdv ci = 0.0;
            for (int j = 0; j < m; ++j) ci += Mi(i, j) * Sr[(size_t)r * m + j];
            if (!std::isfinite(ci.real()) || !std::isfinite(ci.imag())) {
              check[r] = 1;
              break;
            }
            negc[(size_t)r * m + i] = c3(-ci);
          }
        }
        for (int r = 0; r < nrhs; ++r) run[r] = run[r] && !check[r];
        DIE_TRY(set_live(run));
        DIE_TRY(put(dv, negc, st));
        // v = r - dR c; z = P^-1 v; W = -dU c
        DIE_HIP((die::launch_maxpy<double, double, double>(0, dR, vs, n, m, nullptr, dv.as<double2>(), m, R, n, 1.0,
                                                           Vp, n, 0.0, n, nrhs, nullptr, nullptr, live, st)));
        const double2* z = Vp;
        if (defl) {
          DIE_TRY(pinv(Vp, Zp));
          z = Zp;
        }
        DIE_HIP((die::launch_maxpy<double, double, double>(0, dU, vs, n, m, nullptr, dv.as<double2>(), m, nullptr, n,
                                                           0.0, Wp, n, 0.0, n, nrhs, nullptr, nullptr, live, st)));
        std::vector<int> col(nrhs, 0);
        for (int r = 0; r < nrhs; ++r) col[r] = oldest[r];
        // the oldest column of every running right-hand side (they share the phase, not always
        // the column): written through per-right-hand-side masks, one column index at a time
        for (int oc = 0; oc < m; ++oc) {
          std::vector<int> sel(nrhs, 0);
          int ns = 0;
          for (int r = 0; r < nrhs; ++r)
            if (run[r] && oldest[r] == oc) {
              sel[r] = 1;
              ++ns;
            }
          if (!ns) continue;
          DIE_TRY(set_live(sel));
          double2* dUo = dU + (size_t)oc * vs;
          double2* dRo = dR + (size_t)oc * vs;
          if (k == 0) {
            // t = M z, omega = (t, v) / (t, t); dR_o = (v - r) - omega t; dU_o = W + omega z
            DIE_TRY(opM(z, Tp));
            DIE_TRY(dotsv(Tp, Vp, d1));
            DIE_TRY(dotsv(Tp, Tp, d2));
            for (int r = 0; r < nrhs; ++r) {
              if (!sel[r]) continue;
              iters[r] += 1;
              pa[r] += 1;
              if (reg) par[r] += 1;
              omega[r] = d2[r].real() > tiny ? d1[r] / d2[r] : cdv(0.0);
              co[3 * r] = make_double2(1.0, 0.0);
              co[3 * r + 1] = make_double2(-1.0, 0.0);
              co[3 * r + 2] = c3(-omega[r]);
              cu[3 * r] = make_double2(1.0, 0.0);
              cu[3 * r + 1] = c3(omega[r]);
              cu[3 * r + 2] = make_double2(0.0, 0.0);
            }
            DIE_TRY(put(cf, co, st));
            DIE_HIP(die::launch_comb3(dRo, Vp, R, Tp, cf.as<double2>(), n, nrhs, live, st));
            DIE_TRY(put(cf, cu, st));
            DIE_HIP(die::launch_comb3(dUo, Wp, z, nullptr, cf.as<double2>(), n, nrhs, live, st));
          } else {
            // dU_o = W + omega z; dR_o = -M dU_o
            for (int r = 0; r < nrhs; ++r) {
              if (!sel[r]) continue;
              iters[r] += 1;
              pa[r] += 1;
              if (reg) par[r] += 1;
              cu[3 * r] = make_double2(1.0, 0.0);
              cu[3 * r + 1] = c3(omega[r]);
              cu[3 * r + 2] = make_double2(0.0, 0.0);
              co[3 * r] = make_double2(-1.0, 0.0);
            }
            DIE_TRY(put(cf, cu, st));
            DIE_HIP(die::launch_comb3(dUo, Wp, z, nullptr, cf.as<double2>(), n, nrhs, live, st));
            DIE_TRY(opM(dUo, Tp));
            DIE_TRY(put(cf, co, st));
            DIE_HIP(die::launch_comb3(dRo, Tp, nullptr, nullptr, cf.as<double2>(), n, nrhs, live, st));
          }
          // u += dU_o; r += dR_o; the column of S^H dR and S^H r
          std::vector<double2> one3((size_t)nrhs * 3, make_double2(1.0, 0.0));
          DIE_TRY(put(cf, one3, st));
          DIE_HIP(die::launch_comb3(u, u, dUo, nullptr, cf.as<double2>(), n, nrhs, live, st));
          DIE_HIP(die::launch_comb3(R, R, dRo, nullptr, cf.as<double2>(), n, nrhs, live, st));
          std::vector<int> runs = run;
          run = sel;
          DIE_TRY(shadow_dots(dRo, true, col));
          run = runs;
        }
        DIE_TRY(set_live(run));
        for (int r = 0; r < nrhs; ++r) {
          if (!run[r]) continue;
          oldest[r] = (oldest[r] + 1) % m;
          phase[r] = m + (k + 1) % (m + 1);
        }
      }
    } else if (!gcr) {
      // rho1 = (r^, r); p = r + beta (p - omega v)
      DIE_TRY(dotsv(Rh.as<double2>(), R, d1));
      std::vector<double2> co((size_t)nrhs * 3, make_double2(0.0, 0.0));
      for (int r = 0; r < nrhs; ++r) {
        if (!run[r]) continue;
        const cdv beta = (d1[r] / rho[r]) * (alpha[r] / omega[r]);
        if (std::abs(d1[r]) <= tiny || !std::isfinite(std::abs(beta))) {
          check[r] = 1;  // breakdown: restart from the true residual
          continue;
        }
        rho[r] = d1[r];
        co[3 * r] = make_double2(1.0, 0.0);
        co[3 * r + 1] = make_double2(beta.real(), beta.imag());
        const cdv bo = -beta * omega[r];
        co[3 * r + 2] = make_double2(bo.real(), bo.imag());
      }
      for (int r = 0; r < nrhs; ++r) run[r] = run[r] && !check[r];
      DIE_TRY(set_live(run));
      DIE_TRY(put(cf, co, st));
      DIE_HIP(die::launch_comb3(Pv.as<double2>(), R, Pv.as<double2>(), Vv.as<double2>(), cf.as<double2>(), n, nrhs,
                                live, st));
      const double2* ph = Pv.as<double2>();
      if (defl) {
        DIE_TRY(pinv(Pv.as<double2>(), Ph.as<double2>()));
        ph = Ph.as<double2>();
      }
      DIE_TRY(opM(ph, Vv.as<double2>()));
      // alpha = rho1 / (r^, v); s = r - alpha v
      DIE_TRY(dotsv(Rh.as<double2>(), Vv.as<double2>(), d2));
      for (int r = 0; r < nrhs; ++r) {
        if (!run[r]) continue;
        iters[r] += 1;
        pa[r] += 1;
        if (reg) par[r] += 1;
        if (std::abs(d2[r]) <= tiny) {
          check[r] = 1;
          co[3 * r] = co[3 * r + 1] = co[3 * r + 2] = make_double2(0.0, 0.0);
          continue;
        }
        alpha[r] = rho[r] / d2[r];
        co[3 * r] = make_double2(1.0, 0.0);
        co[3 * r + 1] = make_double2(-alpha[r].real(), -alpha[r].imag());
        co[3 * r + 2] = make_double2(0.0, 0.0);
      }
      for (int r = 0; r < nrhs; ++r) run[r] = run[r] && !check[r];
      DIE_TRY(set_live(run));
      DIE_TRY(put(cf, co, st));
      DIE_HIP(die::launch_comb3(Sv.as<double2>(), R, Vv.as<double2>(), nullptr, cf.as<double2>(), n, nrhs, live, st));
      const double2* sh = Sv.as<double2>();
      if (defl) {
        DIE_TRY(pinv(Sv.as<double2>(), Sh.as<double2>()));
        sh = Sh.as<double2>();
      }
      DIE_TRY(opM(sh, Tv.as<double2>()));
      // omega = (t, s) / (t, t); u += alpha p^ + omega s^; r = s - omega t
      DIE_TRY(dotsv(Tv.as<double2>(), Sv.as<double2>(), d1));
      DIE_TRY(dotsv(Tv.as<double2>(), Tv.as<double2>(), d2));
      std::vector<double2> cu((size_t)nrhs * 3, make_double2(0.0, 0.0));
      for (int r = 0; r < nrhs; ++r) {
        if (!run[r]) continue;
        iters[r] += 1;
        pa[r] += 1;
        if (reg) par[r] += 1;
        omega[r] = d2[r].real() > 0 ? d1[r] / d2[r] : cdv(0.0);
        cu[3 * r] = make_double2(1.0, 0.0);
        cu[3 * r + 1] = make_double2(alpha[r].real(), alpha[r].imag());
        cu[3 * r + 2] = make_double2(omega[r].real(), omega[r].imag());
        co[3 * r] = make_double2(1.0, 0.0);
        co[3 * r + 1] = make_double2(-omega[r].real(), -omega[r].imag());
        co[3 * r + 2] = make_double2(0.0, 0.0);
      }
      DIE_TRY(put(cf, cu, st));
      DIE_HIP(die::launch_comb3(u, u, ph, sh, cf.as<double2>(), n, nrhs, live, st));
      DIE_TRY(put(cf, co, st));
      DIE_HIP(die::launch_comb3(R, Sv.as<double2>(), Tv.as<double2>(), nullptr, cf.as<double2>(), n, nrhs, live, st));
      for (int r = 0; r < nrhs; ++r)
        if (run[r] && std::abs(omega[r]) <= tiny) check[r] = 1;  // stagnation: restart
    } else {
      // z = P^-1 r into slot k, q = M z; CGS2 of q against the slots before it (z alike);
      // q, z scaled to ||q|| = 1; alpha = (q, r); u += alpha z; r -= alpha q
      // every right-hand side of one call uses the same slot index: slots advance together
      int k = -1;
      for (int r = 0; r < nrhs; ++r)
        if (run[r]) k = std::max(k, kslot[r]);
      for (int r = 0; r < nrhs; ++r)
        if (run[r] && kslot[r] != k) {  // right-hand sides that restarted at another slot wait
          run[r] = 0;
        }
      DIE_TRY(set_live(run));
      const size_t vs = (size_t)nrhs * n;
      double2* zk = Pd.as<double2>() + (size_t)k * vs;
      double2* qk = Qd.as<double2>() + (size_t)k * vs;
      if (defl) {
        DIE_TRY(pinv(R, zk));
      } else {
        DIE_HIP(hipMemcpyAsync(zk, R, dbytes, hipMemcpyDeviceToDevice, st));
      }
      DIE_TRY(opM(zk, qk));
      for (int pass = 0; pass < 2 && k > 0; ++pass) {
        DIE_HIP((die::launch_mdot<double, double>(Qd.as<double2>(), vs, n, k, nullptr, qk, n, n, nrhs,
                                                  part.as<double2>(), live, st)));
        DIE_HIP(die::launch_reduce(part.as<double2>(), k, nblk, nrhs, -1.0, nullptr, dv.as<double2>(), live, st));
        DIE_HIP((die::launch_maxpy<double, double, double>(0, Qd.as<double2>(), vs, n, k, nullptr, dv.as<double2>(), k,
                                                           nullptr, n, 0.0, qk, n, 1.0, n, nrhs, nullptr, nullptr,
                                                           live, st)));
        DIE_HIP((die::launch_maxpy<double, double, double>(0, Pd.as<double2>(), vs, n, k, nullptr, dv.as<double2>(), k,
                                                           nullptr, n, 0.0, zk, n, 1.0, n, nrhs, nullptr, nullptr,
                                                           live, st)));
      }
      std::vector<double> qn(nrhs);
      DIE_TRY(norms(qk, qn));
      std::vector<double> inv(nrhs, 0.0);
      for (int r = 0; r < nrhs; ++r) {
        if (!run[r]) continue;
        iters[r] += 1;
        pa[r] += 1;
        if (reg) par[r] += 1;
        if (!(qn[r] > tiny) || !std::isfinite(qn[r])) {
          check[r] = 1;  // the new direction lies in the span of the kept ones
          continue;
        }
        inv[r] = 1.0 / qn[r];
      }
      for (int r = 0; r < nrhs; ++r) run[r] = run[r] && !check[r];
      DIE_TRY(set_live(run));
      DIE_TRY(put(scl, inv, st));
      DIE_HIP((die::launch_scale<double, double>(qk, n, qk, n, scl.as<double>(), 1, n, nrhs, live, st)));
      DIE_HIP((die::launch_scale<double, double>(zk, n, zk, n, scl.as<double>(), 1, n, nrhs, live, st)));
      DIE_TRY(dotsv(qk, R, d1));
      std::vector<double2> cu((size_t)nrhs * 3, make_double2(0.0, 0.0)), co((size_t)nrhs * 3, make_double2(0.0, 0.0));
      for (int r = 0; r < nrhs; ++r) {
        if (!run[r]) continue;
        cu[3 * r] = make_double2(1.0, 0.0);
        cu[3 * r + 1] = make_double2(d1[r].real(), d1[r].imag());
        co[3 * r] = make_double2(1.0, 0.0);
        co[3 * r + 1] = make_double2(-d1[r].real(), -d1[r].imag());
        kslot[r] = (kslot[r] + 1) % m;
      }
      DIE_TRY(put(cf, cu, st));
      DIE_HIP(die::launch_comb3(u, u, zk, nullptr, cf.as<double2>(), n, nrhs, live, st));
      DIE_TRY(put(cf, co, st));
      DIE_HIP(die::launch_comb3(R, R, qk, nullptr, cf.as<double2>(), n, nrhs, live, st));
    }
    // the recurrence residuals: a right-hand side at its target, or out of iterations, is checked
    std::vector<double> rr(nrhs);
    DIE_TRY(norms(R, rr));
    for (int r = 0; r < nrhs; ++r) {
      if (!run[r]) continue;
      rn[r] = rr[r];
      if (!std::isfinite(rr[r]) || rr[r] <= target[r] || iters[r] >= o.max_iters) check[r] = 1;
    }
  }
  // right-hand sides that stopped short of the tolerance get their best checked iterate back
  {
    std::vector<int> bm(nrhs, 0);
    DIE_TRY(restore_best(u, Ubest.as<double2>(), n, nrhs, conv, brk, best, relres, bm, bmask.as<int>(),
                         one.as<double>(), st));
  }
  int rc = DIE_OK;
  for (int r = 0; r < nrhs; ++r) {
    if (brk[r]) rc = std::min(rc, (int)DIE_E_BREAKDOWN);
    else if (!conv[r] && rc == DIE_OK) rc = DIE_NOT_CONVERGED;
    if (info) {
      info[r].status = brk[r] ? DIE_E_BREAKDOWN : (conv[r] ? DIE_OK : DIE_NOT_CONVERGED);
      info[r].iters = iters[r];
      info[r].products_A = pa[r];
      info[r].products_AR = par[r];
      info[r].cycles = cyc[r];
      info[r].rel_res_true = relres[r];
      info[r].finish_iters = 0;
    }
  }
  if (rc == DIE_E_BREAKDOWN) return fail(DIE_E_BREAKDOWN, "Krylov solver met a non-finite value");
  return rc;
}

// ------------------------------------------------------------------ block GMRES
// Scratch of the block products: the projection's chunk products (accumulation type) and the
// Gram matrices' chunk partials (complex FP64).
constexpr size_t kTsqPartial = (size_t)1 << 25;
constexpr size_t kGramPartial = (size_t)1 << 20;

// Host <-> device transfers of a small column-major matrix (rows x cols, leading dimension
// = rows on the device) in the precision of T.
template <class T> int download(const void* d, int rows, int cols, die::la::Mat& M, hipStream_t st) {
  std::vector<c2<T>> h((size_t)rows * cols);
  DIE_HIP(hipMemcpyAsync(h.data(), d, h.size() * sizeof(c2<T>), hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  M = die::la::Mat(rows, cols);
  for (size_t e = 0; e < h.size(); ++e) M.a[e] = cd((double)h[e].x, (double)h[e].y);
  return DIE_OK;
}
template <class T> int upload(const die::la::Mat& M, void* d, hipStream_t st, std::vector<c2<T>>& stage) {
  stage.resize(M.a.size());
  for (size_t e = 0; e < M.a.size(); ++e) stage[e] = die::mk<T>((T)M.a[e].real(), (T)M.a[e].imag());
  DIE_HIP(hipMemcpyAsync(d, stage.data(), stage.size() * sizeof(c2<T>), hipMemcpyHostToDevice, st));
  DIE_HIP(hipStreamSynchronize(st));  // the staging vector is reused by the next upload
  return DIE_OK;
}

// CholQR of a new block: one pass when the smallest pivot of the unit-diagonal Gram's Cholesky is
// at least this (the second pass of CholQR2 otherwise)
constexpr double kCholQRSinglePivot = 0.05;

// Page-locked host memory (hipHostMalloc), released with the owner.
struct PinnedBuf {
  void* p = nullptr;
  size_t cap = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  int alloc(size_t bytes) {  // at least `bytes`, keeping a large enough earlier allocation
    if (p && cap >= bytes) return DIE_OK;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    if (hipHostMalloc(&p, bytes, hipHostMallocDefault) != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(DIE_E_NOMEM, "hipHostMalloc failed");
    }
    cap = bytes;
    return DIE_OK;
  }
};

// Events recorded once per block step (created on first use, reused by later cycles and calls).
struct EventRing {
  std::vector<hipEvent_t> ev;
  EventRing() = default;
  EventRing(const EventRing&) = delete;
  EventRing& operator=(const EventRing&) = delete;
  ~EventRing() {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
  }
  int ensure(int n) {
    while ((int)ev.size() < n) {
      hipEvent_t e = nullptr;
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        return fail(DIE_E_HIP, "hipEventCreateWithFlags failed");
      }
      ev.push_back(e);
    }
    return DIE_OK;
  }
};

struct BlockWork {
  DBuf Rs, Sd, partn, nrm, active, Vb, Wt, Zb, Tm, Ra, Tb, sm, sm2, Ht, Hls, Bls, ones, idxd, part, coef, cnt, scl, Uq,
      sq;
  // the device CholQR of each block step: the first factor (FP64), the steps' flags (device and a
  // page-locked copy the host reads one step later) and the steps' events
  DBuf Rf, Fl;
  PinnedBuf pflag;
  EventRing ev;
  // the planar Gram-Schmidt on the matrix cores: the basis shadows (T1, T2), the block being
  // orthogonalised (planar in the basis precision) and its T1 copy, the projection's chunk
  // products and their two-stage sums, the real update matrix, the FP64 planar copy of the first
  // block and the Gram result
  DBuf Q1, Q2, Wacc, W1, Cpart, Csum, Hbm, P64, Gd;
  DBuf Zall;                 // per right-hand side: the correction V Y of its last cycle (FP64)
  std::vector<char> zvalid;  // which columns of Zall hold one
  DBuf Ubest, bmask;         // best iterate so far per right-hand side, and the copy mask
};

// Frees the buffers that scale with the basis (kept: the per-right-hand-side corrections and best
// iterates); the next block solve allocates them again at the size it needs.
void release_block_basis(BlockWork& bw) {
  for (DBuf* b : {&bw.Vb, &bw.Wt, &bw.Zb, &bw.Tm, &bw.Tb, &bw.Ra, &bw.Q1, &bw.Q2, &bw.Wacc, &bw.W1, &bw.P64})
    b->release();
}

// Buffers of the planar Gram-Schmidt for element type E (basis precision T): nrow padded rows,
// column capacity ccap of the basis shadows, block width at most pw.
template <class T, class E>
int planar_alloc(BlockWork& bw, size_t nrow, size_t ccap, int pw) {
  using A = typename die::GemmTile<E>::Acc;
  static_assert(std::is_same<A, T>::value, "the planar block is held in the basis precision");
  const size_t cols = die::gemm_pad((size_t)2 * pw);
  DIE_TRY(bw.Q1.alloc(nrow * ccap * sizeof(E)));
  DIE_TRY(bw.Q2.alloc(nrow * ccap * sizeof(E)));
  DIE_TRY(bw.Wacc.alloc(nrow * cols * sizeof(A)));
  DIE_TRY(bw.W1.alloc(nrow * cols * sizeof(E)));
  DIE_TRY(bw.Cpart.alloc(kTsqPartial * sizeof(A)));
  DIE_TRY(bw.Csum.alloc(die::kTsqScratch * sizeof(double)));
  DIE_TRY(bw.Hbm.alloc(ccap * 2 * pw * sizeof(E)));
  DIE_TRY(bw.P64.alloc(nrow * cols * sizeof(double)));
  DIE_TRY(bw.Gd.alloc((size_t)die::kPanelMaxCols * die::kPanelMaxCols * sizeof(double2)));
  return DIE_OK;
}

// Block j (n x p) of the basis into columns [2 p j, 2 p (j + 1)) of both shadows.
template <class T, class E>
int planar_shadow(BlockWork& bw, const c2<T>* X, size_t n, int p, int j, size_t nrow, size_t ccap, hipStream_t st) {
  using A = typename die::GemmTile<E>::Acc;
  DIE_HIP((die::launch_tsq_split<T, A, E>(X, n, n, p, 2 * p * j, nrow, ccap, nullptr, 0, bw.Q1.as<E>(), bw.Q2.as<E>(),
                                          st)));
  return DIE_OK;
}

// npass block classical Gram-Schmidt passes of W (n x p) against the first nq basis columns on
// the matrix cores: per pass H_pass = Q^H W (nq x p, rounded to E) and W -= Q H_pass as real
// products of the planar shadows.  W is split into the planar Wacc (basis precision; planar_in:
// the product wrote it there) and stays there, its T1 copy remade for each projection; the caller's
// CholQR factor application reads it planar and writes the complex block.
template <class T, class E>
int planar_block_cgs(die_te_ctx* c, BlockWork& bw, const c2<T>* W, size_t n, int nq, int p, int npass, size_t nrow,
                     size_t ccap, c2<T>* const* H, hipStream_t st, bool planar_in = false) {
  using A = typename die::GemmTile<E>::Acc;
  A* Ws = bw.Wacc.as<A>();
  E* W1 = bw.W1.as<E>();
  const int M = 2 * nq, P2 = 2 * p, ldhb = (int)die::gemm_pad((size_t)M);
  if (planar_in)  // the product wrote W planar into Wacc already
    DIE_HIP((die::launch_tsq_to_t1<A, E>(Ws, nrow, nrow, P2, W1, st)));
  else
    DIE_HIP((die::launch_tsq_split<T, A, E>(W, n, n, p, 0, nrow, ccap, Ws, nrow, W1, nullptr, st)));
  for (int pass = 0; pass < npass; ++pass) {
    if (pass > 0) DIE_HIP((die::launch_tsq_to_t1<A, E>(Ws, nrow, nrow, P2, W1, st)));
    int nch = 0;
    DIE_HIP((die::launch_tsq_proj<E>(bw.Q1.as<E>(), M, W1, P2, nrow, bw.Cpart.as<A>(), kTsqPartial, &nch, st)));
    DIE_HIP((die::launch_tsq_combine<A, E, T>(bw.Cpart.as<A>(), nch, nq, p, H[pass], bw.Hbm.as<E>(), ldhb,
                                              bw.Csum.as<double>(), die::kTsqScratch, st)));
    // flops 8 n p nq; operands: Q (n x 2nq) and Hb read, Ws (n x 2p) read and written
    ProfScope prof(c, DIE_PROF_GEMM, st, 8.0 * (double)n * p * nq,
                   (double)sizeof(E) * ((double)n * M + (double)M * P2) + 2.0 * sizeof(A) * (double)n * P2);
    DIE_HIP((die::launch_tsq_update<E>(bw.Q2.as<E>(), M, ccap, nrow, bw.Hbm.as<E>(), ldhb, P2, Ws, nrow, st)));
  }
  return DIE_OK;
}

// G = X^H X (p x p <= 64 x 64) of the complex block held planar in Xs (nrow rows), downloaded to
// the host (FP64 sums of products in A).
template <class A>
int gram_planar_dev(BlockWork& bw, const A* Xs, size_t nrow, int p, hipStream_t st, const int* gate = nullptr) {
  DIE_HIP(die::launch_gram_planar<A>(Xs, nrow, p, bw.Cpart.as<A>(), kTsqPartial, bw.Csum.as<double>(),
                                     die::kTsqScratch, bw.Gd.as<double2>(), st, gate));
  return DIE_OK;
}
template <class A>
int gram_planar(BlockWork& bw, const A* Xs, size_t nrow, int p, die::la::Mat& G, hipStream_t st) {
  DIE_TRY(gram_planar_dev<A>(bw, Xs, nrow, p, st));
  return download<double>(bw.Gd.p, p, p, G, st);
}
// The same for a complex block X (n x p, leading dimension n): split into planar Xs first.
template <class T>
int gram_complex(BlockWork& bw, const c2<T>* X, size_t n, size_t nrow, int p, T* Xs, die::la::Mat& G, hipStream_t st) {
  DIE_HIP((die::launch_tsq_split<T, T, T>(X, n, n, p, 0, nrow, 32, Xs, nrow, nullptr, nullptr, st)));
  return gram_planar<T>(bw, Xs, nrow, p, G, st);
}

// A narrowed block (at most this many right-hand sides of an object left) starts its cycle from
// the residuals and the previous cycle's corrections of the same right-hand sides.
constexpr int kAugmentMax = 16;

// Restarted block GMRES(m) (Section 4's GMRES applied to all right-hand sides of an object
// at once): per object (in groups of at most kPanelMaxCols right-hand sides), the active
// residuals (normalised) span the first block through a rank-revealing (pivoted) Cholesky QR;
// block Arnoldi with CGS2 on the matrix cores and CholQR2 for each new block; the block least
// squares once per cycle on the GPU (panel Householder QR and a triangular solve); every cycle
// restarts from the FP64 true residual, as in the per-rhs solver.  Objects are processed one
// after another.
template <class T>
int block_gmres_solve(die_te_ctx* c, const double2* b, double2* u, int nrhs, const die_te_solve_opts& o,
                      die_te_solve_info* info, hipStream_t st, std::vector<char>* stalled = nullptr,
                      const std::vector<char>* only = nullptr) {
  using die::la::Mat;
  namespace la = die::la;
  const size_t n = c->nvec;
  const int m = o.restart;
  const int nblk = die::blas_blocks(n);
  const bool reg = c->regularize != 0;
  const bool defl = c->r > 0;
  const int rpo = nrhs / c->nobj;  // right-hand sides per object
  // the widest block the buffers hold: rpo, or the most right-hand sides of one object in `only`
  // (the only ones iterated when it is given), at most kPanelMaxCols (wider sets run in groups)
  int pw = rpo;
  if (only) {
    pw = 1;
    for (int ob = 0; ob < c->nobj; ++ob) {
      int cntv = 0;
      for (int r = ob * rpo; r < (ob + 1) * rpo; ++r) cntv += (*only)[r] ? 1 : 0;
      pw = std::max(pw, cntv);
    }
  }
  pw = std::min(pw, die::kPanelMaxCols);
  const double tol = o.tol > 0 ? o.tol : 1e-8;
  const double chol_tol = std::is_same<T, float>::value ? 1e-6 : 1e-12;  // rank test of a new block
  const double rank_tau2 = 1e-12;  // initial block: drop residual directions below 1e-6 (unit columns)
  const int npass = o.orth == 1 ? 1 : 2;  // block CGS passes against the previous blocks
  if ((size_t)n > (size_t)INT32_MAX || (size_t)(m + 1) * pw > 65535)
    return fail(DIE_E_INVALID, "block GMRES: vectors or blocks too large");
  if ((size_t)m * pw > (size_t)die::kTrsmMaxRows)
    return fail(DIE_E_INVALID, "block GMRES: restart times block width exceeds the device least squares (" +
                                   std::to_string(die::kTrsmMaxRows) + ")");
  const int ldh = (m + 1) * pw;
  const size_t dbytes = (size_t)nrhs * n * sizeof(double2);
  // work buffers live in the context, so repeated calls (restarted solves, batches) reuse them
  if (!c->bw) c->bw = std::make_shared<BlockWork>();
  BlockWork& bw = *c->bw;
  DBuf &Rs = bw.Rs, &Sd = bw.Sd, &partn = bw.partn, &nrm = bw.nrm, &active = bw.active, &Vb = bw.Vb, &Wt = bw.Wt,
       &Zb = bw.Zb, &Tm = bw.Tm, &Ra = bw.Ra, &Tb = bw.Tb, &sm = bw.sm, &sm2 = bw.sm2, &Ht = bw.Ht, &Hls = bw.Hls,
       &Bls = bw.Bls, &ones = bw.ones, &idxd = bw.idxd, &part = bw.part, &coef = bw.coef, &cnt = bw.cnt,
       &scl = bw.scl, &Uq = bw.Uq, &sq = bw.sq;
  DIE_TRY(Rs.alloc(dbytes));
  if (reg) DIE_TRY(Sd.alloc(dbytes));
  DIE_TRY(partn.alloc((size_t)nrhs * nblk * sizeof(double)));
  DIE_TRY(nrm.alloc(nrhs * sizeof(double)));
  DIE_TRY(active.alloc(nrhs * sizeof(int)));
  DIE_TRY(Vb.alloc((size_t)(m + 1) * pw * n * sizeof(c2<T>)));
  DIE_TRY(Wt.alloc((size_t)pw * n * sizeof(c2<T>)));
  if (defl) DIE_TRY(Zb.alloc((size_t)pw * n * sizeof(c2<T>)));
  if (reg) DIE_TRY(Tm.alloc((size_t)pw * n * sizeof(c2<T>)));
  DIE_TRY(Ra.alloc((size_t)2 * pw * n * sizeof(double2)));  // residual block, then its orthonormal basis
  DIE_TRY(Tb.alloc((size_t)pw * n * sizeof(c2<T>)));
  DIE_TRY(sm.alloc((size_t)ldh * pw * sizeof(double2)));
  DIE_TRY(sm2.alloc((size_t)ldh * pw * sizeof(c2<T>)));
  DIE_TRY(Ht.alloc((size_t)ldh * m * pw * sizeof(c2<T>)));
  DIE_TRY(Hls.alloc((size_t)ldh * m * pw * sizeof(double2)));
  DIE_TRY(Bls.alloc((size_t)ldh * pw * sizeof(double2)));
  DIE_TRY(ones.alloc(sizeof(double)));
  DIE_TRY(idxd.alloc(pw * sizeof(int)));
  DIE_TRY(scl.alloc(pw * sizeof(double)));
  // the planar Gram-Schmidt: binary16 shadows with block = 2 (complex64 only), else the basis
  // precision
  const bool hgemm = std::is_same<T, float>::value && o.block == 2;
  const size_t nrow = die::gemm_pad(n), ccap = die::gemm_pad((size_t)2 * (m + 1) * pw);
  if constexpr (std::is_same<T, float>::value) {
    if (hgemm)
      DIE_TRY((planar_alloc<T, _Float16>(bw, nrow, ccap, pw)));
    else
      DIE_TRY((planar_alloc<T, T>(bw, nrow, ccap, pw)));
  } else {
    DIE_TRY((planar_alloc<T, T>(bw, nrow, ccap, pw)));
  }
  // rows n .. nrow - 1 of the planar block stay zero (the products write rows below n only)
  if (nrow > n) DIE_HIP(hipMemsetAsync(bw.Wacc.p, 0, bw.Wacc.bytes, st));
  auto shadow = [&](const c2<T>* X, int p, int j) -> int {
    if constexpr (std::is_same<T, float>::value)
      if (hgemm) return planar_shadow<T, _Float16>(bw, X, n, p, j, nrow, ccap, st);
    return planar_shadow<T, T>(bw, X, n, p, j, nrow, ccap, st);
  };
  DIE_TRY(Uq.alloc((size_t)die::kPanelMaxRows * die::kPanelMaxCols * sizeof(double2)));  // panel reflectors
  DIE_TRY(sq.alloc(die::kPanelMaxCols * sizeof(double)));
  // the device CholQR of the block steps: first factor, per-step flags and events
  DIE_TRY(bw.Rf.alloc((size_t)die::kCholQRMax * die::kCholQRMax * sizeof(double2)));
  DIE_TRY(bw.Fl.alloc((size_t)8 * m * sizeof(int)));
  DIE_TRY(bw.pflag.alloc((size_t)8 * m * sizeof(int)));
  DIE_TRY(bw.ev.ensure(m));
  const int* pflag = (const int*)bw.pflag.p;
  if (defl) {
    DIE_TRY(part.alloc((size_t)pw * std::max((size_t)c->r * nblk, die::gmres_part_elems(n, c->r)) *
                       sizeof(double2)));
    DIE_TRY(coef.alloc((size_t)pw * c->r * sizeof(double2)));
    DIE_TRY(cnt.alloc((size_t)pw * die::kCounterStride * sizeof(int)));
    DIE_HIP(hipMemsetAsync(cnt.p, 0, (size_t)pw * die::kCounterStride * sizeof(int), st));
  }
  const double one = 1.0;
  DIE_HIP(hipMemcpyAsync(ones.p, &one, sizeof(double), hipMemcpyHostToDevice, st));
  {  // pick the FFT pass variants before any timing-sensitive work
    const int* pv = nullptr;
    DIE_TRY(fft_plan<T>(c, pw, st, &pv));
    DIE_TRY(fft_plan<double>(c, nrhs, st, &pv));
  }
  DIE_TRY(ensure_work(c, std::max(work_bytes(c, nrhs, sizeof(double2)), work_bytes(c, pw, sizeof(c2<T>))), st));
  c2<T>* vb = Vb.as<c2<T>>();
  std::vector<c2<T>> stage;
  std::vector<double> bnorm(nrhs), rnorm(nrhs), snorm(nrhs), hn(nrhs), relres(nrhs, 1.0);
  std::vector<int> act(nrhs, 1), iters(nrhs, 0), pa(nrhs, 0), par(nrhs, 0), cycles(nrhs, 0), conv(nrhs, 0),
      brk(nrhs, 0);
  std::vector<char> full_cycle(c->nobj, 0);  // per object: its last cycle ran all m block steps
  DIE_TRY(bw.Zall.alloc((size_t)nrhs * n * sizeof(double2)));
  // corrections kept from an earlier call serve only its continuation (a call given x0)
  if (bw.zvalid.size() != (size_t)nrhs || !o.x0_given) bw.zvalid.assign(nrhs, 0);
  // best iterate so far (returned when the tolerance is not reached)
  DIE_TRY(bw.Ubest.alloc(dbytes));
  DIE_TRY(bw.bmask.alloc((size_t)nrhs * sizeof(int)));
  std::vector<double> best(nrhs, std::numeric_limits<double>::infinity());
  std::vector<int> bm(nrhs, 0);
  bool first_check = true;
  // the records of every right-hand side as they stand (also before a breakdown return)
  auto fill_info = [&]() {
    if (!info) return;
    for (int r = 0; r < nrhs; ++r) {
      info[r].status = brk[r] ? DIE_E_BREAKDOWN : (conv[r] ? DIE_OK : DIE_NOT_CONVERGED);
      info[r].iters = iters[r];
      info[r].products_A = pa[r];
      info[r].products_AR = par[r];
      info[r].cycles = cycles[r];
      info[r].rel_res_true = relres[r];
      info[r].finish_iters = 0;
    }
  };
  if (only)
    for (int r = 0; r < nrhs; ++r) act[r] = (*only)[r] ? 1 : 0;
  if (!o.x0_given) DIE_HIP(hipMemsetAsync(u, 0, dbytes, st));
  DIE_HIP((die::launch_norm2<double>(b, n, n, nrhs, partn.as<double>(), nullptr, st)));
  DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), nullptr, st));
  DIE_HIP(hipMemcpyAsync(hn.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  for (int r = 0; r < nrhs; ++r) {
    bnorm[r] = std::sqrt(hn[r]);
    if (!std::isfinite(bnorm[r])) return fail(DIE_E_INVALID, "e_in contains non-finite values");
  }
  for (;;) {
    // ---- FP64 true residual res = b - A u
    DIE_HIP(hipMemcpyAsync(active.p, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    const int* dact = active.as<int>();
    double2* res = Rs.as<double2>();
    DIE_TRY(apply_op<double>(c, u, res, nrhs, false, dact, st, rpo));
    DIE_HIP((die::launch_maxpy<double, double, double>(2, (const double2*)nullptr, 0, 0, 0, nullptr, nullptr, 0, b, n,
                                                       1.0, res, n, -1.0, n, nrhs, nullptr, partn.as<double>(), dact,
                                                       st)));
    DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), dact, st));
    DIE_HIP(hipMemcpyAsync(hn.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    int nact = 0, nfb = 0;
    for (int r = 0; r < nrhs; ++r) {
      if (!act[r]) continue;
      pa[r] += 1;
      rnorm[r] = std::sqrt(hn[r]);
      const double before = relres[r];
      relres[r] = bnorm[r] > 0 ? rnorm[r] / bnorm[r] : 0.0;
      if (first_check && o.x0_given && !(std::isfinite(rnorm[r]) && rnorm[r] < bnorm[r])) {
        // a given guess that is non-finite or no better than zero is replaced by zero
        DIE_HIP(hipMemsetAsync(u + (size_t)r * n, 0, n * sizeof(double2), st));
        bw.zvalid[r] = 0;
        relres[r] = 1.0;
        ++nfb;
      } else if (!std::isfinite(rnorm[r])) {
        brk[r] = 1;
        act[r] = 0;
        bw.zvalid[r] = 0;
      } else if (relres[r] <= tol || bnorm[r] == 0.0) {
        conv[r] = 1;
        act[r] = 0;
      } else if (iters[r] >= o.max_iters) {
        act[r] = 0;
      } else if (stalled && full_cycle[r / rpo] && relres[r] > 0.9 * before) {
        // a full cycle took this residual down by less than 10%: the inner precision limits it
        // (its condition times the FP32 rounding nears one); the caller finishes it in FP64
        (*stalled)[r] = 1;
        act[r] = 0;
      } else {
        ++nact;
      }
    }
    first_check = false;
    if (nfb) continue;  // residuals of the zeroed guesses
    if (nact == 0) break;
    DIE_HIP(hipMemcpyAsync(active.p, act.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
    const double2* s = res;
    if (reg) {
      DIE_TRY(apply_op<double>(c, res, Sd.as<double2>(), nrhs, true, dact, st, rpo));
      s = Sd.as<double2>();
      for (int r = 0; r < nrhs; ++r) par[r] += act[r];
    }
    DIE_HIP((die::launch_norm2<double>(s, n, n, nrhs, partn.as<double>(), dact, st)));
    DIE_HIP(die::launch_reduce_norm(partn.as<double>(), nblk, nrhs, nrm.as<double>(), dact, st));
    DIE_HIP(hipMemcpyAsync(hn.data(), nrm.p, nrhs * sizeof(double), hipMemcpyDeviceToHost, st));
    DIE_HIP(hipStreamSynchronize(st));
    nact = 0;
    for (int r = 0; r < nrhs; ++r) {
      snorm[r] = std::sqrt(hn[r]);
      if (!act[r]) continue;
      if (!std::isfinite(snorm[r])) {
        brk[r] = 1;
        act[r] = 0;
      } else if (!(snorm[r] > 0)) {
        act[r] = 0;  // regularized residual vanished: nothing a cycle can do (as in the per-rhs solver)
      } else {
        ++nact;
      }
    }
    if (nact == 0) break;
    // the iterates about to be corrected are kept when they are the best ones so far
    {
      int nb = 0;
      for (int r = 0; r < nrhs; ++r) {
        bm[r] = act[r] && relres[r] < best[r];
        if (bm[r]) {
          best[r] = relres[r];
          ++nb;
        }
      }
      if (nb) {
        DIE_HIP(hipMemcpyAsync(bw.bmask.p, bm.data(), nrhs * sizeof(int), hipMemcpyHostToDevice, st));
        DIE_HIP((die::launch_scale<double, double>(u, n, bw.Ubest.as<double2>(), n, ones.as<double>(), 0, n, nrhs,
                                                   bw.bmask.as<int>(), st)));
      }
    }
    bool progress = false;  // some object took a block step this cycle
    // the work units of this cycle: per object, its active right-hand sides in groups of at most pw
    std::vector<std::pair<int, std::vector<int>>> groups;
    for (int ob = 0; ob < c->nobj; ++ob) {
      std::vector<int> Kall;
      for (int r = ob * rpo; r < (ob + 1) * rpo; ++r)
        if (act[r] && snorm[r] > 0 && std::isfinite(snorm[r])) Kall.push_back(r);
      for (size_t g0 = 0; g0 < Kall.size(); g0 += (size_t)pw)
        groups.emplace_back(ob, std::vector<int>(Kall.begin() + g0, Kall.begin() + std::min(Kall.size(), g0 + pw)));
    }
    for (const auto& grp : groups) {
      const int ob = grp.first;
      const std::vector<int>& K = grp.second;
      const int k = (int)K.size();
      // ---- first block: normalised residuals, rank-revealing Cholesky QR (two passes, FP64)
      double2* ra = Ra.as<double2>();
      double2* v0 = ra + (size_t)pw * n;
      std::vector<double> inv(k);
      for (int q = 0; q < k; ++q) {
        DIE_HIP(hipMemcpyAsync(ra + (size_t)q * n, s + (size_t)K[q] * n, n * sizeof(double2), hipMemcpyDeviceToDevice,
                               st));
        inv[q] = 1.0 / snorm[K[q]];
      }
      DIE_HIP(hipMemcpyAsync(scl.p, inv.data(), k * sizeof(double), hipMemcpyHostToDevice, st));
      DIE_HIP((die::launch_scale<double, double>(ra, n, ra, n, scl.as<double>(), 1, n, k, nullptr, st)));
      // a narrowed block also takes its right-hand sides' previous corrections (a restart that keeps
      // the last error approximation, against stagnation): extra columns of the first block that
      // carry no right-hand side of their own
      int kt = k;
      if (k <= kAugmentMax)
        for (int q = 0; q < k && kt < pw; ++q)
          if (bw.zvalid[K[q]]) {
            DIE_HIP(hipMemcpyAsync(ra + (size_t)kt * n, bw.Zall.as<double2>() + (size_t)K[q] * n,
                                   n * sizeof(double2), hipMemcpyDeviceToDevice, st));
            ++kt;
          }
      Mat G, L;
      double* p64 = bw.P64.as<double>();
      DIE_TRY(gram_complex<double>(bw, ra, n, nrow, kt, p64, G, st));
      std::vector<double> dz(kt, 1.0);  // the correction columns enter with unit norm
      for (int i = k; i < kt; ++i) {
        const double g = G(i, i).real();
        dz[i] = (g > 0.0 && std::isfinite(g)) ? 1.0 / std::sqrt(g) : 0.0;
      }
      for (int j = 0; j < kt; ++j)
        for (int i = 0; i < kt; ++i) G(i, j) *= dz[i] * dz[j];
      std::vector<int> perm;
      const int p = la::pivoted_cholesky(G, rank_tau2, L, perm);
      if (p == 0) continue;
      Mat R1(p, p);
      for (int j = 0; j < p; ++j)
        for (int i = 0; i <= j; ++i) R1(i, j) = std::conj(L(j, i));
      const Mat R1i = la::upper_inverse(R1);
      Mat Msel(kt, p), S0(p, k);
      for (int i = 0; i < p; ++i)
        for (int j = 0; j < p; ++j) Msel(perm[i], j) = R1i(i, j) * dz[perm[i]];
      // the k right-hand sides (columns 0 .. k-1, wherever the pivoting put them) in the p pivots
      for (int i = 0; i < kt; ++i)
        if (perm[i] < k)
          for (int q = 0; q < p; ++q) S0(q, perm[i]) = std::conj(L(i, q));
      std::vector<double2> stage64;
      DIE_TRY(upload<double>(Msel, sm.p, st, stage64));
      DIE_HIP(die::launch_cplx_rmul<double>(ra, n, kt, sm.as<double2>(), kt, p, n, v0, n, st));
      Mat G2, R2;
      DIE_TRY(gram_complex<double>(bw, v0, n, nrow, p, p64, G2, st));
      if (!la::chol_upper_scaled(G2, 1e-14, R2)) continue;  // not expected after the pivoted selection
      DIE_TRY(upload<double>(la::upper_inverse(R2), sm.p, st, stage64));
      DIE_HIP(die::launch_cplx_rmul<double>(v0, n, p, sm.as<double2>(), p, p, n, ra, n, st));
      {
        Mat S(p, k);
        for (int j = 0; j < k; ++j)
          for (int i = 0; i < p; ++i) {
            cd a = 0.0;
            for (int q = i; q < p; ++q) a += R2(i, q) * S0(q, j);
            S(i, j) = a;
          }
        S0 = S;
      }
      DIE_HIP((die::launch_scale<double, T>(ra, n, vb, n, ones.as<double>(), 0, n, p, nullptr, st)));
      DIE_TRY(shadow(vb, p, 0));
      // ---- block Arnoldi: H ((m+1) p x m p, on the device in the basis precision, leading
      // dimension ldhp), CGS2 on the matrix cores, CholQR2 of every new block
      const int ldhp = (m + 1) * p;
      c2<T>* Hd = Ht.as<c2<T>>();
      DIE_HIP(hipMemsetAsync(Hd, 0, (size_t)ldhp * m * p * sizeof(c2<T>), st));
      int meff = m;
      bool early = false;
      for (int j = 0; j < m; ++j) {
        c2<T>* Vj = vb + (size_t)j * p * n;
        c2<T>* W = vb + (size_t)(j + 1) * p * n;
        const c2<T>* z = Vj;
        if (defl) {
          // rpo = p: every field of the block uses object ob's V and C
          DIE_TRY(apply_pinv<T>(c, Vj, Zb.as<c2<T>>(), p, part.as<double2>(), coef.as<double2>(), cnt.as<int>(), nullptr,
                                st, p, ob));
          z = Zb.as<c2<T>>();
        }
        // the product of the new block goes planar into Wacc (its complex form is made only after
        // the Gram-Schmidt passes and CholQR, by the factor application into W)
        DIE_TRY(apply_M<T>(c, reg, z, reg ? Tm.as<c2<T>>() : nullptr, W, p, nullptr, st, 0, ob, bw.Wacc.as<T>(),
                           nrow));
        const int nq = (j + 1) * p;
        c2<T>* hc[2] = {sm.as<c2<T>>(), sm2.as<c2<T>>()};  // the projections (nq x p each)
        if constexpr (std::is_same<T, float>::value) {
          if (hgemm)
            DIE_TRY((planar_block_cgs<T, _Float16>(c, bw, W, n, nq, p, npass, nrow, ccap, hc, st, true)));
          else
            DIE_TRY((planar_block_cgs<T, T>(c, bw, W, n, nq, p, npass, nrow, ccap, hc, st, true)));
        } else {
          DIE_TRY((planar_block_cgs<T, T>(c, bw, W, n, nq, p, npass, nrow, ccap, hc, st, true)));
        }
        // column block j of H: the sum of the projections
        if (npass == 2)
          DIE_HIP(die::launch_cadd2<T>(hc[0], nq, hc[1], nq, nq, p, Hd + (size_t)j * p * ldhp, ldhp, st));
        else
          DIE_HIP(hipMemcpy2DAsync(Hd + (size_t)j * p * ldhp, ldhp * sizeof(c2<T>), hc[0], nq * sizeof(c2<T>),
                                   nq * sizeof(c2<T>), p, hipMemcpyDeviceToDevice, st));
        // CholQR of the orthogonalised block (planar in Wacc) without a host round trip: its Gram,
        // the factor and its inverse by one workgroup, the factor application into W (one pass) or
        // Wt (two passes: the second Gram, factor and application then run, gated on the device),
        // and H(j + 1, j) (= R1, or R2 R1) straight into H.  The host reads the step's flags one
        // step later, when the next step is already queued behind it.
        T* ws = bw.Wacc.as<T>();
        int* fl = bw.Fl.as<int>() + (size_t)8 * j;
        double2* r1 = bw.Rf.as<double2>();
        c2<T>* wt = Wt.as<c2<T>>();
        c2<T>* hblk = Hd + (size_t)j * p * ldhp + (size_t)(j + 1) * p;
        DIE_TRY(gram_planar_dev<T>(bw, ws, nrow, p, st));
        DIE_HIP(die::launch_cholqr_factor<T>(bw.Gd.as<double2>(), p, chol_tol, kCholQRSinglePivot, 1, r1, sm.as<c2<T>>(),
                                             fl, hblk, ldhp, st));
        DIE_HIP(die::launch_cplx_rmul_planar<T>(ws, nrow, p, sm.as<c2<T>>(), p, p, n, W, n, st, fl, wt));
        DIE_HIP((die::launch_tsq_split<T, T, T>(wt, n, n, p, 0, nrow, 32, ws, nrow, nullptr, nullptr, st, fl + 2)));
        DIE_TRY(gram_planar_dev<T>(bw, ws, nrow, p, st, fl + 2));
        DIE_HIP(die::launch_cholqr_factor<T>(bw.Gd.as<double2>(), p, chol_tol, kCholQRSinglePivot, 2, r1,
                                             sm2.as<c2<T>>(), fl, hblk, ldhp, st));
        DIE_HIP(die::launch_cplx_rmul<T>(wt, n, p, sm2.as<c2<T>>(), p, p, n, W, n, st, fl + 4, W));
        // a block that could not be orthonormalised is cleared: the next step, queued before the
        // host sees the flag, then works on zeros (an unwritten block could hold non-finite values,
        // and 0 x NaN in its updates would reach the zero padding rows of the planar buffers)
        DIE_HIP(die::launch_zero_unless<T>(W, n, n, p, fl + 3, st));
        DIE_HIP(hipMemcpyAsync((int*)bw.pflag.p + (size_t)8 * j, fl, 8 * sizeof(int), hipMemcpyDeviceToHost, st));
        DIE_HIP(hipEventRecord(bw.ev.ev[j], st));
        DIE_TRY(shadow(W, p, j + 1));
        // the previous step's block: a numerically dependent one ends the cycle before it (this
        // step's work, already queued, is then never used)
        if (j > 0) {
          DIE_HIP(hipEventSynchronize(bw.ev.ev[j - 1]));
          if (!pflag[8 * (j - 1) + 3]) {
            meff = j;
            early = true;
            break;
          }
        }
      }
      if (!early) {
        DIE_HIP(hipEventSynchronize(bw.ev.ev[m - 1]));
        if (!pflag[8 * (m - 1) + 3]) {
          meff = m;
          early = true;
        }
      }
      // ---- block least squares min || E1 S0 - H Y || on the GPU, then u += P^-1 V Y
      const int mr = early ? meff * p : (meff + 1) * p, nc = meff * p;
      {
        Mat Bm(mr, k);
        for (int j = 0; j < k; ++j)
          for (int i = 0; i < p; ++i) Bm(i, j) = S0(i, j);
        // H (mr x nc) to FP64 with leading dimension mr: column j is "right-hand side" j of the scale kernel
        DIE_HIP((die::launch_scale<T, double>(Hd, ldhp, Hls.as<double2>(), mr, ones.as<double>(), 0, mr, nc, nullptr,
                                              st)));
        DIE_TRY(upload<double>(Bm, Bls.p, st, stage64));
        // Householder QR panel by panel (H has at most p sub-diagonals), then R Y = Q^H B
        DIE_HIP(die::launch_block_hessenberg_qr(Hls.as<double2>(), mr, mr, nc, p, Bls.as<double2>(), mr, k,
                                                Uq.as<double2>(), sq.as<double>(), st));
        DIE_HIP(die::launch_trsm_upper(Hls.as<double2>(), mr, nc, Bls.as<double2>(), mr, k, st));
        Mat Y;
        DIE_TRY(download<double>(Bls.p, mr, k, Y, st));
        bool finite = true;
        for (int j = 0; j < k && finite; ++j)
          for (int i = 0; i < nc; ++i)
            if (!std::isfinite(Y(i, j).real()) || !std::isfinite(Y(i, j).imag())) finite = false;
        if (!finite) {
          for (int q = 0; q < k; ++q) brk[K[q]] = 1;
          fill_info();
          return fail(DIE_E_BREAKDOWN, "block GMRES: rank-deficient block Hessenberg");
        }
        Mat Ys(nc, k);  // columns scaled back by the residual norms
        for (int j = 0; j < k; ++j)
          for (int i = 0; i < nc; ++i) Ys(i, j) = Y(i, j) * snorm[K[j]];
        DIE_TRY(upload<T>(Ys, sm.p, st, stage));
      }
      c2<T>* tb = Tb.as<c2<T>>();
      DIE_HIP(die::launch_cplx_rmul<T>(vb, n, nc, sm.as<c2<T>>(), nc, k, n, tb, n, st));
      // keep each right-hand side's correction V Y (before the projector) for a later narrowed block
      for (int q = 0; q < k; ++q) {
        DIE_HIP((die::launch_scale<T, double>(tb + (size_t)q * n, n, bw.Zall.as<double2>() + (size_t)K[q] * n, n,
                                              ones.as<double>(), 0, n, 1, nullptr, st)));
        bw.zvalid[K[q]] = 1;
      }
      if (defl)
        DIE_TRY(apply_pinv<T>(c, tb, tb, k, part.as<double2>(), coef.as<double2>(), cnt.as<int>(), nullptr, st, k, ob));
      DIE_HIP(hipMemcpyAsync(idxd.p, K.data(), k * sizeof(int), hipMemcpyHostToDevice, st));
      DIE_HIP(die::launch_add_cols<T>(tb, n, idxd.as<int>(), k, u, st));
      DIE_HIP(hipStreamSynchronize(st));  // K and the staging vectors are reused by the next object
      const int prods = (meff * p + k - 1) / k;
      full_cycle[ob] = meff == m;
      progress = true;
      for (int q = 0; q < k; ++q) {
        const int r = K[q];
        iters[r] += meff;
        cycles[r] += 1;
        pa[r] += prods;
        if (reg) par[r] += prods;
      }
    }
    if (!progress) {
      for (int r = 0; r < nrhs; ++r)
        if (act[r]) brk[r] = 1;
      fill_info();
      return fail(DIE_E_BREAKDOWN, "block GMRES: no residual block could be orthonormalised");
    }
  }
  // right-hand sides that stopped short of the tolerance get their best iterate back
  DIE_TRY(restore_best(u, bw.Ubest.as<double2>(), n, nrhs, conv, brk, best, relres, bm, bw.bmask.as<int>(),
                       ones.as<double>(), st));
  int rc = DIE_OK;
  for (int r = 0; r < nrhs; ++r) {
    if (brk[r]) rc = std::min(rc, (int)DIE_E_BREAKDOWN);
    else if (!conv[r] && rc == DIE_OK) rc = DIE_NOT_CONVERGED;
  }
  fill_info();
  if (rc == DIE_E_BREAKDOWN) return fail(DIE_E_BREAKDOWN, "block GMRES met a non-finite value");
  return rc;
}

int check_ctx(const die_te_ctx* c) {
  if (!c) return fail(DIE_E_INVALID, "null context");
  return DIE_OK;
}

}  // namespace

// ====================================================================== C ABI
extern "C" {

const char* die_te_last_error(void) { return die_host::last_error().c_str(); }

int die_te_setup_multi(die_te_ctx** out, const die_te_grid* gr, int nobj, const void* eps_r,
                       const die_te_setup_opts* opts, void* stream) {
  die_host::last_error().clear();
  if (!out || !gr || !eps_r) return fail(DIE_E_INVALID, "null argument");
  if (nobj < 1 || nobj > 65536) return fail(DIE_E_INVALID, "nobj must be in [1, 65536]");
  *out = nullptr;
  hipStream_t st = (hipStream_t)stream;
  if (gr->nx < 1 || gr->ny < 1 || gr->nx > 2048 || gr->ny > 2048)
    return fail(DIE_E_INVALID, "nx, ny must be in [1, 2048]");
  if (!(gr->h > 0) || !std::isfinite(gr->h)) return fail(DIE_E_INVALID, "h must be positive and finite");
  const double k = gr->k_b == 0 ? 2.0 * M_PI : gr->k_b;
  if (!(k > 0) || !std::isfinite(k)) return fail(DIE_E_INVALID, "k_b must be positive and finite");
  const int px = gr->px ? gr->px : auto_pad(gr->nx);
  const int py = gr->py ? gr->py : auto_pad(gr->ny);
  if (!is_pow2(px) || !is_pow2(py) || px < 2 || py < 2 || px > 4096 || py > 4096 || px < 2 * gr->nx - 1 ||
      py < 2 * gr->ny - 1)
    return fail(DIE_E_INVALID, "px, py must be powers of two in [max(2, 2n-1), 4096]");
  die_te_setup_opts o{};
  if (opts) o = *opts;
  if (o.deflate_k < -1) return fail(DIE_E_INVALID, "deflate_k must be >= -1");
  if (o.deflate_max < 0) return fail(DIE_E_INVALID, "deflate_max must be >= 0");
  if (o.fft_variant < 0 || o.fft_variant > die::kFftVariants)
    return fail(DIE_E_INVALID, "fft_variant must be 0 (autotune) or 1 + v with v in [0, 3]");
  if (o.polarization != 0 && o.polarization != 1) return fail(DIE_E_INVALID, "polarization must be 0 (TE) or 1 (TM)");
  if (o.magnetic != 0 && o.magnetic != 1) return fail(DIE_E_INVALID, "magnetic must be 0 or 1");
  if (o.polarization == 1 && (o.magnetic || o.mu_r))
    return fail(DIE_E_INVALID, "the TM operator has no magnetic contrast option (E3 only)");
  if (o.mu_r && !o.magnetic) return fail(DIE_E_INVALID, "mu_r needs magnetic = 1 (the E1, E2, H3 system)");
  if (o.polarization == 1 && o.regularize)
    return fail(DIE_E_INVALID, "the TM operator is identity plus compact: no regularizer (regularize must be 0)");

  auto* c = new (std::nothrow) die_te_ctx();
  if (!c) return fail(DIE_E_NOMEM, "host allocation failed");
  auto guard = [&](int rc) {
    if (rc < 0) delete c;
    return rc;
  };
  if (hipGetDevice(&c->dev) != hipSuccess) return guard(fail(DIE_E_HIP, "hipGetDevice failed"));
  {  // device address of this device's static scratch (die_te_matvec_noalloc), once per device
    const hipError_t es = die::scratch_init(c->dev);
    if (es != hipSuccess)
      return guard(fail(DIE_E_HIP, std::string("looking up the static scratch array failed: ") + hipGetErrorString(es)));
  }
  c->nx = gr->nx; c->ny = gr->ny; c->px = px; c->py = py;
  c->lpx = ilog2(px); c->lpy = ilog2(py);
  c->h = gr->h; c->k = k;
  c->ncell = (size_t)gr->nx * gr->ny;
  c->ncomp = o.polarization == 1 ? 1 : (o.magnetic ? 3 : 2);
  c->nvec = (size_t)c->ncomp * c->ncell;
  c->nobj = nobj;
  c->regularize = o.regularize ? 1 : 0;
  c->fft_force = o.fft_variant - 1;
  const size_t ncells = c->ncell * (size_t)nobj;

  // contrast (eq. ElectricContrast) and regularizer contrast (eq. InverseSymbol)
  std::vector<double2> eps(ncells);
  if (hipMemcpyAsync(eps.data(), eps_r, ncells * sizeof(double2), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return guard(fail(DIE_E_HIP, "reading eps_r failed (is it a device pointer?)"));
  std::vector<double2> chi(ncells), chir(ncells);
  std::vector<float2> chi32(ncells), chir32(ncells);
  for (size_t e = 0; e < ncells; ++e) {
    const cd ev(eps[e].x, eps[e].y);
    if (!std::isfinite(ev.real()) || !std::isfinite(ev.imag()))
      return guard(fail(DIE_E_INVALID, "eps_r contains non-finite values"));
    if (ev == cd(0.0, 0.0))
      return guard(fail(DIE_E_SINGULAR, "eps_r == 0 at cell " + std::to_string(e % c->ncell) + " of object " +
                                            std::to_string(e / c->ncell) + ": no solution exists"));
    const cd x = ev - 1.0, xr = 1.0 / ev - 1.0;
    chi[e] = make_double2(x.real(), x.imag());
    chir[e] = make_double2(xr.real(), xr.imag());
    chi32[e] = make_float2((float)x.real(), (float)x.imag());
    chir32[e] = make_float2((float)xr.real(), (float)xr.imag());
  }
  int rc;
  if ((rc = c->chi64.alloc(ncells * sizeof(double2))) < 0 || (rc = c->chir64.alloc(ncells * sizeof(double2))) < 0 ||
      (rc = c->chi32.alloc(ncells * sizeof(float2))) < 0 || (rc = c->chir32.alloc(ncells * sizeof(float2))) < 0)
    return guard(rc);
  if (hipMemcpyAsync(c->chi64.p, chi.data(), ncells * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->chir64.p, chir.data(), ncells * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->chi32.p, chi32.data(), ncells * sizeof(float2), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipMemcpyAsync(c->chir32.p, chir32.data(), ncells * sizeof(float2), hipMemcpyHostToDevice, st) != hipSuccess)
    return guard(fail(DIE_E_HIP, "uploading the contrast failed"));
  if (c->ncomp == 3) {
    // magnetic contrast chi_m = mu_r - 1 (eq. ElectricContrast's magnetic counterpart) and the
    // regularizer's chi_m' = 1/mu_r - 1; mu_r == NULL: no magnetic contrast (H3 then follows E)
    std::vector<double2> mu(ncells, make_double2(1.0, 0.0));
    if (o.mu_r && (hipMemcpyAsync(mu.data(), o.mu_r, ncells * sizeof(double2), hipMemcpyDeviceToHost, st) != hipSuccess ||
                   hipStreamSynchronize(st) != hipSuccess))
      return guard(fail(DIE_E_HIP, "reading mu_r failed (is it a device pointer?)"));
    std::vector<double2> cm(ncells), cmr(ncells);
    std::vector<float2> cm32(ncells), cmr32(ncells);
    for (size_t e = 0; e < ncells; ++e) {
      const cd mv(mu[e].x, mu[e].y);
      if (!std::isfinite(mv.real()) || !std::isfinite(mv.imag()))
        return guard(fail(DIE_E_INVALID, "mu_r contains non-finite values"));
      if (mv == cd(0.0, 0.0))
        return guard(fail(DIE_E_SINGULAR, "mu_r == 0 at cell " + std::to_string(e % c->ncell)));
      const cd x = mv - 1.0, xr = 1.0 / mv - 1.0;
      cm[e] = make_double2(x.real(), x.imag());
      cmr[e] = make_double2(xr.real(), xr.imag());
      cm32[e] = make_float2((float)x.real(), (float)x.imag());
      cmr32[e] = make_float2((float)xr.real(), (float)xr.imag());
    }
    if ((rc = c->chim64.alloc(ncells * sizeof(double2))) < 0 || (rc = c->chimr64.alloc(ncells * sizeof(double2))) < 0 ||
        (rc = c->chim32.alloc(ncells * sizeof(float2))) < 0 || (rc = c->chimr32.alloc(ncells * sizeof(float2))) < 0)
      return guard(rc);
    if (hipMemcpyAsync(c->chim64.p, cm.data(), ncells * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->chimr64.p, cmr.data(), ncells * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->chim32.p, cm32.data(), ncells * sizeof(float2), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(c->chimr32.p, cmr32.data(), ncells * sizeof(float2), hipMemcpyHostToDevice, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return guard(fail(DIE_E_HIP, "uploading the magnetic contrast failed"));
  }

  // Green tensor, circulant embedding, symbol = FFT2 / (px py) on the GPU
  {
    std::vector<cd> planes;
    const int npl = die::sym_planes(c->ncomp);
    die::green::embed(c->nx, c->ny, px, py, c->h, c->k, c->ncomp, planes);
    const size_t plane = (size_t)px * py;
    DBuf E, W;
    if ((rc = E.alloc(npl * plane * sizeof(double2))) < 0 || (rc = W.alloc(npl * plane * sizeof(double2))) < 0)
      return guard(rc);
    if (hipMemcpyAsync(E.p, planes.data(), npl * plane * sizeof(double2), hipMemcpyHostToDevice, st) != hipSuccess)
      return guard(fail(DIE_E_HIP, "uploading the Green tensor failed"));
    if ((rc = c->sym64.alloc(npl * plane * sizeof(double2))) < 0 ||
        (rc = c->sym32.alloc(npl * plane * sizeof(float2))) < 0)
      return guard(rc);
    hipError_t e1 = die::launch_rows_fwd<double, double>(c->lpx, false, E.as<double2>(), nullptr, nullptr,
                                                         W.as<double2>(), px, py, npl, 1, 0, 0, nullptr, st);
    hipError_t e2 = die::launch_cols_plain<double>(c->lpy, false, W.as<double2>(), px, npl, st);
    hipError_t e3 = die::launch_pack_symbol(W.as<double2>(), c->sym64.as<double2>(), c->sym32.as<float2>(), px, py,
                                            npl, 1.0 / ((double)px * (double)py), st);
    if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || hipStreamSynchronize(st) != hipSuccess)
      return guard(fail(DIE_E_HIP, "symbol transform failed"));
  }
  // slots for nslot objects with r vectors each, cleared (zero vectors leave P^-1 unchanged)
  auto alloc_deflation = [&](int nslot, int r) -> int {
    int e;
    if ((e = c->V.alloc((size_t)nslot * r * c->nvec * sizeof(double2))) < 0 ||
        (e = c->Cdev.alloc((size_t)nslot * r * r * sizeof(double2))) < 0)
      return e;
    if (hipMemsetAsync(c->V.p, 0, (size_t)nslot * r * c->nvec * sizeof(double2), st) != hipSuccess ||
        hipMemsetAsync(c->Cdev.p, 0, (size_t)nslot * r * r * sizeof(double2), st) != hipSuccess)
      return fail(DIE_E_HIP, "clearing the deflation data failed");
    c->Chost.assign((size_t)nslot * r * r, cd(0, 0));
    c->ritz.assign((size_t)nslot * r, cd(0, 0));
    c->r = r;
    return DIE_OK;
  };
  std::vector<int> want(nobj, o.deflate_k);  // eigenpairs wanted per object
  if (o.deflate_k == -1) {
    // automatic size (Section 5): the deflation radius R of each object from its contrast, then
    // r doubled from 16 until fewer than r of the r largest Ritz values lie beyond R
    const int rcap = (int)std::min<size_t>(o.deflate_max > 0 ? (size_t)o.deflate_max : 256, c->nvec / 2);
    if (rcap < 1) return guard(fail(DIE_E_INVALID, "automatic deflation needs 2 nx ny >= 2"));
    c->radius.assign(nobj, 1.0);
    for (int ob = 0; ob < nobj; ++ob) {
      // TM: no dense segments; the paper deflates every eigenvalue outside the unit circle
      const double R = c->ncomp == 1 ? 1.0
                                     : die_host::deflation_radius(eps.data() + (size_t)ob * c->ncell, c->ncell,
                                                                  c->regularize != 0);
      c->radius[ob] = R;
      for (int rt = std::min(16, rcap);; rt = std::min(2 * rt, rcap)) {
        if ((rc = alloc_deflation(1, rt)) < 0) return guard(rc);
        rc = run_eigs(c, ob, 0, rt, o.eigs_tol, o.eigs_krylov, o.eigs_max_restarts, o.seed, st);
        if (rc < 0) return guard(rc);
        int beyond = 0;
        for (int i = 0; i < rt; ++i) beyond += std::abs(c->ritz[i]) > R ? 1 : 0;
        want[ob] = beyond;
        if (beyond < rt || rt >= rcap) break;
      }
    }
  } else if (o.deflate_k > 0 && (size_t)o.deflate_k >= c->nvec) {
    return guard(fail(DIE_E_INVALID, "deflate_k must be < 2 nx ny"));
  }
  const int rdef = *std::max_element(want.begin(), want.end());
  c->r = 0;
  if (rdef > 0) {
    if ((rc = alloc_deflation(nobj, rdef)) < 0) return guard(rc);
    int conv = rdef;
    for (int ob = 0; ob < nobj; ++ob) {
      if (want[ob] <= 0) continue;
      rc = run_eigs(c, ob, ob, want[ob], o.eigs_tol, o.eigs_krylov, o.eigs_max_restarts, o.seed, st);
      if (rc < 0) return guard(rc);
      conv = std::min(conv, c->eigs_converged);
    }
    c->eigs_converged = conv;
  } else {
    c->V.release();
    c->Cdev.release();
    c->Chost.clear();
    c->ritz.clear();
  }
  *out = c;
  return DIE_OK;
}

int die_te_setup(die_te_ctx** out, const die_te_grid* gr, const void* eps_r, const die_te_setup_opts* opts,
                 void* stream) {
  return die_te_setup_multi(out, gr, 1, eps_r, opts, stream);
}

static int product(die_te_ctx* c, const void* x, void* y, int nrhs, int prec, void* stream, bool reg) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!x || !y || nrhs < 1) return fail(DIE_E_INVALID, "null pointer or nrhs < 1");
  if (x == y) return fail(DIE_E_INVALID, "x and y must not overlap");
  if (nrhs % c->nobj) return fail(DIE_E_INVALID, "nrhs must be a multiple of the number of objects");
  hipStream_t st = (hipStream_t)stream;
  const int rpo = nrhs / c->nobj;
  if (prec == DIE_C128) return apply_op<double>(c, (const double2*)x, (double2*)y, nrhs, reg, nullptr, st, rpo);
  if (prec == DIE_C64) return apply_op<float>(c, (const float2*)x, (float2*)y, nrhs, reg, nullptr, st, rpo);
  return fail(DIE_E_INVALID, "prec must be DIE_C128 or DIE_C64");
}

int die_te_matvec(die_te_ctx* c, const void* x, void* y, int nrhs, int prec, void* stream) {
  return product(c, x, y, nrhs, prec, stream, false);
}

int die_te_matvec_noalloc(die_te_ctx* c, const void* x, void* y, int nrhs, int prec, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!x || !y || nrhs < 1) return fail(DIE_E_INVALID, "null pointer or nrhs < 1");
  if (x == y) return fail(DIE_E_INVALID, "x and y must not overlap");
  if (nrhs % c->nobj) return fail(DIE_E_INVALID, "nrhs must be a multiple of the number of objects");
  if (prec != DIE_C128 && prec != DIE_C64) return fail(DIE_E_INVALID, "prec must be DIE_C128 or DIE_C64");
  const size_t es = prec == DIE_C128 ? sizeof(double2) : sizeof(float2);
  const size_t need = work_bytes(c, nrhs, es);
  if (need > die::kScratchBytes)
    return fail(DIE_E_INVALID, "die_te_matvec_noalloc: the FFT intermediate (" + std::to_string(need) +
                                   " bytes) exceed the static scratch of " + std::to_string(die::kScratchBytes) +
                                   " bytes");
  int cur = -1;
  DIE_HIP(hipGetDevice(&cur));
  if (cur != c->dev) return fail(DIE_E_INVALID, "the context's device must be the current device");
  void* W = die::scratch_ptr(c->dev);
  if (!W) return fail(DIE_E_HIP, "the static scratch of this device was not looked up at setup");
  // pass variants without tuning (tuning allocates): those a product of this batch-size class
  // already uses, else the forced variant, else the radix tuned for the grid with the full tile
  const int pi = prec == DIE_C128 ? 0 : 1, bc = batch_class(nrhs);
  int v[3] = {0, 0, 0};
  if (c->fftv[pi][bc][0] >= 0) {
    for (int p = 0; p < 3; ++p) v[p] = c->fftv[pi][bc][p];
  } else if (c->fft_force >= 0) {
    v[0] = v[1] = v[2] = c->fft_force;
  } else {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(TuneKey{c->dev, pi, c->lpx, c->lpy, c->nx, c->ny, c->ncomp});
    if (it != g_tune.end())
      for (int p = 0; p < 3; ++p) v[p] = std::max(it->second.radix[p], 0);
  }
  hipStream_t st = (hipStream_t)stream;
  const int rpo = nrhs / c->nobj;
  for (int pass = 0; pass < 3; ++pass) {
    if (prec == DIE_C128)
      DIE_HIP(launch_pass<double>(c, pass, v[pass], (const double2*)x, (double2*)y, (double2*)W, nrhs, nullptr, st,
                                  rpo, chi_of<double>(c, false), chi2_of<double>(c, false)));
    else
      DIE_HIP(launch_pass<float>(c, pass, v[pass], (const float2*)x, (float2*)y, (float2*)W, nrhs, nullptr, st, rpo,
                                 chi_of<float>(c, false), chi2_of<float>(c, false)));
  }
  return DIE_OK;
}

int die_te_regularize(die_te_ctx* c, const void* x, void* y, int nrhs, int prec, void* stream) {
  return product(c, x, y, nrhs, prec, stream, true);
}

int die_te_solve(die_te_ctx* c, const void* e_in, void* e_tot, int nrhs, const die_te_solve_opts* opts,
                 die_te_solve_info* info, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!e_in || !e_tot || nrhs < 1 || !opts) return fail(DIE_E_INVALID, "null pointer or nrhs < 1");
  if (e_in == e_tot) return fail(DIE_E_INVALID, "e_in and e_tot must not overlap");
  if (nrhs % c->nobj) return fail(DIE_E_INVALID, "nrhs must be a multiple of the number of objects");
  die_te_solve_opts o = *opts;
  if (o.restart < 1 || o.restart > (o.block ? 65534 : 510))
    return fail(DIE_E_INVALID, "restart must be in [1, 510] (block solver: [1, 65534])");
  if (o.orth != 0 && o.orth != 1) return fail(DIE_E_INVALID, "orth must be 0 (CGS2) or 1 (one-reduction CGS2)");
  if (o.max_iters < 1) return fail(DIE_E_INVALID, "max_iters must be >= 1");
  if (o.tol < 0 || !std::isfinite(o.tol)) return fail(DIE_E_INVALID, "tol must be >= 0");
  hipStream_t st = (hipStream_t)stream;
  if (o.mixed < 0 || o.mixed > 2) return fail(DIE_E_INVALID, "mixed must be 0, 1 or 2");
  if (o.mixed == 2 && o.orth != 1) return fail(DIE_E_INVALID, "mixed = 2 (binary16 basis) needs orth = 1");
  if (o.block < 0 || o.block > 2) return fail(DIE_E_INVALID, "block must be 0, 1 or 2");
  if (o.method < 0 || o.method > 3)
    return fail(DIE_E_INVALID, "method must be 0 (GMRES), 1 (Bi-CGSTAB), 2 (GCR) or 3 (IDR(s))");
  if (o.method) {
    if (o.block || o.mixed)
      return fail(DIE_E_INVALID, "Bi-CGSTAB, GCR and IDR(s) run per right-hand side in FP64 (block = mixed = 0)");
    if (o.method == 3 && o.restart > 64) return fail(DIE_E_INVALID, "IDR(s): s = restart must be <= 64");
    return alt_solve(c, (const double2*)e_in, (double2*)e_tot, nrhs, o, info, st);
  }
  if (o.block) {
    if (o.mixed == 2) return fail(DIE_E_INVALID, "block GMRES needs mixed = 0 or 1");
    if (o.block == 2 && o.mixed != 1) return fail(DIE_E_INVALID, "block = 2 (binary16 GEMMs) needs mixed = 1");
    if (!o.mixed) return block_gmres_solve<double>(c, (const double2*)e_in, (double2*)e_tot, nrhs, o, info, st);
    // complex64 cycles with FP64 refinement; right-hand sides whose FP32 cycles stall (a full cycle
    // gains less than 10%) are finished by FP64 block cycles from the fields reached, with buffers
    // sized for them alone
    std::vector<char> stalled(nrhs, 0);
    // records the solver did not reach (an error return) read as errors, never as converged
    die_te_solve_info unset{};
    unset.status = DIE_E_HIP;
    unset.rel_res_true = std::numeric_limits<double>::quiet_NaN();
    std::vector<die_te_solve_info> i32(nrhs, unset);
    int rc = block_gmres_solve<float>(c, (const double2*)e_in, (double2*)e_tot, nrhs, o, i32.data(), st, &stalled);
    int used = -1;
    for (int r = 0; r < nrhs; ++r)
      if (stalled[r]) used = std::max(used, i32[r].iters);
    if (rc >= 0 && used >= 0) {
      if (used < o.max_iters) {
        // the complex64 basis and its shadows make room for the FP64 ones (the corrections kept
        // for augmented restarts and the best iterates stay)
        DIE_HIP(hipStreamSynchronize(st));
        if (c->bw) release_block_basis(*c->bw);
        die_te_solve_opts o64 = o;
        o64.mixed = 0;
        o64.block = 1;
        o64.x0_given = 1;
        o64.max_iters = o.max_iters - used;
        std::vector<die_te_solve_info> i64(nrhs, unset);
        rc = block_gmres_solve<double>(c, (const double2*)e_in, (double2*)e_tot, nrhs, o64, i64.data(), st,
                                       nullptr, &stalled);
        for (int r = 0; r < nrhs; ++r) {
          if (!stalled[r]) continue;
          i32[r].status = i64[r].status;
          i32[r].iters += i64[r].iters;
          i32[r].products_A += i64[r].products_A;
          i32[r].products_AR += i64[r].products_AR;
          i32[r].cycles += i64[r].cycles;
          i32[r].rel_res_true = i64[r].rel_res_true;
          i32[r].finish_iters = i64[r].iters;
        }
      } else {
        for (int r = 0; r < nrhs; ++r)
          if (stalled[r]) i32[r].status = DIE_NOT_CONVERGED;
      }
      if (rc >= 0) {
        rc = DIE_OK;
        for (int r = 0; r < nrhs; ++r)
          if (i32[r].status != DIE_OK) rc = DIE_NOT_CONVERGED;
      }
    }
    if (info)
      for (int r = 0; r < nrhs; ++r) info[r] = i32[r];
    return rc;
  }
  if (o.mixed == 2)
    return gmres_solve<float, _Float16>(c, (const double2*)e_in, (double2*)e_tot, nrhs, o, info, st);
  if (o.mixed) return gmres_solve<float>(c, (const double2*)e_in, (double2*)e_tot, nrhs, o, info, st);
  return gmres_solve<double>(c, (const double2*)e_in, (double2*)e_tot, nrhs, o, info, st);
}

int die_te_solve_batch(die_te_ctx* const* ctx, int nctx, const void* const* e_in, void* const* e_tot,
                       const int* nrhs, const die_te_solve_opts* opts, die_te_solve_info* const* info,
                       void* stream) {
  die_host::last_error().clear();
  if (!ctx || !e_in || !e_tot || !nrhs || !opts || nctx < 1)
    return fail(DIE_E_INVALID, "null pointer or nctx < 1");
  for (int i = 0; i < nctx; ++i) {
    if (!ctx[i]) return fail(DIE_E_INVALID, "context " + std::to_string(i) + " is null");
    for (int k = 0; k < i; ++k)
      if (ctx[k] == ctx[i]) return fail(DIE_E_INVALID, "context " + std::to_string(i) + " is listed twice");
  }
  DIE_HIP(hipStreamSynchronize((hipStream_t)stream));  // the caller's queued work (inputs) is complete
  struct Result {
    int rc = DIE_OK;
    std::string msg;
  };
  std::vector<Result> res(nctx);
  auto run = [&](int i) {
    die_te_ctx* c = ctx[i];
    hipStream_t s = nullptr;
    if (hipSetDevice(c->dev) != hipSuccess || hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      res[i] = {DIE_E_HIP, "stream creation failed"};
      return;
    }
    res[i].rc = die_te_solve(c, e_in[i], e_tot[i], nrhs[i], opts, info ? info[i] : nullptr, s);
    res[i].msg = die_host::last_error();
    // timing brackets recorded on this stream are read back before it goes away
    if (prof_resolve(c) != DIE_OK && res[i].rc >= 0) res[i] = {DIE_E_HIP, die_host::last_error()};
    (void)hipStreamDestroy(s);
  };
  std::vector<std::thread> th;
  th.reserve(nctx);
  for (int i = 0; i < nctx; ++i) th.emplace_back(run, i);
  for (auto& t : th) t.join();
  for (int i = 0; i < nctx; ++i)
    if (res[i].rc < 0) return fail(res[i].rc, "context " + std::to_string(i) + ": " + res[i].msg);
  for (int i = 0; i < nctx; ++i)
    if (res[i].rc != DIE_OK) return res[i].rc;
  return DIE_OK;
}

int die_te_fft_plan(die_te_ctx* c, int prec, int nrhs, int* variants, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!variants || nrhs < 1) return fail(DIE_E_INVALID, "null variants or nrhs < 1");
  if (prec != DIE_C128 && prec != DIE_C64) return fail(DIE_E_INVALID, "prec must be DIE_C128 or DIE_C64");
  const int* v = nullptr;
  if (prec == DIE_C128) DIE_TRY(fft_plan<double>(c, nrhs, (hipStream_t)stream, &v));
  else DIE_TRY(fft_plan<float>(c, nrhs, (hipStream_t)stream, &v));
  for (int p = 0; p < 3; ++p) variants[p] = v[p];
  return DIE_OK;
}

int die_te_apply_deflation(die_te_ctx* c, const void* x, void* y, int nrhs, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (c->r <= 0) return fail(DIE_E_INVALID, "the context has no deflation basis");
  if (!x || !y || nrhs < 1) return fail(DIE_E_INVALID, "null pointer or nrhs < 1");
  if (nrhs % c->nobj) return fail(DIE_E_INVALID, "nrhs must be a multiple of the number of objects");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = c->nvec;
  const int nblk = die::blas_blocks(n);
  DBuf part, coef, cnt;
  DIE_TRY(part.alloc((size_t)nrhs * std::max((size_t)c->r * nblk, die::gmres_part_elems(n, c->r)) *
                     sizeof(double2)));
  DIE_TRY(coef.alloc((size_t)nrhs * c->r * sizeof(double2)));
  DIE_TRY(cnt.alloc((size_t)nrhs * die::kCounterStride * sizeof(int)));
  DIE_HIP(hipMemsetAsync(cnt.p, 0, (size_t)nrhs * die::kCounterStride * sizeof(int), st));
  DIE_TRY(apply_pinv<double>(c, (const double2*)x, (double2*)y, nrhs, part.as<double2>(), coef.as<double2>(),
                             cnt.as<int>(), nullptr, st, nrhs / c->nobj));
  DIE_HIP(hipStreamSynchronize(st));  // part/coef are freed on return
  return DIE_OK;
}

int die_te_operator_dense(die_te_ctx* c, int which, int obj, void* out, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!out) return fail(DIE_E_INVALID, "null out");
  if (which < 0 || which > 3) return fail(DIE_E_INVALID, "which must be 0 (A), 1 (A_R), 2 (A_R A) or 3 (M P^-1)");
  if (obj < 0 || obj >= c->nobj) return fail(DIE_E_INVALID, "obj out of range");
  hipStream_t st = (hipStream_t)stream;
  const size_t n = c->nvec;
  // columns in batches: the identity columns e_j, then the operator on them (object obj)
  const int nb = (int)std::min<size_t>(n, 256);
  const int nblk = die::blas_blocks(n);
  DBuf X, T1, T2, part, coef, cnt;
  DIE_TRY(X.alloc((size_t)nb * n * sizeof(double2)));
  DIE_TRY(T1.alloc((size_t)nb * n * sizeof(double2)));
  if (which == 3 && c->r > 0) {
    DIE_TRY(T2.alloc((size_t)nb * n * sizeof(double2)));
    DIE_TRY(part.alloc((size_t)nb * std::max((size_t)c->r * nblk, die::gmres_part_elems(n, c->r)) * sizeof(double2)));
    DIE_TRY(coef.alloc((size_t)nb * c->r * sizeof(double2)));
    DIE_TRY(cnt.alloc((size_t)nb * die::kCounterStride * sizeof(int)));
    DIE_HIP(hipMemsetAsync(cnt.p, 0, (size_t)nb * die::kCounterStride * sizeof(int), st));
  }
  const bool reg = c->regularize != 0;
  for (size_t c0 = 0; c0 < n; c0 += (size_t)nb) {
    const int k = (int)std::min<size_t>((size_t)nb, n - c0);
    double2* y = (double2*)out + c0 * n;
    double2* x = X.as<double2>();
    DIE_HIP(die::launch_unit_cols(x, n, c0, k, st));
    switch (which) {
      case 0:
        DIE_TRY(apply_op<double>(c, x, y, k, false, nullptr, st, k, obj));
        break;
      case 1:
        DIE_TRY(apply_op<double>(c, x, y, k, true, nullptr, st, k, obj));
        break;
      case 2:
        DIE_TRY(apply_M<double>(c, true, x, T1.as<double2>(), y, k, nullptr, st, k, obj));
        break;
      default: {
        const double2* z = x;
        if (c->r > 0) {
          DIE_TRY(apply_pinv<double>(c, x, T2.as<double2>(), k, part.as<double2>(), coef.as<double2>(), cnt.as<int>(),
                                     nullptr, st, k, obj));
          z = T2.as<double2>();
        }
        DIE_TRY(apply_M<double>(c, reg, z, T1.as<double2>(), y, k, nullptr, st, k, obj));
      }
    }
  }
  DIE_HIP(hipStreamSynchronize(st));  // the batch buffers are freed on return
  return DIE_OK;
}

int die_te_spectrum(die_te_ctx* c, int which, int obj, void* eig, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!eig) return fail(DIE_E_INVALID, "null eig");
  const size_t n = c->nvec;
  if (n > (size_t)kSpectrumMaxOrder)
    return fail(DIE_E_INVALID, "the dense eigenvalue problem is limited to " + std::to_string(kSpectrumMaxOrder) +
                                   " unknowns (the host QR iteration is O(n^3))");
  hipStream_t st = (hipStream_t)stream;
  DBuf D;
  DIE_TRY(D.alloc(n * n * sizeof(double2)));
  DIE_TRY(die_te_operator_dense(c, which, obj, D.p, stream));
  die::la::Mat A((int)n, (int)n);
  DIE_HIP(hipMemcpyAsync(A.a.data(), D.p, n * n * sizeof(double2), hipMemcpyDeviceToHost, st));
  DIE_HIP(hipStreamSynchronize(st));
  die::la::Mat Z0;  // no Schur vectors: eigenvalues only
  die::la::hessenberg(A, Z0);
  if (!die::la::schur(A, Z0)) return fail(DIE_E_BREAKDOWN, "spectrum: QR iteration did not converge");
  cd* e = (cd*)eig;
  for (size_t i = 0; i < n; ++i) e[i] = A((int)i, (int)i);
  return DIE_OK;
}

int die_te_deflation_info(die_te_ctx* c, int* r, void* ritz, void* V, void* C, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!r) return fail(DIE_E_INVALID, "null r");
  *r = c->r;
  hipStream_t st = (hipStream_t)stream;
  const size_t no = (size_t)c->nobj;
  if (ritz && c->r > 0) std::memcpy(ritz, c->ritz.data(), no * c->r * sizeof(cd));
  if (C && c->r > 0) std::memcpy(C, c->Chost.data(), no * c->r * c->r * sizeof(cd));
  if (V && c->r > 0) {
    DIE_HIP(hipMemcpyAsync(V, c->V.p, no * c->r * c->nvec * sizeof(double2), hipMemcpyDeviceToDevice, st));
    DIE_HIP(hipStreamSynchronize(st));
  }
  return DIE_OK;
}

int die_te_fft2(void* data, int px, int py, int batch, int inverse, int prec, void* stream) {
  die_host::last_error().clear();
  if (!data || batch < 1) return fail(DIE_E_INVALID, "null data or batch < 1");
  if (!is_pow2(px) || !is_pow2(py) || px < 2 || py < 2 || px > 4096 || py > 4096)
    return fail(DIE_E_INVALID, "px, py must be powers of two in [2, 4096]");
  hipStream_t st = (hipStream_t)stream;
  const size_t plane = (size_t)px * py;
  const bool inv = inverse != 0;
  DBuf W;
  if (prec == DIE_C128) {
    DIE_TRY(W.alloc(batch * plane * sizeof(double2)));
    DIE_HIP((die::launch_rows_fwd<double, double>(ilog2(px), inv, (const double2*)data, nullptr, nullptr, W.as<double2>(), px,
                                                  py, batch, 1, 0, 0, nullptr, st)));
    DIE_HIP(die::launch_cols_plain<double>(ilog2(py), inv, W.as<double2>(), px, batch, st));
    DIE_HIP(die::launch_transpose<double>(W.as<double2>(), (double2*)data, px, py, batch, st));
  } else if (prec == DIE_C64) {
    DIE_TRY(W.alloc(batch * plane * sizeof(float2)));
    DIE_HIP((die::launch_rows_fwd<float, float>(ilog2(px), inv, (const float2*)data, nullptr, nullptr, W.as<float2>(), px, py,
                                                batch, 1, 0, 0, nullptr, st)));
    DIE_HIP(die::launch_cols_plain<float>(ilog2(py), inv, W.as<float2>(), px, batch, st));
    DIE_HIP(die::launch_transpose<float>(W.as<float2>(), (float2*)data, px, py, batch, st));
  } else {
    return fail(DIE_E_INVALID, "prec must be DIE_C128 or DIE_C64");
  }
  DIE_HIP(hipStreamSynchronize(st));
  return DIE_OK;
}

int die_te_profile(die_te_ctx* c, int enable) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  c->prof_on = enable > 0;
  if (enable > 0) {
    c->prof_every = enable;
    for (size_t& u : c->prof_used) u = 0;
    for (auto& sn : c->prof_seen) sn = 0;
    for (double& b : c->prof_bytes) b = 0;
    for (double& b : c->prof_mem) b = 0;
    for (double& b : c->prof_ms) b = 0;
    for (size_t& r : c->prof_resolved) r = 0;
  }
  return DIE_OK;
}

int die_te_profile_read(die_te_ctx* c, int kind, long long* launches, long long* seen, double* total_ms,
                        double* bytes) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (kind < 0 || kind > 3 || !launches || !total_ms) return fail(DIE_E_INVALID, "bad profile kind or null output");
  if (seen) *seen = (long long)c->prof_seen[kind];
  if (bytes) *bytes = c->prof_bytes[kind];
  DIE_TRY(prof_resolve(c));
  *launches = (long long)c->prof_used[kind];
  *total_ms = c->prof_ms[kind];
  return DIE_OK;
}

int die_te_profile_mem(die_te_ctx* c, int kind, double* mem_bytes) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (kind < 0 || kind > 3 || !mem_bytes) return fail(DIE_E_INVALID, "bad profile kind or null output");
  *mem_bytes = c->prof_mem[kind];
  return DIE_OK;
}

int die_te_warm_start(die_te_ctx* c, die_te_unet* net, const void* e_in, void* x0, int nrhs, void* stream) {
  die_host::last_error().clear();
  DIE_TRY(check_ctx(c));
  if (!net || !e_in || !x0 || nrhs < 1) return fail(DIE_E_INVALID, "null argument or nrhs < 1");
  if (nrhs % c->nobj) return fail(DIE_E_INVALID, "nrhs must be a multiple of the number of objects");
  if (e_in == x0) return fail(DIE_E_INVALID, "e_in and x0 must not overlap");
  if (c->ncomp != 2) return fail(DIE_E_INVALID, "the warm-start network serves the TE (E1, E2) system only");
  return die_host::unet_guess(net, c->chi64.as<double2>(), nrhs / c->nobj, (const double2*)e_in, (double2*)x0, nrhs,
                              c->ny, c->nx, (hipStream_t)stream);
}

int die_te_destroy(die_te_ctx* c) {
  die_host::last_error().clear();
  if (!c) return DIE_OK;
  (void)hipDeviceSynchronize();
  delete c;
  return DIE_OK;
}

}  // extern "C"
