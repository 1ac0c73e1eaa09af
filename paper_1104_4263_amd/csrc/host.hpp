// Host-side helpers shared by the library's translation units: the per-thread error
// message behind die_te_last_error(), HIP error checks and an owning device buffer.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "die_te.h"

namespace die_host {

// The message of the most recent error return in the calling thread (defined in die_te.cpp).
std::string& last_error();

inline int fail(int code, const std::string& msg) {
  last_error() = msg;
  return code;
}

// Owning device allocation; alloc() keeps the current block when it is large enough.
struct DBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DBuf() = default;
  DBuf(const DBuf&) = delete;
  DBuf& operator=(const DBuf&) = delete;
  DBuf(DBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  DBuf& operator=(DBuf&& o) noexcept {
    if (this != &o) {
      release();
      p = o.p;
      bytes = o.bytes;
      o.p = nullptr;
      o.bytes = 0;
    }
    return *this;
  }
  ~DBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  int alloc(size_t b) {
    if (b <= bytes && p) return DIE_OK;
    release();
    if (b == 0) b = 16;
    hipError_t e = hipMalloc(&p, b);
    if (e != hipSuccess) {
      p = nullptr;
      (void)hipGetLastError();
      return fail(e == hipErrorOutOfMemory ? DIE_E_NOMEM : DIE_E_HIP,
                  "hipMalloc(" + std::to_string(b) + " bytes): " + hipGetErrorString(e));
    }
    bytes = b;
    return DIE_OK;
  }
  template <class X> X* as() const { return static_cast<X*>(p); }
};

// Section 5's deflation radius of eps_r[0 .. ncells) (complex128), with (regularized) or
// without the regularizer (plan.cpp).
double deflation_radius(const double2* eps, size_t ncells, bool regularized);

}  // namespace die_host

#define DIE_HIP(expr)                                                                                  \
  do {                                                                                                 \
    hipError_t _e = (expr);                                                                            \
    if (_e != hipSuccess) return die_host::fail(DIE_E_HIP, std::string(#expr) + ": " + hipGetErrorString(_e)); \
  } while (0)

#define DIE_TRY(expr)        \
  do {                       \
    int _rc = (expr);        \
    if (_rc < 0) return _rc; \
  } while (0)
