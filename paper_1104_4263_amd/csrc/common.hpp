// Shared device/host helpers of the TE DIE library (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace die {

template <class T> struct c2t;
template <> struct c2t<double> { using type = double2; };
template <> struct c2t<float> { using type = float2; };
// complex with IEEE binary16 parts: the storage type of the compressed Krylov basis
struct alignas(4) half2c {
  _Float16 x, y;
};
template <> struct c2t<_Float16> { using type = half2c; };
template <class T> using c2 = typename c2t<T>::type;

template <class T> __host__ __device__ __forceinline__ c2<T> mk(T re, T im) {
  c2<T> r; r.x = re; r.y = im; return r;
}
template <class T> __device__ __forceinline__ c2<T> cadd(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <class T> __device__ __forceinline__ c2<T> csub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <class T> __device__ __forceinline__ c2<T> cmul(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// conj(a) * b
template <class T> __device__ __forceinline__ c2<T> cmulc(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// a * (-i) and a * (+i)
template <class T> __device__ __forceinline__ c2<T> mul_mi(c2<T> a) { return mk<T>(a.y, -a.x); }
template <class T> __device__ __forceinline__ c2<T> mul_pi(c2<T> a) { return mk<T>(-a.y, a.x); }

// Block barrier that the compiler may not move LDS accesses across: without the memory clobber,
// LDS reads issued before __syncthreads() have been sunk below it (into the next loop
// iteration's exchange), racing with other waves' writes after the barrier.
__device__ __forceinline__ void lds_sync() {
  asm volatile("" ::: "memory");
  __syncthreads();
  asm volatile("" ::: "memory");
}

// Widening / narrowing loads and stores between storage precision S and compute precision T.
template <class T, class S> __device__ __forceinline__ c2<T> ld(const c2<S>* p) {
  c2<S> v = *p; return mk<T>((T)v.x, (T)v.y);
}
template <class S, class T> __device__ __forceinline__ void st(c2<S>* p, c2<T> v) {
  *p = mk<S>((S)v.x, (S)v.y);
}

// Twiddle table exp(-2 pi i j / 4096), j < 4096, in both precisions (device globals,
// filled once per device from values rounded on the host from long double).
constexpr int kLogTw = 12;
constexpr int kTw = 1 << kLogTw;

}  // namespace die
