// Common device/host helpers for the variable-density solver library.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <cstddef>

namespace vd {

// Complex number in registers / memory: (re, im) of the real type R.
template <typename R> struct C2 { R x, y; };

template <typename R> struct VecOf;
template <> struct VecOf<double> { using type = double2; };
template <> struct VecOf<float>  { using type = float2; };

template <typename R>
__device__ __forceinline__ C2<R> cmk(R a, R b) { return C2<R>{a, b}; }
template <typename R>
__device__ __forceinline__ C2<R> operator+(C2<R> a, C2<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> operator-(C2<R> a, C2<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <typename R>
__device__ __forceinline__ C2<R> cmulc(C2<R> a, C2<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <typename R>
__device__ __forceinline__ C2<R> cscale(C2<R> a, R s) { return {a.x * s, a.y * s}; }
template <typename R>
__device__ __forceinline__ C2<R> cconj(C2<R> a) { return {a.x, -a.y}; }
// i * k * a
template <typename R>
__device__ __forceinline__ C2<R> cik(C2<R> a, R k) { return {-a.y * k, a.x * k}; }

template <typename R>
__device__ __forceinline__ C2<R> ldg(const C2<R>* p) {
  using V = typename VecOf<R>::type;
  V v = *reinterpret_cast<const V*>(p);
  return C2<R>{v.x, v.y};
}
template <typename R>
__device__ __forceinline__ void stg(C2<R>* p, C2<R> a) {
  using V = typename VecOf<R>::type;
  V v; v.x = a.x; v.y = a.y;
  *reinterpret_cast<V*>(p) = v;
}

// Spectral index helpers.  Axis of n points: storage index i in [0, n)
// holds integer wavenumber kappa = i for i <= n/2, i - n otherwise.  The
// first-derivative symbol zeroes the Nyquist index (i == n/2); the second
// derivative keeps it.
__device__ __forceinline__ int kappa_of(int i, int n) { return i <= n / 2 ? i : i - n; }
template <typename R>
__device__ __forceinline__ R kprime_of(int i, int n, R scale) {
  return (i == n / 2) ? R(0) : R(kappa_of(i, n)) * scale;
}
template <typename R>
__device__ __forceinline__ R ksq_of(int i, int n, R scale) {
  R k = R(kappa_of(i, n)) * scale;
  return k * k;
}

}  // namespace vd
