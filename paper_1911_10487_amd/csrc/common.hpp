// Shared device helpers: complex arithmetic on (re, im) pairs and small
// wave-level utilities for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

template <typename T>
struct cx {
  T x, y;
};

using z64 = cx<double>;
using z32 = cx<float>;

template <typename T>
__host__ __device__ __forceinline__ cx<T> mk(T a, T b) {
  cx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cx<T> operator*(T s, cx<T> a) { return mk(s * a.x, s * a.y); }
template <typename T>
__device__ __forceinline__ cx<T> cj(cx<T> a) { return mk(a.x, -a.y); }
template <typename T>
__device__ __forceinline__ T nrm2(cx<T> a) { return a.x * a.x + a.y * a.y; }
// conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cmulc(cx<T> a, cx<T> b) {
  return mk(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
// acc + a * b
template <typename T>
__device__ __forceinline__ cx<T> cfma(cx<T> acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(a.y, b.x, acc.y));
  return acc;
}
// acc + conj(a) * b
template <typename T>
__device__ __forceinline__ cx<T> cfmac(cx<T> acc, cx<T> a, cx<T> b) {
  acc.x = fma(a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(a.x, b.y, fma(-a.y, b.x, acc.y));
  return acc;
}
// multiply by -i (dir < 0) or +i (dir > 0)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  if (DIR < 0) return mk(a.y, -a.x);
  return mk(-a.y, a.x);
}

template <typename A, typename B>
__device__ __forceinline__ cx<A> cast(cx<B> v) {
  return mk((A)v.x, (A)v.y);
}

// Wave64 butterfly sum over lanes that share (lane / width): width a power of
// two <= 64. Every lane of a group returns the group's sum; the summation
// order is fixed, so results are reproducible.
template <int WIDTH>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = WIDTH / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
template <int WIDTH>
__device__ __forceinline__ float group_sum(float v) {
#pragma unroll
  for (int o = WIDTH / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

}  // namespace fl
