// Shared device helpers: complex arithmetic on (re, im) pairs and small
// wave-level utilities for gfx950 (wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fl {

// aligned to its size, so that a complex double moves in one 16-byte access
template <typename T>
struct alignas(2 * sizeof(T)) cx {
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
// acc - a * b
template <typename T>
__device__ __forceinline__ cx<T> cfms(cx<T> acc, cx<T> a, cx<T> b) {
  acc.x = fma(-a.x, b.x, fma(a.y, b.y, acc.x));
  acc.y = fma(-a.x, b.y, fma(-a.y, b.x, acc.y));
  return acc;
}
// acc - a * conj(b)
template <typename T>
__device__ __forceinline__ cx<T> cfmsc(cx<T> acc, cx<T> a, cx<T> b) {
  acc.x = fma(-a.x, b.x, fma(-a.y, b.y, acc.x));
  acc.y = fma(-a.y, b.x, fma(a.x, b.y, acc.y));
  return acc;
}
// multiply by -i (dir < 0) or +i (dir > 0)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> rot90(cx<T> a) {
  if (DIR < 0) return mk(a.y, -a.x);
  return mk(-a.y, a.x);
}

// Householder reflectors of one n x n factorization, packed row after row:
// reflector k holds entries k + off .. n - 1 (off = 0: left reflectors,
// which start on the diagonal; off = 1: right reflectors) and starts at
// tri_start(k, n, off); one factorization's set takes tri_size(n, off).
__host__ __device__ __forceinline__ long tri_start(int k, int n, int off) {
  return (long)k * (n - off) - (long)k * (k - 1) / 2;
}
__host__ __device__ __forceinline__ long tri_size(int n, int off) { return tri_start(n, n, off); }

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

// ---- reciprocal and reciprocal square root: hardware estimate + two Newton
// steps (quadratic convergence), for positive normal arguments
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(fma(-x, r, 1.0), r, r);
  r = fma(fma(-x, r, 1.0), r, r);
  return r;
}
__device__ __forceinline__ double rsq_nr(double x) {
  double r = __builtin_amdgcn_rsq(x);
  r = r * fma(-0.5 * x * r, r, 1.5);
  r = r * fma(-0.5 * x * r, r, 1.5);
  return r;
}

// ---- cross-lane moves without the LDS crossbar (gfx950 DPP / permlane)

// DPP read of another lane's value. Only permutations inside a row of 16 are
// used (mirror, half-mirror, quad_perm), where every lane has a valid source,
// so the move needs no "old" value.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  int lo = __double2loint(v), hi = __double2hiint(v);
  lo = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  hi = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// v plus the value of lane (i ^ 16). The swap leaves each lane holding its
// own value and its partner's, and both lanes of a pair add them in the same
// order (lower lane's value first), so they get bitwise the same sum.
__device__ __forceinline__ double add_xor16(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto rl = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(rh[0], rl[0]) + __hiloint2double(rh[1], rl[1]);
}

// v plus the value of lane (i ^ 32), same pairing as add_xor16
__device__ __forceinline__ double add_xor32(double v) {
  const int lo = __double2loint(v), hi = __double2hiint(v);
  const auto rl = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(rh[0], rl[0]) + __hiloint2double(rh[1], rl[1]);
}

// Sum over the 16 lanes of a DPP row; every lane receives the bitwise same
// total (each step adds a symmetric pair).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_d<0x140>(v);  // row_mirror: i <-> 15 - i
  v += dpp_d<0x141>(v);  // row_half_mirror: i <-> 7 - i within 8
  v += dpp_d<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_d<0xB1>(v);   // quad_perm [1,0,3,2]
  return v;
}

// value of lane l (uniform) of the wave, whatever the execution mask
__device__ __forceinline__ double lane_read(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ cx<double> lane_read(cx<double> v, int l) {
  return mk(lane_read(v.x, l), lane_read(v.y, l));
}

// ---- reduce-scatter steps: of the pair (lo, hi) of values held by every
// lane, the lanes on the lower side of a lane pairing end with lo summed over
// the pair and the lanes on the upper side with hi summed over the pair, so
// each sum is formed once and the values to carry halve.

// pairing i <-> i ^ 16 (lower side: bit 4 clear). The swap leaves the lower
// lane (lo, partner's lo) and the upper lane (partner's hi, hi).
__device__ __forceinline__ double rs_xor16(double lo, double hi) {
  const auto rl = __builtin_amdgcn_permlane16_swap(__double2loint(lo), __double2loint(hi), false, false);
  const auto rh = __builtin_amdgcn_permlane16_swap(__double2hiint(lo), __double2hiint(hi), false, false);
  return __hiloint2double(rh[0], rl[0]) + __hiloint2double(rh[1], rl[1]);
}
// pairing i <-> i ^ 32 (lower side: bit 5 clear)
__device__ __forceinline__ double rs_xor32(double lo, double hi) {
  const auto rl = __builtin_amdgcn_permlane32_swap(__double2loint(lo), __double2loint(hi), false, false);
  const auto rh = __builtin_amdgcn_permlane32_swap(__double2hiint(lo), __double2hiint(hi), false, false);
  return __hiloint2double(rh[0], rl[0]) + __hiloint2double(rh[1], rl[1]);
}
// A DPP pairing inside each row of 16 lanes whose lower side is the lanes of
// the DPP banks (groups of four lanes) in LOWER: row_mirror (i <-> 15 - i,
// lower = banks 0 and 1) or row_half_mirror (i <-> 7 - i within eight,
// lower = banks 0 and 2). A DPP move writes only the lanes of its enabled
// banks, so the lower lanes take their partner's lo and keep their own, the
// upper lanes their partner's hi.
template <int CTRL, int LOWER>
__device__ __forceinline__ double rs_dpp(double lo, double hi) {
  const int ll = __double2loint(lo), lh = __double2hiint(lo);
  const int hl = __double2loint(hi), hh = __double2hiint(hi);
  const int tl = __builtin_amdgcn_update_dpp(hl, ll, CTRL, 0xF, LOWER, false);
  const int th = __builtin_amdgcn_update_dpp(hh, lh, CTRL, 0xF, LOWER, false);
  const int ul = __builtin_amdgcn_update_dpp(ll, hl, CTRL, 0xF, 0xF ^ LOWER, false);
  const int uh = __builtin_amdgcn_update_dpp(lh, hh, CTRL, 0xF, 0xF ^ LOWER, false);
  return __hiloint2double(th, tl) + __hiloint2double(uh, ul);
}

// Sum over aligned groups of W lanes (W = 16, 32, 64).
template <int W>
__device__ __forceinline__ double lanes_sum(double v) {
  v = row16_sum(v);
  if (W >= 32) v = add_xor16(v);
  if (W >= 64) v = add_xor32(v);
  return v;
}

// Sum over the lanes of a wave that share (lane mod W): strides W .. 32.
template <int W>
__device__ __forceinline__ double strided_sum(double v) {
  if (W <= 16) v = add_xor16(v);
  if (W <= 32) v = add_xor32(v);
  return v;
}

}  // namespace fl
