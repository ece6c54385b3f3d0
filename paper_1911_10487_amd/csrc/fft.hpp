// Batched mixed-radix (4, 2, 3, 5) Stockham FFTs staged through LDS.
//
// A workgroup loads a tile of CB transforms of length L from global memory
// (any element / batch / plane strides, loads ordered so that the unit-stride
// index is the fastest across lanes), runs the self-sorting Stockham passes
// between two LDS buffers, and stores the result with its own strides. Input
// may be zero-extended (only `lin` elements are read, placed at `in_off`) and
// output may be pruned (only elements [out_off, out_off + lout) are written),
// which is how the zero-padded convolution and the crop to X's window avoid
// moving zeros through HBM.
//
// Convention: forward = sum_k x_k exp(-2 pi i k m / L), inverse uses +i and is
// unnormalized; callers fold 1/L factors into `scale` or into tables.
#pragma once
#include "common.hpp"

namespace fl {

struct FftArgs {
  const void* in;
  void* out;
  const void* tw;   // tw[i] = exp(-2 pi i i / L), i < L
  long in_sk, in_sb, in_sp;
  long out_sk, out_sb, out_sp;
  int L;
  int lin, in_off;
  int lout, out_off;
  int B;            // transforms per plane
  int planes;
  int in_kfast, out_kfast;
  double scale;
  const z64* add;   // optional FP64 addend laid out like the output
  double* rowsq;    // optional, power-of-two kernels: sum of |input|^2 per
                    // transform, [plane][b]
};

template <typename T>
__device__ __forceinline__ cx<T> twiddle(const cx<T>* tw, int idx, int dir) {
  cx<T> w = tw[idx];
  if (dir > 0) w.y = -w.y;
  return w;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft4(cx<T>* v) {
  cx<T> t0 = v[0] + v[2], t1 = v[0] - v[2];
  cx<T> t2 = v[1] + v[3], t3 = rot90<T, DIR>(v[1] - v[3]);
  v[0] = t0 + t2;
  v[2] = t0 - t2;
  v[1] = t1 + t3;
  v[3] = t1 - t3;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft2(cx<T>* v) {
  cx<T> a = v[0];
  v[0] = a + v[1];
  v[1] = a - v[1];
}

template <typename T, int DIR>
__device__ __forceinline__ void dft3(cx<T>* v) {
  const T c = (T)0.86602540378443864676;  // sqrt(3)/2
  cx<T> s = v[1] + v[2];
  cx<T> d = v[1] - v[2];
  cx<T> m = v[0] - (T)0.5 * s;
  cx<T> r = rot90<T, DIR>(c * d);  // DIR*i*sqrt(3)/2*d
  v[0] = v[0] + s;
  v[1] = m + r;
  v[2] = m - r;
}

template <typename T, int DIR>
__device__ __forceinline__ void dft5(cx<T>* v) {
  // b_s = sum_q a_q exp(DIR 2 pi i q s / 5)
  const T c1 = (T)0.30901699437494742410;   // cos(2pi/5)
  const T c2 = (T)-0.80901699437494742410;  // cos(4pi/5)
  const T s1 = (T)0.95105651629515357212;   // sin(2pi/5)
  const T s2 = (T)0.58778525229247312917;   // sin(4pi/5)
  cx<T> a1 = v[1] + v[4], b1 = v[1] - v[4];
  cx<T> a2 = v[2] + v[3], b2 = v[2] - v[3];
  cx<T> m1 = v[0] + c1 * a1 + c2 * a2;
  cx<T> m2 = v[0] + c2 * a1 + c1 * a2;
  // DIR*i*(s1 b1 + s2 b2) and DIR*i*(s2 b1 - s1 b2)
  cx<T> r1 = rot90<T, DIR>(s1 * b1 + s2 * b2);
  cx<T> r2 = rot90<T, DIR>(s2 * b1 - s1 * b2);
  v[0] = v[0] + a1 + a2;
  v[1] = m1 + r1;
  v[4] = m1 - r1;
  v[2] = m2 + r2;
  v[3] = m2 - r2;
}

template <typename T, int DIR, int R>
__device__ __forceinline__ void stockham_pass(const cx<T>* __restrict__ src, cx<T>* __restrict__ dst,
                                              const cx<T>* __restrict__ tw, int CB, int L, int LP,
                                              int Ns, int tid, int nt) {
  const int LR = L / R;
  const int tstep = L / (Ns * R);
  for (int t = tid; t < CB * LR; t += nt) {
    int bb = t / LR;
    int j = t - bb * LR;
    int k = j % Ns;
    const cx<T>* s = src + bb * LP;
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = s[j + r * LR];
    if (k > 0) {
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = v[r] * twiddle(tw, (r * k * tstep) % L, DIR);
    }
    if (R == 4) dft4<T, DIR>(v);
    if (R == 2) dft2<T, DIR>(v);
    if (R == 3) dft3<T, DIR>(v);
    if (R == 5) dft5<T, DIR>(v);
    int idx = (j / Ns) * Ns * R + k;
    cx<T>* d = dst + bb * LP;
#pragma unroll
    for (int r = 0; r < R; ++r) d[idx + r * Ns] = v[r];
  }
}

// Runs the whole transform; returns the buffer that holds the result.
template <typename T, int DIR>
__device__ cx<T>* lds_fft(cx<T>* a, cx<T>* b, const cx<T>* tw, int CB, int L, int LP, int tid,
                          int nt) {
  int Ns = 1;
  while (Ns < L) {
    int rem = L / Ns;
    if (rem % 4 == 0) {
      stockham_pass<T, DIR, 4>(a, b, tw, CB, L, LP, Ns, tid, nt);
      Ns *= 4;
    } else if (rem % 2 == 0) {
      stockham_pass<T, DIR, 2>(a, b, tw, CB, L, LP, Ns, tid, nt);
      Ns *= 2;
    } else if (rem % 3 == 0) {
      stockham_pass<T, DIR, 3>(a, b, tw, CB, L, LP, Ns, tid, nt);
      Ns *= 3;
    } else {
      stockham_pass<T, DIR, 5>(a, b, tw, CB, L, LP, Ns, tid, nt);
      Ns *= 5;
    }
    __syncthreads();
    cx<T>* t = a;
    a = b;
    b = t;
  }
  return a;
}

// Load a tile: elements [0, lin) of every transform in the WG's batch chunk
// land at positions in_off + k; everything else in the transform is zero.
// Each thread issues all of its global loads (up to 16) before the first LDS
// store, so that many loads are in flight per CU.
template <typename TI, typename T>
__device__ __forceinline__ void tile_load(const FftArgs& g, cx<T>* a, int CB, int LP, int b0,
                                          int plane, int tid, int nt) {
  const cx<TI>* in = (const cx<TI>*)g.in + (long)plane * g.in_sp;
  const int L = g.L;
  if (g.lin < L) {
    for (int t = tid; t < CB * L; t += nt) {
      int bb = t / L, k = t - bb * L;
      if (k < g.in_off || k >= g.in_off + g.lin) a[bb * LP + k] = mk((T)0, (T)0);
    }
  }
  const int n = CB * g.lin;
  constexpr int MAXE = 16;
  for (int base = 0; base < n; base += MAXE * nt) {
    cx<TI> buf[MAXE];
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int t = base + tid + e * nt;
      buf[e] = mk((TI)0, (TI)0);
      if (t < n) {
        int bb, k;
        if (g.in_kfast) {
          bb = t / g.lin;
          k = t - bb * g.lin;
        } else {
          k = t / CB;
          bb = t - k * CB;
        }
        const int b = b0 + bb;
        if (b < g.B) buf[e] = in[(long)b * g.in_sb + (long)k * g.in_sk];
      }
    }
#pragma unroll
    for (int e = 0; e < MAXE; ++e) {
      const int t = base + tid + e * nt;
      if (t < n) {
        int bb, k;
        if (g.in_kfast) {
          bb = t / g.lin;
          k = t - bb * g.lin;
        } else {
          k = t / CB;
          bb = t - k * CB;
        }
        a[bb * LP + g.in_off + k] = cast<T>(buf[e]);
      }
    }
  }
}

// Twiddles of length L staged into LDS once per workgroup.
template <typename T>
__device__ __forceinline__ void stage_twiddles(const cx<T>* __restrict__ tw, cx<T>* s, int L, int tid,
                                               int nt) {
  for (int i = tid; i < L; i += nt) s[i] = tw[i];
}

template <typename TO, typename T>
__device__ __forceinline__ void tile_store(const FftArgs& g, const cx<T>* a, int CB, int LP, int b0,
                                           int plane, int tid, int nt) {
  cx<TO>* out = (cx<TO>*)g.out + (long)plane * g.out_sp;
  const int n = CB * g.lout;
  const T sc = (T)g.scale;
  for (int t = tid; t < n; t += nt) {
    int bb, k;
    if (g.out_kfast) {
      bb = t / g.lout;
      k = t - bb * g.lout;
    } else {
      k = t / CB;
      bb = t - k * CB;
    }
    int b = b0 + bb;
    if (b < g.B) {
      cx<T> v = a[bb * LP + g.out_off + k];
      long o = (long)plane * g.out_sp + (long)b * g.out_sb + (long)k * g.out_sk;
      cx<TO> r = cast<TO>(sc * v);
      if (g.add) {
        z64 ad = g.add[o];
        r = mk((TO)(r.x + ad.x), (TO)(r.y + ad.y));
      }
      out[o - (long)plane * g.out_sp] = r;
    }
  }
}

// grid: (ceil(B / CB), planes); dynamic LDS: 2 * CB * (L + 1) * sizeof(cx<T>)
template <typename TI, typename T, typename TO, int DIR>
__global__ __launch_bounds__(256) void k_fft(FftArgs g, int CB) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int LP = g.L + 1;
  cx<T>* tws = (cx<T>*)smem;
  cx<T>* a = tws + g.L;
  cx<T>* b = a + CB * LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b0 = blockIdx.x * CB;
  const int plane = blockIdx.y;
  stage_twiddles<T>((const cx<T>*)g.tw, tws, g.L, tid, nt);
  tile_load<TI, T>(g, a, CB, LP, b0, plane, tid, nt);
  __syncthreads();
  cx<T>* r = lds_fft<T, DIR>(a, b, tws, CB, g.L, LP, tid, nt);
  tile_store<TO, T>(g, r, CB, LP, b0, plane, tid, nt);
}

// Pointwise-multiplied convolution along one axis: forward FFT of the
// zero-extended input, multiply by mul[k * mul_sk + b] (per plane offset
// mul_sp), inverse FFT, store the pruned output. Used for the z direction of
// the 3D volume convolution, where b runs over horizontal wavenumbers.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_conv(FftArgs g, const void* mul, long mul_sk,
                                                  long mul_sp, int CB, int conj_mul) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int LP = g.L + 1;
  cx<T>* tws = (cx<T>*)smem;
  cx<T>* a = tws + g.L;
  cx<T>* b = a + CB * LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b0 = blockIdx.x * CB;
  const int plane = blockIdx.y;
  stage_twiddles<T>((const cx<T>*)g.tw, tws, g.L, tid, nt);
  tile_load<T, T>(g, a, CB, LP, b0, plane, tid, nt);
  __syncthreads();
  cx<T>* r = lds_fft<T, -1>(a, b, tws, CB, g.L, LP, tid, nt);
  const cx<T>* K = (const cx<T>*)mul + (long)plane * mul_sp;
  for (int t = tid; t < CB * g.L; t += nt) {
    int k = t / CB, bb = t - k * CB;
    int bg = b0 + bb;
    if (bg < g.B) {
      cx<T> kk = K[(long)k * mul_sk + bg];
      if (conj_mul) kk.y = -kk.y;
      r[bb * LP + k] = r[bb * LP + k] * kk;
    }
  }
  __syncthreads();
  cx<T>* o = (r == a) ? b : a;
  r = lds_fft<T, 1>(r, o, tws, CB, g.L, LP, tid, nt);
  tile_store<T, T>(g, r, CB, LP, b0, plane, tid, nt);
}

// Row kernel of stage (c): inverse FFT of a row of v^ (already inverse-
// transformed along y), crop to X's window and scale into v (stored), then
// re-embed v at the start of a zero row and forward transform it for the
// volume convolution. One transform per row; rows are contiguous.
//   in   rows of length L (stride L), out_v rows of length nwin (stride nwin),
//   out_f rows of length L. win_off: first column of X's window.
template <typename T>
__global__ __launch_bounds__(256) void k_rows_crop_pad(const cx<T>* __restrict__ in,
                                                       cx<double>* __restrict__ out_v,
                                                       cx<T>* __restrict__ out_f,
                                                       const cx<T>* __restrict__ tw, int L, int nwin,
                                                       int win_off, int rows, double scale, int CB) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int LP = L + 1;
  cx<T>* tws = (cx<T>*)smem;
  cx<T>* a = tws + L;
  cx<T>* b = a + CB * LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const long r0 = (long)blockIdx.x * CB;
  stage_twiddles<T>(tw, tws, L, tid, nt);
  {
    FftArgs g{};
    g.in = in;
    g.L = L;
    g.lin = L;
    g.in_sk = 1;
    g.in_sb = L;
    g.B = rows;
    g.in_kfast = 1;
    tile_load<T, T>(g, a, CB, LP, (int)r0, 0, tid, nt);
  }
  __syncthreads();
  cx<T>* r = lds_fft<T, 1>(a, b, tws, CB, L, LP, tid, nt);
  cx<T>* o = (r == a) ? b : a;
  const T sc = (T)scale;
  for (int t = tid; t < CB * L; t += nt) {
    int bb = t / L, k = t - bb * L;
    long row = r0 + bb;
    cx<T> v = mk((T)0, (T)0);
    if (k < nwin) {
      v = sc * r[bb * LP + win_off + k];
      if (row < rows) out_v[row * nwin + k] = cast<double>(v);
    }
    o[bb * LP + k] = v;
  }
  __syncthreads();
  cx<T>* s = lds_fft<T, -1>(o, r, tws, CB, L, LP, tid, nt);
  for (int t = tid; t < CB * L; t += nt) {
    int bb = t / L, k = t - bb * L;
    long row = r0 + bb;
    if (row < rows) out_f[row * L + k] = s[bb * LP + k];
  }
}

// ---------------------------------------------------------------------------
// Power-of-two lengths 32..1024: register-blocked Stockham transforms.
//
// A transform of length L is shared by TT = L / E threads, each holding E
// elements in registers: thread t holds elements k = t + TT s (s < E) both
// before the first pass and after the last one (the Stockham passes sort
// themselves). A pass of radix R runs E / R butterflies per thread entirely
// in registers; consecutive passes exchange data through one padded LDS row
// per transform. Every size, stride and radix is a compile-time constant, so
// the index arithmetic is shifts and masks.

template <int L>
struct P2;
template <> struct P2<32>   { static constexpr int E = 8,  NP = 2, R0 = 8,  R1 = 4,  R2 = 1; };
template <> struct P2<64>   { static constexpr int E = 8,  NP = 2, R0 = 8,  R1 = 8,  R2 = 1; };
template <> struct P2<128>  { static constexpr int E = 16, NP = 2, R0 = 16, R1 = 8,  R2 = 1; };
template <> struct P2<256>  { static constexpr int E = 16, NP = 2, R0 = 16, R1 = 16, R2 = 1; };
template <> struct P2<512>  { static constexpr int E = 8,  NP = 3, R0 = 8,  R1 = 8,  R2 = 8; };
template <> struct P2<1024> { static constexpr int E = 16, NP = 3, R0 = 16, R1 = 16, R2 = 4; };

__host__ __device__ constexpr bool p2_supported(int L) {
  return L == 32 || L == 64 || L == 128 || L == 256 || L == 512 || L == 1024;
}

// one pad slot after every 16 elements keeps strided scatters off one bank
__device__ __forceinline__ int p2pad(int x) { return x + (x >> 4); }
// Row pitch of a transform in LDS: the padded length rounded up to 1 mod 32
// elements, so that consecutive transforms (the lanes of a column map) start
// on different banks.
template <int L>
__host__ __device__ constexpr int p2_row() {
  return L + L / 16 + (((1 - (L + L / 16)) % 32) + 32) % 32;
}

// Element of the LDS exchange rows. FP64 transforms exchange the real and
// then the imaginary parts through a row of doubles: half the LDS per
// transform, so twice as many transforms stay resident on a CU (the FP64
// kernels are HBM-bound and otherwise LDS-limited to 1.5 waves per SIMD).
// FP32 transforms exchange whole complex values.
template <typename T>
struct P2Lds {
  using type = cx<T>;
  static constexpr bool split = false;
};
template <>
struct P2Lds<double> {
  using type = double;
  static constexpr bool split = true;
};

// Transforms per workgroup: up to 512 threads and 64 KiB of LDS (twiddles
// plus one padded row per transform).
template <int L, typename T>
__host__ __device__ constexpr int p2_cb() {
  constexpr int TT = L / P2<L>::E;
  int cb = 512 / TT;
  while (cb > 1 && (size_t)L * sizeof(cx<T>) +
                           (size_t)cb * p2_row<L>() * sizeof(typename P2Lds<T>::type) > 65536)
    cb /= 2;
  return cb;
}

// exp(DIR 2 pi i j / 16) for compile-time j, as (cos, DIR sin)
template <typename T, int DIR>
__device__ __forceinline__ cx<T> w16(int j) {
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173;
  const T c2 = (T)0.70710678118654752440;
  T c = 1, s = 0;
  switch (j & 15) {
    case 0: c = 1; s = 0; break;
    case 1: c = c1; s = s1; break;
    case 2: c = c2; s = c2; break;
    case 3: c = s1; s = c1; break;
    case 4: c = 0; s = 1; break;
    case 5: c = -s1; s = c1; break;
    case 6: c = -c2; s = c2; break;
    case 7: c = -c1; s = s1; break;
    case 8: c = -1; s = 0; break;
    case 9: c = -c1; s = -s1; break;
    case 10: c = -c2; s = -c2; break;
    case 11: c = -s1; s = -c1; break;
    case 12: c = 0; s = -1; break;
    case 13: c = s1; s = -c1; break;
    case 14: c = c2; s = -c2; break;
    default: c = c1; s = -s1; break;
  }
  return mk(c, (T)DIR * s);
}

// a * exp(DIR 2 pi i j / 16); j is a compile-time constant after unrolling
template <typename T, int DIR>
__device__ __forceinline__ cx<T> mul_w16(cx<T> a, int j) {
  j &= 15;
  if (j == 0) return a;
  if (j == 4) return rot90<T, DIR>(a);
  if (j == 8) return mk(-a.x, -a.y);
  if (j == 12) return rot90<T, -DIR>(a);
  return a * w16<T, DIR>(j);
}

// length-8 DFT in place: n = n1 + 2 n2, k = 4 k1 + k2
template <typename T, int DIR>
__device__ __forceinline__ void dft8(cx<T>* v) {
  cx<T> a[4] = {v[0], v[2], v[4], v[6]};
  cx<T> b[4] = {v[1], v[3], v[5], v[7]};
  dft4<T, DIR>(a);
  dft4<T, DIR>(b);
#pragma unroll
  for (int k2 = 1; k2 < 4; ++k2) b[k2] = mul_w16<T, DIR>(b[k2], 2 * k2);
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    v[k2] = a[k2] + b[k2];
    v[4 + k2] = a[k2] - b[k2];
  }
}

// length-16 DFT in place: n = n1 + 4 n2, k = 4 k1 + k2
template <typename T, int DIR>
__device__ __forceinline__ void dft16(cx<T>* v) {
  cx<T> y[4][4];
#pragma unroll
  for (int n1 = 0; n1 < 4; ++n1) {
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) y[n1][n2] = v[n1 + 4 * n2];
    dft4<T, DIR>(y[n1]);
#pragma unroll
    for (int k2 = 1; k2 < 4; ++k2) y[n1][k2] = mul_w16<T, DIR>(y[n1][k2], n1 * k2);
  }
#pragma unroll
  for (int k2 = 0; k2 < 4; ++k2) {
    cx<T> z[4] = {y[0][k2], y[1][k2], y[2][k2], y[3][k2]};
    dft4<T, DIR>(z);
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) v[4 * k1 + k2] = z[k1];
  }
}

template <typename T, int DIR, int R>
__device__ __forceinline__ void dft_r(cx<T>* v) {
  if constexpr (R == 2) dft2<T, DIR>(v);
  if constexpr (R == 4) dft4<T, DIR>(v);
  if constexpr (R == 8) dft8<T, DIR>(v);
  if constexpr (R == 16) dft16<T, DIR>(v);
}

// Butterflies of one pass (stride NS, radix R) on the thread's registers:
// butterfly q uses e[q + r E/R], r < R.
template <typename T, int DIR, int L, int R, int NS>
__device__ __forceinline__ void p2_butterflies(cx<T> (&e)[P2<L>::E], const cx<T>* tws, int t) {
  constexpr int E = P2<L>::E, TT = L / E, NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    cx<T> v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = e[q + r * NB];
    if constexpr (NS > 1) {
      const int k = (t + TT * q) & (NS - 1);
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = v[r] * twiddle(tws, r * k * (L / (NS * R)), DIR);
    }
    dft_r<T, DIR, R>(v);
#pragma unroll
    for (int r = 0; r < R; ++r) e[q + r * NB] = v[r];
  }
}

// Stockham placement of a pass's outputs in the LDS row.
template <typename T, int L, int R, int NS>
__device__ __forceinline__ void p2_scatter(const cx<T> (&e)[P2<L>::E], cx<T>* row, int t) {
  constexpr int E = P2<L>::E, TT = L / E, NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int i = t + TT * q;
    const int base = (i / NS) * NS * R + (i & (NS - 1));
#pragma unroll
    for (int r = 0; r < R; ++r) row[p2pad(base + r * NS)] = e[q + r * NB];
  }
}

// Every pass reads element t + TT s into e[s].
template <typename T, int L>
__device__ __forceinline__ void p2_gather(cx<T> (&e)[P2<L>::E], const cx<T>* row, int t) {
  constexpr int E = P2<L>::E, TT = L / E;
#pragma unroll
  for (int s = 0; s < E; ++s) e[s] = row[p2pad(t + TT * s)];
}

// The same placement and read for one part (IM: imaginary) through a row of
// reals. Between the two parts the registers hold the new real parts and
// the old imaginary ones, which the second scatter still reads in the old
// order.
template <typename T, int L, int R, int NS, bool IM>
__device__ __forceinline__ void p2_scatter_part(const cx<T> (&e)[P2<L>::E], T* row, int t) {
  constexpr int E = P2<L>::E, TT = L / E, NB = E / R;
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const int i = t + TT * q;
    const int base = (i / NS) * NS * R + (i & (NS - 1));
#pragma unroll
    for (int r = 0; r < R; ++r) row[p2pad(base + r * NS)] = IM ? e[q + r * NB].y : e[q + r * NB].x;
  }
}
template <typename T, int L, bool IM>
__device__ __forceinline__ void p2_gather_part(cx<T> (&e)[P2<L>::E], const T* row, int t) {
  constexpr int E = P2<L>::E, TT = L / E;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const T v = row[p2pad(t + TT * s)];
    if (IM)
      e[s].y = v;
    else
      e[s].x = v;
  }
}

// One exchange between passes: Stockham placement, barrier, reads.
template <typename T, int L, int R, int NS>
__device__ __forceinline__ void p2_exchange(cx<T> (&e)[P2<L>::E], typename P2Lds<T>::type* row,
                                            int t) {
  if constexpr (P2Lds<T>::split) {
    p2_scatter_part<T, L, R, NS, false>(e, row, t);
    __syncthreads();
    p2_gather_part<T, L, false>(e, row, t);
    __syncthreads();
    p2_scatter_part<T, L, R, NS, true>(e, row, t);
    __syncthreads();
    p2_gather_part<T, L, true>(e, row, t);
  } else {
    p2_scatter<T, L, R, NS>(e, row, t);
    __syncthreads();
    p2_gather<T, L>(e, row, t);
  }
}

// The whole transform, registers to registers. SYNC_IN: the LDS row may still
// be read by other threads (a previous transform's last gather).
template <typename T, int DIR, int L, bool SYNC_IN>
__device__ __forceinline__ void p2_fft(cx<T> (&e)[P2<L>::E], typename P2Lds<T>::type* row,
                                       const cx<T>* tws, int t) {
  using P = P2<L>;
  p2_butterflies<T, DIR, L, P::R0, 1>(e, tws, t);
  if constexpr (SYNC_IN) __syncthreads();
  p2_exchange<T, L, P::R0, 1>(e, row, t);
  p2_butterflies<T, DIR, L, P::R1, P::R0>(e, tws, t);
  if constexpr (P::NP == 3) {
    __syncthreads();
    p2_exchange<T, L, P::R1, P::R0>(e, row, t);
    p2_butterflies<T, DIR, L, P::R2, P::R0 * P::R1>(e, tws, t);
  }
}

// Thread -> (transform, position) map. Row transforms (unit element stride)
// put consecutive threads on consecutive elements; column transforms (unit
// batch stride) put them on consecutive transforms.
template <int L, int CB>
__device__ __forceinline__ void p2_map(int kfast, int& t, int& bl) {
  constexpr int TT = L / P2<L>::E;
  const int tid = threadIdx.x;
  if (kfast) {
    t = tid % TT;
    bl = tid / TT;
  } else {
    bl = tid % CB;
    t = tid / CB;
  }
}

template <typename TI, typename T, int L>
__device__ __forceinline__ void p2_load(const FftArgs& g, cx<T> (&e)[P2<L>::E], int b, int plane, int t) {
  constexpr int E = P2<L>::E, TT = L / E;
  const bool ok = b < g.B;
  const cx<TI>* in = (const cx<TI>*)g.in + (long)plane * g.in_sp + (long)b * g.in_sb;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int kk = t + TT * s - g.in_off;
    e[s] = (ok && kk >= 0 && kk < g.lin) ? cast<T>(in[(long)kk * g.in_sk]) : mk((T)0, (T)0);
  }
}

template <typename TO, typename T, int L>
__device__ __forceinline__ void p2_store(const FftArgs& g, const cx<T> (&e)[P2<L>::E], int b, int plane,
                                         int t) {
  constexpr int E = P2<L>::E, TT = L / E;
  if (b >= g.B) return;
  const T sc = (T)g.scale;
  const long ob = (long)plane * g.out_sp + (long)b * g.out_sb;
#pragma unroll
  for (int s = 0; s < E; ++s) {
    const int kk = t + TT * s - g.out_off;
    if (kk >= 0 && kk < g.lout) {
      const long o = ob + (long)kk * g.out_sk;
      cx<TO> r = cast<TO>(sc * e[s]);
      if (g.add) {
        const z64 ad = g.add[o];
        r = mk((TO)(r.x + ad.x), (TO)(r.y + ad.y));
      }
      ((cx<TO>*)g.out)[o] = r;
    }
  }
}

// Block (bx, by) of a 2D grid, renumbered so that each XCD takes a
// contiguous range of the blocks in linear order (workgroups go to the eight
// XCDs in turn by linear block id): neighbouring groups of columns, which at
// 8 bytes per element share 128-byte lines, then meet in one L2.
__device__ __forceinline__ void xcd_block(int& bx, int& by) {
  const long G = gridDim.x, T = G * gridDim.y;
  const long lin = blockIdx.x + blockIdx.y * G;
  const long q = T / 8, r = T % 8, x = lin % 8, j = lin / 8;
  const long lp = x * q + (x < r ? x : r) + j;
  bx = (int)(lp % G);
  by = (int)(lp / G);
}

template <typename T, int L>
__device__ __forceinline__ void p2_stage_twiddles(const cx<T>* __restrict__ tw, cx<T>* tws, int nt) {
  for (int i = threadIdx.x; i < L; i += nt) tws[i] = tw[i];
}

// grid (ceil(B / CB), planes), block CB * L / E threads; same arguments and
// semantics as k_fft (in_kfast selects the thread map, out_kfast must equal it)
template <typename TI, typename T, typename TO, int DIR, int L>
__global__ __launch_bounds__((p2_cb<L, T>() * (L / P2<L>::E))) void k_fft_p2(FftArgs g) {
  constexpr int CB = p2_cb<L, T>(), NT = CB * (L / P2<L>::E);
  __shared__ cx<T> tws[L];
  __shared__ typename P2Lds<T>::type lds[CB * p2_row<L>()];
  int t, bl, bx, by;
  p2_map<L, CB>(g.in_kfast, t, bl);
  xcd_block(bx, by);
  const int b = bx * CB + bl, plane = by;
  p2_stage_twiddles<T, L>((const cx<T>*)g.tw, tws, NT);
  cx<T> e[P2<L>::E];
  p2_load<TI, T, L>(g, e, b, plane, t);
  if (g.rowsq) {
    // the row's sum of squares while it is in registers (the threads of a
    // transform are consecutive lanes on the unit-stride map)
    double sq = 0.0;
#pragma unroll
    for (int s = 0; s < P2<L>::E; ++s)
      sq = fma((double)e[s].x, (double)e[s].x, fma((double)e[s].y, (double)e[s].y, sq));
    sq = group_sum<L / P2<L>::E>(sq);
    if (t == 0 && b < g.B) g.rowsq[(long)plane * g.B + b] = sq;
  }
  p2_fft<T, DIR, L, false>(e, lds + bl * p2_row<L>(), tws, t);
  p2_store<TO, T, L>(g, e, b, plane, t);
}

// z-direction convolution (column map): forward transform of the
// zero-extended input, product with mul[k * mul_sk + b] (plane offset
// mul_sp, conjugated when conj_mul), inverse transform, pruned store. EVEN:
// mul is the transform of a kernel even in z (entries 0..L/2 are read);
// otherwise every entry is read.
template <typename T, int L, bool EVEN = true>
__global__ __launch_bounds__((p2_cb<L, T>() * (L / P2<L>::E))) void k_fft_conv_p2(FftArgs g, const void* mul,
                                                                              long mul_sk, long mul_sp,
                                                                              int conj_mul) {
  constexpr int CB = p2_cb<L, T>(), E = P2<L>::E, TT = L / E, NT = CB * TT;
  __shared__ cx<T> tws[L];
  __shared__ typename P2Lds<T>::type lds[CB * p2_row<L>()];
  int t, bl, bx, by;
  p2_map<L, CB>(0, t, bl);
  xcd_block(bx, by);
  const int b = bx * CB + bl, plane = by;
  p2_stage_twiddles<T, L>((const cx<T>*)g.tw, tws, NT);
  cx<T> e[E];
  p2_load<T, T, L>(g, e, b, plane, t);
  typename P2Lds<T>::type* row = lds + bl * p2_row<L>();
  p2_fft<T, -1, L, false>(e, row, tws, t);
  if (b < g.B) {
    // The volume kernel of the z-convolution is even in z (the sampled
    // kernel at -d equals the one at d), so its transform is even in k:
    // entry L - k is read as entry k, which another thread of the same
    // transform reads at the same time, halving the table's HBM reads.
    const cx<T>* K = (const cx<T>*)mul + (long)plane * mul_sp + b;
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int k = t + TT * s;
      const int kt = EVEN ? (k <= L / 2 ? k : L - k) : k;
      cx<T> kk = K[(long)kt * mul_sk];
      if (conj_mul) kk.y = -kk.y;
      e[s] = e[s] * kk;
    }
  }
  p2_fft<T, 1, L, true>(e, row, tws, t);
  p2_store<T, T, L>(g, e, b, plane, t);
}

// Row kernel of stage (c) for power-of-two rows (row map): inverse
// transform, crop to X's window and scale into out_v (FP64), then the window
// re-embedded at the start of a zero row and transformed forward into out_f.
template <typename T, int L>
__global__ __launch_bounds__((p2_cb<L, T>() * (L / P2<L>::E))) void k_rows_crop_pad_p2(
    const cx<T>* __restrict__ in, cx<double>* __restrict__ out_v, cx<T>* __restrict__ out_f,
    const cx<T>* __restrict__ tw, int nwin, int win_off, int rows, double scale) {
  constexpr int CB = p2_cb<L, T>(), E = P2<L>::E, TT = L / E, NT = CB * TT;
  __shared__ cx<T> tws[L];
  __shared__ typename P2Lds<T>::type lds[CB * p2_row<L>()];
  int t, bl;
  p2_map<L, CB>(1, t, bl);
  const long row_i = (long)blockIdx.x * CB + bl;
  const bool ok = row_i < rows;
  p2_stage_twiddles<T, L>(tw, tws, NT);
  cx<T> e[E];
#pragma unroll
  for (int s = 0; s < E; ++s) e[s] = ok ? in[row_i * L + t + TT * s] : mk((T)0, (T)0);
  typename P2Lds<T>::type* row = lds + bl * p2_row<L>();
  p2_fft<T, 1, L, false>(e, row, tws, t);
  const T sc = (T)scale;
  __syncthreads();
  if constexpr (P2Lds<T>::split) {
    // the scaled window, then its real and imaginary parts in turn through
    // the row of reals (the window at the start, zeros after it)
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int kk = t + TT * s - win_off;
      if (kk >= 0 && kk < nwin) {
        e[s] = sc * e[s];
        if (ok) out_v[row_i * nwin + kk] = cast<double>(e[s]);
      }
    }
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int k = t + TT * s;
      const int kk = k - win_off;
      if (kk >= 0 && kk < nwin) row[p2pad(kk)] = e[s].x;
      if (k >= nwin) row[p2pad(k)] = (T)0;
    }
    __syncthreads();
    p2_gather_part<T, L, false>(e, row, t);
    __syncthreads();
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int k = t + TT * s;
      const int kk = k - win_off;
      if (kk >= 0 && kk < nwin) row[p2pad(kk)] = e[s].y;
      if (k >= nwin) row[p2pad(k)] = (T)0;
    }
    __syncthreads();
    p2_gather_part<T, L, true>(e, row, t);
  } else {
#pragma unroll
    for (int s = 0; s < E; ++s) {
      const int k = t + TT * s;
      const int kk = k - win_off;
      if (kk >= 0 && kk < nwin) {
        const cx<T> v = sc * e[s];
        if (ok) out_v[row_i * nwin + kk] = cast<double>(v);
        row[p2pad(kk)] = v;
      }
      if (k >= nwin) row[p2pad(k)] = mk((T)0, (T)0);
    }
    __syncthreads();
    p2_gather<T, L>(e, row, t);
  }
  p2_fft<T, -1, L, true>(e, row, tws, t);
  if (ok) {
#pragma unroll
    for (int s = 0; s < E; ++s) out_f[row_i * L + t + TT * s] = e[s];
  }
}

}  // namespace fl
