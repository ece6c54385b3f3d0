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
  for (int t = tid; t < n; t += nt) {
    int bb, k;
    if (g.in_kfast) {
      bb = t / g.lin;
      k = t - bb * g.lin;
    } else {
      k = t / CB;
      bb = t - k * CB;
    }
    int b = b0 + bb;
    cx<T> v = mk((T)0, (T)0);
    if (b < g.B) v = cast<T>(in[(long)b * g.in_sb + (long)k * g.in_sk]);
    a[bb * LP + g.in_off + k] = v;
  }
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
  cx<T>* a = (cx<T>*)smem;
  cx<T>* b = a + CB * LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b0 = blockIdx.x * CB;
  const int plane = blockIdx.y;
  tile_load<TI, T>(g, a, CB, LP, b0, plane, tid, nt);
  __syncthreads();
  cx<T>* r = lds_fft<T, DIR>(a, b, (const cx<T>*)g.tw, CB, g.L, LP, tid, nt);
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
  cx<T>* a = (cx<T>*)smem;
  cx<T>* b = a + CB * LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int b0 = blockIdx.x * CB;
  const int plane = blockIdx.y;
  tile_load<T, T>(g, a, CB, LP, b0, plane, tid, nt);
  __syncthreads();
  cx<T>* r = lds_fft<T, -1>(a, b, (const cx<T>*)g.tw, CB, g.L, LP, tid, nt);
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
  r = lds_fft<T, 1>(r, o, (const cx<T>*)g.tw, CB, g.L, LP, tid, nt);
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
  cx<T>* a = (cx<T>*)smem;
  cx<T>* b = a + CB * LP;
  const int tid = threadIdx.x, nt = blockDim.x;
  const long r0 = (long)blockIdx.x * CB;
  for (int t = tid; t < CB * L; t += nt) {
    int bb = t / L, k = t - bb * L;
    long row = r0 + bb;
    a[bb * LP + k] = row < rows ? in[row * L + k] : mk((T)0, (T)0);
  }
  __syncthreads();
  cx<T>* r = lds_fft<T, 1>(a, b, tw, CB, L, LP, tid, nt);
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
  cx<T>* s = lds_fft<T, -1>(o, r, tw, CB, L, LP, tid, nt);
  for (int t = tid; t < CB * L; t += nt) {
    int bb = t / L, k = t - bb * L;
    long row = r0 + bb;
    if (row < rows) out_f[row * L + k] = s[bb * LP + k];
  }
}

}  // namespace fl
