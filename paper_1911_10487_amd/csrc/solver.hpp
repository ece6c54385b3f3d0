// Per-system regularized solve of A_m v = w_m (Algorithm 2, item 1) for every
// active (frequency, wavenumber) system, in FP64.
//
//   k_classify / k_block_count / k_scan / k_scatter
//       ||w_m||^2 per system, the zero test ||w_m|| <= tau delta_m, and a
//       deterministic, m-ordered compaction of the systems that need a solve.
//   k_bidiag<TR, TC, NA, NB>
//       one workgroup per system: A_m (Toeplitz, generated from a 2n-1 entry
//       table row) is held in registers, distributed 2D-cyclically over a
//       TR x TC thread grid (thread (r, c) owns rows r + TR a, columns
//       c + TC b), and reduced to upper bidiagonal form by Householder
//       reflections from both sides: A = U B V^H. The left reflections are
//       applied to w on the fly (q = U^H w); the right ones are written out
//       for the back-transform.
//   k_dp
//       one lane per system: phase-scale B to a real bidiagonal, pick alpha by
//       the discrepancy principle with a safeguarded Newton iteration on
//       log(alpha), every trial an O(n) Givens QR of [B; sqrt(alpha) I]
//       (Elden's bidiagonal Tikhonov solve), and solve at the chosen alpha.
//   k_backtransform
//       one wave per system: v^ = V y, scattered into the plane-major v^.
#pragma once
#include "common.hpp"

namespace fl {

// ---------------------------------------------------------------- classify

// thread per (f, m): wn2 = sum_j |W^[f][j][m]|^2; flag = system needs a solve
template <typename T>
__global__ __launch_bounds__(256) void k_classify(const cx<T>* __restrict__ What, int nd, long N,
                                                  int F, const double* __restrict__ thr2,
                                                  double* __restrict__ wn2, int* __restrict__ flag) {
  long fm = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (fm >= (long)F * N) return;
  int f = (int)(fm / N);
  long m = fm - (long)f * N;
  const cx<T>* w = What + (long)f * nd * N + m;
  double s = 0.0;
  for (int j = 0; j < nd; ++j) {
    cx<T> v = w[(long)j * N];
    s = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, s));
  }
  wn2[fm] = s;
  // thr2[f] < 0 marks noise-free data: every nonzero system is solved
  double t = thr2[f];
  flag[fm] = (t < 0.0) ? (s > 0.0) : (s > t);
}

__device__ __forceinline__ int block_excl_scan(int v, int* wsum, int* total) {
  // 1024-thread block: ballot-based exclusive scan of 0/1 values
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  unsigned long long bal = __ballot(v);
  int pre = __popcll(bal & ((1ull << lane) - 1ull));
  if (lane == 0) wsum[wv] = __popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int i = 0; i < nw; ++i) {
      int t = wsum[i];
      wsum[i] = acc;
      acc += t;
    }
    *total = acc;
  }
  __syncthreads();
  return wsum[wv] + pre;
}

__global__ __launch_bounds__(1024) void k_block_count(const int* __restrict__ flag, long n,
                                                      int* __restrict__ cnt) {
  __shared__ int wsum[16];
  __shared__ int total;
  long i = (long)blockIdx.x * 1024 + threadIdx.x;
  int v = (i < n) ? flag[i] : 0;
  block_excl_scan(v, wsum, &total);
  if (threadIdx.x == 0) cnt[blockIdx.x] = total;
}

// single block: exclusive scan of nb block counts; writes the total to *count
__global__ __launch_bounds__(1024) void k_scan(int* __restrict__ cnt, int nb, int* __restrict__ count) {
  __shared__ int wsum[16];
  __shared__ int total;
  int carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    int i = base + threadIdx.x;
    int v = (i < nb) ? cnt[i] : 0;
    // inclusive scan of arbitrary ints: simple two-level (wave shuffles)
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      int y = __shfl_up(x, o, 64);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      int acc = 0;
      for (int w = 0; w < 16; ++w) {
        int t = wsum[w];
        wsum[w] = acc;
        acc += t;
      }
      total = acc;
    }
    __syncthreads();
    int excl = carry + wsum[wv] + x - v;
    if (i < nb) cnt[i] = excl;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) *count = carry;
}

__global__ __launch_bounds__(1024) void k_scatter(const int* __restrict__ flag, long n,
                                                  const int* __restrict__ off, int* __restrict__ list) {
  __shared__ int wsum[16];
  __shared__ int total;
  long i = (long)blockIdx.x * 1024 + threadIdx.x;
  int v = (i < n) ? flag[i] : 0;
  int p = block_excl_scan(v, wsum, &total);
  if (v) list[off[blockIdx.x] + p] = (int)i;
}

// ---------------------------------------------------------------- bidiag

struct BidiagOut {
  z64* dg;      // [n][C] diagonal of B (complex)
  z64* sp;      // [n][C] superdiagonal of B (complex; entry n-1 unused)
  z64* q;       // [n][C] U^H w
  double* fro;  // [C] ||A||_F^2
  double* wn2;  // [C] ||w||^2
  z64* refl;    // [C][n][n] right reflector k in row k, entries k+1..n-1
  double* gam;  // [C][n]
};

template <int TR, int TC, int NA, int NB>
__global__ __launch_bounds__(TR* TC) void k_bidiag(const z64* __restrict__ gsys, int tpitch,
                                                   const z64* __restrict__ What, long N,
                                                   const int* __restrict__ list,
                                                   const int* __restrict__ count, int chunk0, int C,
                                                   BidiagOut o) {
  constexpr int n = TR * NA;
  static_assert(TR * NA == TC * NB, "square system");
  constexpr int NT = TR * TC;
  constexpr int NW = (NT + 63) / 64;
  __shared__ z64 tb[2 * n];
  __shared__ z64 us[n];
  __shared__ z64 vs[n];
  __shared__ z64 xr[n];
  __shared__ z64 qv[n];
  __shared__ z64 zpart[NW][n];
  __shared__ z64 dg[n], sp[n];
  __shared__ double scal[4];
  __shared__ double red[NW];

  const int tid = threadIdx.x;
  const int r = tid % TR, c = tid / TR;
  const int lane = tid & 63, wv = tid >> 6;
  const int total = *count;

  for (int sl = blockIdx.x; sl < C; sl += gridDim.x) {
    const int gs = chunk0 + sl;
    if (gs >= total) break;
    const int fm = list[gs];
    const long m = fm % N;
    const int f = (int)(fm / N);
    const z64* trow = gsys + ((long)f * N + m) * tpitch;
    for (int t = tid; t < 2 * n - 1; t += NT) tb[t] = trow[t];
    for (int t = tid; t < n; t += NT) qv[t] = What[((long)f * n + t) * N + m];
    __syncthreads();

    z64 A[NA][NB];
    double fr = 0.0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        int i = r + TR * a, j = c + TC * b;
        A[a][b] = tb[i - j + n - 1];
        fr += nrm2(A[a][b]);
      }
    // block sums of ||A||_F^2 and ||w||^2 (fixed order)
    {
      double wsum = 0.0;
      if (tid < n) wsum = nrm2(qv[tid]);
      fr = group_sum<64>(fr);
      wsum = group_sum<64>(wsum);
      if (lane == 0) red[wv] = fr;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += red[w];
        o.fro[sl] = s;
      }
      __syncthreads();
      if (lane == 0) red[wv] = wsum;
      __syncthreads();
      if (tid == 0) {
        double s = 0.0;
        for (int w = 0; w < NW; ++w) s += red[w];
        o.wn2[sl] = s;
      }
      __syncthreads();
    }

    z64* refl = o.refl + (long)sl * n * n;
    double* gam = o.gam + (long)sl * n;

    for (int k = 0; k < n; ++k) {
      const int ka = k / TR, kr = k % TR;  // row k: row class kr, slot ka
      const int kb = k / TC, kc = k % TC;  // column k: column class kc, slot kb
      // ---------------- left reflector: column k, rows k..n-1
      if (n - k >= 2) {
        if (c == kc) {
          z64 col[NA];
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            col[a] = mk(0.0, 0.0);
#pragma unroll
            for (int b = 0; b < NB; ++b)
              if (b == kb) col[a] = A[a][b];
          }
          double s = 0.0;
          z64 piv = mk(0.0, 0.0);
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            int i = r + TR * a;
            if (i >= k) s += nrm2(col[a]);
            if (a == ka && r == kr) piv = col[a];
          }
          s = group_sum<TR>(s);
          piv.x = group_sum<TR>(piv.x);
          piv.y = group_sum<TR>(piv.y);
          double xn = sqrt(s);
          double ap = sqrt(nrm2(piv));
          z64 ph = ap > 0.0 ? mk(piv.x / ap, piv.y / ap) : mk(1.0, 0.0);
          z64 beta = mk(-ph.x * xn, -ph.y * xn);
          double g = xn > 0.0 ? 1.0 / (xn * (xn + ap)) : 0.0;
#pragma unroll
          for (int a = 0; a < NA; ++a) {
            int i = r + TR * a;
            if (i >= k) us[i] = (i == k) ? (col[a] - beta) : col[a];
          }
          if (r == kr) {
            scal[0] = g;
            dg[k] = beta;
          }
        }
      } else {
        // last column: a 1x1 block, no reflection
        if (c == kc && r == kr) {
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
              if (a == ka && b == kb) dg[k] = A[a][b];
        }
      }
      __syncthreads();
      if (n - k >= 2) {
        const double g = scal[0];
        z64 ur[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          int i = r + TR * a;
          ur[a] = (i >= k) ? us[i] : mk(0.0, 0.0);
        }
        z64 w[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          z64 s = mk(0.0, 0.0);
#pragma unroll
          for (int a = 0; a < NA; ++a) s = cfmac(s, ur[a], A[a][b]);
          s.x = group_sum<TR>(s.x);
          s.y = group_sum<TR>(s.y);
          w[b] = g * s;
        }
#pragma unroll
        for (int a = 0; a < NA; ++a)
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            int j = c + TC * b;
            if (j > k) {
              z64 t = ur[a] * w[b];
              A[a][b] = A[a][b] - t;
            }
          }
        // q <- (I - g u u^H) q, by wave 0
        if (wv == 0) {
          z64 s = mk(0.0, 0.0);
          for (int i = k + lane; i < n; i += 64) s = cfmac(s, us[i], qv[i]);
          s.x = group_sum<64>(s.x);
          s.y = group_sum<64>(s.y);
          s = g * s;
          for (int i = k + lane; i < n; i += 64) qv[i] = qv[i] - us[i] * s;
        }
      }
      // ---------------- right reflector: row k, columns k+1..n-1
      const int rk = n - k - 1;
      if (rk >= 2) {
        if (r == kr) {
#pragma unroll
          for (int b = 0; b < NB; ++b) {
            int j = c + TC * b;
            if (j > k) {
#pragma unroll
              for (int a = 0; a < NA; ++a)
                if (a == ka) xr[j] = A[a][b];
            }
          }
        }
        __syncthreads();
        if (wv == 0) {
          // reflector built from conj(row): row^T P = conj(beta') e_1^T
          double s = 0.0;
          for (int j = k + 1 + lane; j < n; j += 64) s += nrm2(xr[j]);
          s = group_sum<64>(s);
          double xn = sqrt(s);
          z64 piv = cj(xr[k + 1]);
          double ap = sqrt(nrm2(piv));
          z64 ph = ap > 0.0 ? mk(piv.x / ap, piv.y / ap) : mk(1.0, 0.0);
          z64 beta = mk(-ph.x * xn, -ph.y * xn);
          double g = xn > 0.0 ? 1.0 / (xn * (xn + ap)) : 0.0;
          for (int j = k + 1 + lane; j < n; j += 64) {
            z64 v = cj(xr[j]);
            if (j == k + 1) v = v - beta;
            vs[j] = v;
            refl[(long)k * n + j] = v;
          }
          if (lane == 0) {
            scal[1] = g;
            gam[k] = g;
            sp[k] = cj(beta);
          }
        }
        __syncthreads();
        const double g = scal[1];
        z64 vr[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          int j = c + TC * b;
          vr[b] = (j > k) ? vs[j] : mk(0.0, 0.0);
        }
        z64 zp[NA];
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          z64 s = mk(0.0, 0.0);
#pragma unroll
          for (int b = 0; b < NB; ++b) s = cfma(s, A[a][b], vr[b]);
          // sum over the column classes held by this wave
#pragma unroll
          for (int ofs = TR; ofs < 64; ofs <<= 1) {
            s.x += __shfl_xor(s.x, ofs, 64);
            s.y += __shfl_xor(s.y, ofs, 64);
          }
          zp[a] = s;
        }
        if (lane < TR) {
#pragma unroll
          for (int a = 0; a < NA; ++a) zpart[wv][r + TR * a] = zp[a];
        }
        __syncthreads();
#pragma unroll
        for (int a = 0; a < NA; ++a) {
          int i = r + TR * a;
          z64 z = mk(0.0, 0.0);
#pragma unroll
          for (int w = 0; w < NW; ++w) z = z + zpart[w][i];
          z = g * z;
          if (i > k) {
#pragma unroll
            for (int b = 0; b < NB; ++b) {
              int j = c + TC * b;
              if (j > k) A[a][b] = A[a][b] - z * cj(vr[b]);
            }
          }
        }
      } else if (rk == 1) {
        const int jb = (k + 1) / TC, jc = (k + 1) % TC;
        if (r == kr && c == jc) {
#pragma unroll
          for (int a = 0; a < NA; ++a)
#pragma unroll
            for (int b = 0; b < NB; ++b)
              if (a == ka && b == jb) sp[k] = A[a][b];
        }
        if (tid == 0) gam[k] = 0.0;
      } else {
        if (tid == 0) gam[k] = 0.0;
      }
      __syncthreads();
    }
    for (int t = tid; t < n; t += NT) {
      o.dg[(long)t * C + sl] = dg[t];
      o.sp[(long)t * C + sl] = (t < n - 1) ? sp[t] : mk(0.0, 0.0);
      o.q[(long)t * C + sl] = qv[t];
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------- dp

struct DpArgs {
  const z64* dg;
  const z64* sp;
  const z64* q;
  const double* fro;
  const double* wn2;
  const int* list;
  const int* count;
  int chunk0, C, n;
  long N;
  const double* thr2;  // per frequency: (tau delta_m)^2, < 0 for noise-free data
  double eta;
  // scratch, [n][C]
  double* d;
  double* e;
  z64* qr;
  z64* dr;
  double* rho;
  double* off;
  z64* rr;
  z64* y;        // output [n][C]: y = D_R y' (before the right reflectors)
  double* alpha; // [F*N]
  signed char* branch;  // [F*N]
};

// Elden: min ||B y - q||^2 + alpha ||y||^2 for real upper bidiagonal B (d, e)
// by Givens QR of [B; sqrt(alpha) I]; returns phi = ||B y - q||^2 and, when
// want_d, dphi/dalpha = 2 alpha ||R^-T y||^2. Writes y when ys != nullptr.
__device__ double elden(const DpArgs& a, int sl, double alpha, bool want_d, double* dphi,
                        z64* ys) {
  const int n = a.n;
  const long C = a.C;
  const double mu = sqrt(alpha);
  double mt = mu;
  z64 g = mk(0.0, 0.0);
  for (int i = 0; i < n; ++i) {
    const double di = a.d[i * C + sl];
    const z64 qi = a.qr[i * C + sl];
    double p = sqrt(di * di + mt * mt);
    double cs = p > 0.0 ? di / p : 1.0;
    double sn = p > 0.0 ? mt / p : 0.0;
    a.rho[i * C + sl] = p;
    a.rr[i * C + sl] = cs * qi + sn * g;
    z64 gp = (-sn) * qi + cs * g;
    if (i < n - 1) {
      const double ei = a.e[i * C + sl];
      a.off[i * C + sl] = cs * ei;
      double fz = -sn * ei;
      double p2 = sqrt(mu * mu + fz * fz);
      double s2 = p2 > 0.0 ? fz / p2 : 0.0;
      mt = p2;
      g = s2 * gp;
    }
  }
  // back substitution and residual
  z64 yn = mk(0.0, 0.0);
  double phi = 0.0;
  double ynorm_unused = 0.0;
  (void)ynorm_unused;
  for (int i = n - 1; i >= 0; --i) {
    const double p = a.rho[i * C + sl];
    z64 t = a.rr[i * C + sl];
    if (i < n - 1) t = t - a.off[i * C + sl] * yn;
    z64 yi = p > 0.0 ? mk(t.x / p, t.y / p) : mk(0.0, 0.0);
    // residual row i: d_i y_i + e_i y_{i+1} - q_i
    z64 res = a.d[i * C + sl] * yi - a.qr[i * C + sl];
    if (i < n - 1) res = res + a.e[i * C + sl] * yn;
    phi += nrm2(res);
    if (ys) ys[i * C + sl] = yi;
    a.y[i * C + sl] = yi;  // keep y for the derivative pass
    yn = yi;
  }
  if (want_d) {
    z64 zp = mk(0.0, 0.0);
    double zz = 0.0;
    for (int i = 0; i < n; ++i) {
      const double p = a.rho[i * C + sl];
      z64 t = a.y[i * C + sl];
      if (i > 0) t = t - a.off[(i - 1) * C + sl] * zp;
      z64 zi = p > 0.0 ? mk(t.x / p, t.y / p) : mk(0.0, 0.0);
      zz += nrm2(zi);
      zp = zi;
    }
    *dphi = 2.0 * alpha * zz;
  }
  return phi;
}

__global__ __launch_bounds__(64) void k_dp(DpArgs a) {
  const int sl = blockIdx.x * blockDim.x + threadIdx.x;
  if (sl >= a.C) return;
  const int gs = a.chunk0 + sl;
  if (gs >= *a.count) return;
  const int fm = a.list[gs];
  const int f = (int)(fm / a.N);
  const int n = a.n;
  const long C = a.C;
  // phase scaling to a real nonnegative bidiagonal: B = D_L B' D_R^H
  z64 drc = mk(1.0, 0.0);
  for (int i = 0; i < n; ++i) {
    z64 t = a.dg[i * C + sl] * drc;
    double at = sqrt(nrm2(t));
    z64 dl = at > 0.0 ? mk(t.x / at, t.y / at) : mk(1.0, 0.0);
    a.d[i * C + sl] = at;
    a.dr[i * C + sl] = drc;
    a.qr[i * C + sl] = cmulc(dl, a.q[i * C + sl]);
    if (i < n - 1) {
      z64 s = cmulc(dl, a.sp[i * C + sl]);
      double as = sqrt(nrm2(s));
      a.e[i * C + sl] = as;
      drc = as > 0.0 ? mk(s.x / as, -s.y / as) : mk(1.0, 0.0);
    }
  }
  const double T = a.thr2[f];
  const double amin = a.eta * a.fro[sl];
  double alpha = amin;
  signed char br = 1;
  if (T >= 0.0) {
    double dum;
    double p0 = elden(a, sl, amin, false, &dum, nullptr);
    if (p0 < T) {
      br = 2;
      double lo = log(amin);
      double hi = log(a.fro[sl]) + 1.0;
      for (int it = 0; it < 400; ++it) {
        double ph = elden(a, sl, exp(hi), false, &dum, nullptr);
        if (ph >= T || hi > 690.0) break;
        hi += 4.0;
      }
      double x = 0.5 * (lo + hi);
      for (int it = 0; it < 200; ++it) {
        double al = exp(x);
        double dphi = 0.0;
        double ph = elden(a, sl, al, true, &dphi, nullptr);
        double F = ph - T;
        if (F >= 0.0)
          hi = x;
        else
          lo = x;
        double Fp = al * dphi;
        double xn = (Fp > 0.0) ? x - F / Fp : 0.5 * (lo + hi);
        if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
        double step = fabs(xn - x);
        x = xn;
        if (step <= 4e-16 * fmax(1.0, fabs(x)) || hi - lo <= 4e-16 * fmax(1.0, fabs(x))) break;
      }
      alpha = exp(x);
    }
  }
  double dum;
  elden(a, sl, alpha, false, &dum, nullptr);
  for (int i = 0; i < n; ++i) a.y[i * C + sl] = a.dr[i * C + sl] * a.y[i * C + sl];
  a.alpha[fm] = alpha;
  a.branch[fm] = br;
}

// one wave per system: v^ = V y, V = P_0 P_1 ... (right reflectors)
template <typename T>
__global__ __launch_bounds__(256) void k_backtransform(const z64* __restrict__ y,
                                                       const z64* __restrict__ refl,
                                                       const double* __restrict__ gam,
                                                       const int* __restrict__ list,
                                                       const int* __restrict__ count, int chunk0,
                                                       int C, int n, long N, cx<T>* __restrict__ Vh) {
  const int lane = threadIdx.x & 63;
  const int sl = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (sl >= C) return;
  const int gs = chunk0 + sl;
  if (gs >= *count) return;
  const int fm = list[gs];
  const int f = (int)(fm / N);
  const long m = fm - (long)f * N;
  z64 y0 = lane < n ? y[(long)lane * C + sl] : mk(0.0, 0.0);
  z64 y1 = lane + 64 < n ? y[(long)(lane + 64) * C + sl] : mk(0.0, 0.0);
  const z64* R = refl + (long)sl * n * n;
  const double* G = gam + (long)sl * n;
  for (int k = n - 3; k >= 0; --k) {
    const double g = G[k];
    z64 v0 = (lane > k && lane < n) ? R[(long)k * n + lane] : mk(0.0, 0.0);
    z64 v1 = (lane + 64 > k && lane + 64 < n) ? R[(long)k * n + lane + 64] : mk(0.0, 0.0);
    z64 s = mk(0.0, 0.0);
    s = cfmac(s, v0, y0);
    s = cfmac(s, v1, y1);
    s.x = group_sum<64>(s.x);
    s.y = group_sum<64>(s.y);
    s = g * s;
    y0 = y0 - v0 * s;
    y1 = y1 - v1 * s;
  }
  cx<T>* out = Vh + (long)f * n * N + m;
  if (lane < n) out[(long)lane * N] = cast<T>(y0);
  if (lane + 64 < n) out[(long)(lane + 64) * N] = cast<T>(y1);
}

}  // namespace fl
