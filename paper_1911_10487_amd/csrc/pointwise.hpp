// Table builders and pointwise kernels of the inversion path.
#pragma once
#include "common.hpp"

namespace fl {

__device__ __forceinline__ int min_image(int p, int P) { return p <= P / 2 ? p : p - P; }

// omega^2 h^3 G(r) on the torus for every height difference zeta_d:
// out[d][py][px], G(r) = -exp(i k0 r) / (4 pi r) (Section 1), r the distance
// with minimum-image horizontal offsets. zeta_d = zeta0 + d h.
template <typename T>
__global__ __launch_bounds__(256) void k_gplanes(cx<T>* __restrict__ out, int nzeta, int px, int py,
                                                 double h, double hz, double zeta0,
                                                 const double* __restrict__ zt, double k0,
                                                 double wgt) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long N = (long)px * py;
  if (idx >= N * nzeta) return;
  int d = (int)(idx / N);
  long p = idx - (long)d * N;
  int iy = (int)(p / px), ix = (int)(p - (long)iy * px);
  double dx = h * min_image(ix, px), dy = h * min_image(iy, py);
  // height difference d: zeta0 + d hz on X's lattice, else from the list zt
  double z = zt ? zt[d] : zeta0 + d * hz;
  double r = sqrt(dx * dx + dy * dy + z * z);
  double s, c;
  sincos(k0 * r, &s, &c);
  double a = -wgt / (4.0 * M_PI * r);
  out[idx] = mk((T)(a * c), (T)(a * s));
}

// Closed-form table (kernel_mode 1): out[d][m] = wgt * Ĝ(k_m, zeta_d) with
// Ĝ = -i exp(i gamma |zeta|) / (2 gamma), gamma = sqrt(k0c^2 - |k|^2),
// Im gamma >= 0, k0c = k0 (1 + i damping), k_m = 2 pi m / (P h) for the
// signed DFT index m (the continuous 2D transform of G at the torus
// wavenumbers).
__global__ __launch_bounds__(256) void k_gclosed(z64* __restrict__ out, int nzeta, int px, int py,
                                                 double h, double hz, double zeta0,
                                                 const double* __restrict__ zt, double k0,
                                                 double damping, double wgt) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long N = (long)px * py;
  if (idx >= N * nzeta) return;
  const int d = (int)(idx / N);
  const long p = idx - (long)d * N;
  const int iy = (int)(p / px), ix = (int)(p - (long)iy * px);
  const double kx = 2.0 * M_PI * min_image(ix, px) / (px * h);
  const double ky = 2.0 * M_PI * min_image(iy, py) / (py * h);
  // gamma^2 = k0^2 (1 + i damping)^2 - |k|^2
  const double gx = k0 * k0 * (1.0 - damping * damping) - (kx * kx + ky * ky);
  const double gy = 2.0 * k0 * k0 * damping;
  // principal square root (stable forms), then the branch with Im >= 0
  const double r = hypot(gx, gy);
  double sr, si;
  if (gx >= 0.0) {
    sr = sqrt(0.5 * (r + gx));
    si = sr > 0.0 ? gy / (2.0 * sr) : 0.0;
  } else {
    si = copysign(sqrt(0.5 * (r - gx)), gy);
    sr = gy / (2.0 * si);
  }
  if (si < 0.0) {
    sr = -sr;
    si = -si;
  }
  const double z = fabs(zt ? zt[d] : zeta0 + d * hz);
  double sn, cs;
  sincos(sr * z, &sn, &cs);
  const double ex = exp(-si * z);
  // -i e / (2 gamma), e = ex (cs + i sn)
  const z64 num = mk(ex * sn, -ex * cs);
  const double den = 2.0 * (sr * sr + si * si);
  const z64 val = mk((num.x * sr + num.y * si) / den, (num.y * sr - num.x * si) / den);
  out[idx] = mk(wgt * val.x, wgt * val.y);
}

// Volume kernel on the (2nz) x py x px torus with minimum-image offsets:
// h^3 G(h |d|) for d != 0 and the integral of G over the ball of volume h^3 at
// d = 0, all times wgt.
// h: horizontal cell size, hz: vertical (cells h x h x hz).
template <typename T>
__global__ __launch_bounds__(256) void k_kappa(cx<T>* __restrict__ out, int nz2, int px, int py,
                                               double h, double hz, double k0, double wgt) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long N = (long)px * py;
  if (idx >= N * nz2) return;
  int kz = (int)(idx / N);
  long p = idx - (long)kz * N;
  int iy = (int)(p / px), ix = (int)(p - (long)iy * px);
  double dz = min_image(kz, nz2), dy = min_image(iy, py), dx = min_image(ix, px);
  double re, im;
  if (kz == 0 && iy == 0 && ix == 0) {
    // (1 - (1 - i k0 a) e^{i k0 a}) / k0^2 over the ball of the cell's
    // volume: a = (3 h^2 hz / (4 pi))^(1/3)
    double a = cbrt(3.0 * h * h * hz / (4.0 * M_PI));
    double s, c;
    sincos(k0 * a, &s, &c);
    double ka = k0 * a;
    // (1 - i ka)(c + i s) = c + ka s + i (s - ka c)
    re = (1.0 - (c + ka * s)) / (k0 * k0);
    im = -(s - ka * c) / (k0 * k0);
  } else {
    double r = sqrt(h * h * (dx * dx + dy * dy) + hz * hz * dz * dz);
    double s, c;
    sincos(k0 * r, &s, &c);
    double a = -h * h * hz / (4.0 * M_PI * r);
    re = a * c;
    im = a * s;
  }
  out[idx] = mk((T)(wgt * re), (T)(wgt * im));
}

// plane-major [F][nzeta][N] -> system-major [F][N][pitch]
template <typename T>
__global__ __launch_bounds__(256) void k_to_sys(const cx<T>* __restrict__ in, z64* __restrict__ out,
                                                int nzeta, long N, int pitch) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  int f = blockIdx.y;
  if (idx >= N * nzeta) return;
  int d = (int)(idx / N);
  long m = idx - (long)d * N;
  cx<T> v = in[((long)f * nzeta + d) * N + m];
  out[((long)f * N + m) * pitch + d] = cast<double>(v);
}

// per-frequency partial sums of |W|^2: grid (nb, F), partial[f * nb + b]
template <typename TI>
__global__ __launch_bounds__(1024) void k_sumsq(const cx<TI>* __restrict__ W, long per_f,
                                                double* __restrict__ partial) {
  __shared__ double red[16];
  const int f = blockIdx.y, nb = gridDim.x;
  const cx<TI>* w = W + (long)f * per_f;
  // four independent loads in flight per thread and iteration
  constexpr int U = 4;
  const long stride = (long)nb * blockDim.x;
  double s[U] = {0.0, 0.0, 0.0, 0.0};
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < per_f; i += U * stride) {
    cx<TI> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) v[u] = w[i + u * stride];
#pragma unroll
    for (int u = 0; u < U; ++u) s[u] = fma((double)v[u].x, (double)v[u].x, fma((double)v[u].y, (double)v[u].y, s[u]));
  }
  for (; i < per_f; i += stride) {
    const cx<TI> v = w[i];
    s[0] = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, s[0]));
  }
  double t = (s[0] + s[1]) + (s[2] + s[3]);
  t = group_sum<64>(t);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) a += red[k];
    partial[f * nb + blockIdx.x] = a;
  }
}

// thr2[f] = (tau delta)^2 ||W_f||^2, or -1 for noise-free data, from nb
// partial sums per frequency. One 1024-thread block per frequency: strided
// sums with four accumulators, then the lanes and the waves in a fixed order.
__global__ __launch_bounds__(1024) void k_thresholds(const double* __restrict__ partial, int nb,
                                                     int F, double td2, double* __restrict__ thr2,
                                                     double* __restrict__ norm2) {
  __shared__ double red[16];
  const int f = blockIdx.x;
  if (f >= F) return;
  const double* pf = partial + (long)f * nb;
  double a4[4] = {0.0, 0.0, 0.0, 0.0};
  int b = threadIdx.x;
  for (; b + 3 * 1024 < nb; b += 4 * 1024) {
#pragma unroll
    for (int u = 0; u < 4; ++u) a4[u] += pf[b + u * 1024];
  }
  for (; b < nb; b += 1024) a4[0] += pf[b];
  double s = (a4[0] + a4[1]) + (a4[2] + a4[3]);
  s = group_sum<64>(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    norm2[f] = t;
    thr2[f] = td2 > 0.0 ? td2 * t : -1.0;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_zero(cx<T>* __restrict__ p, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = mk((T)0, (T)0);
}

__global__ __launch_bounds__(256) void k_narrow(const z64* __restrict__ in, z32* __restrict__ out,
                                                long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cast<float>(in[i]);
}

__global__ __launch_bounds__(256) void k_zero_real(double* __restrict__ p, long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

template <typename TI>
__global__ __launch_bounds__(256) void k_widen(const cx<TI>* __restrict__ in, z64* __restrict__ out,
                                               long n) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = cast<double>(in[i]);
}

// item 3: xi = sum_f conj(u_f) v_f / sum_f |u_f|^2 (0 where the denominator
// vanishes), with the frequency weights fw as factors of both sums when fw
// is given; per_f != 0 writes one quotient per frequency instead.
__global__ __launch_bounds__(256) void k_xi(const z64* __restrict__ u, const z64* __restrict__ v,
                                            long nvox, int F, int per_f,
                                            const double* __restrict__ fw,
                                            z64* __restrict__ xi) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox) return;
  if (per_f) {
    for (int f = 0; f < F; ++f) {
      z64 uu = u[(long)f * nvox + i], vv = v[(long)f * nvox + i];
      double dn = nrm2(uu);
      z64 nm = cmulc(uu, vv);
      xi[(long)f * nvox + i] = dn > 0.0 ? mk(nm.x / dn, nm.y / dn) : mk(0.0, 0.0);
    }
    return;
  }
  // weighted least squares when fw is given (weights of the frequencies)
  z64 num = mk(0.0, 0.0);
  double den = 0.0;
  for (int f = 0; f < F; ++f) {
    z64 uu = u[(long)f * nvox + i], vv = v[(long)f * nvox + i];
    if (fw) {
      // w_f conj(u) v = conj(w_f u) v
      const double w = fw[f];
      num = cfmac(num, w * uu, vv);
      den += w * nrm2(uu);
    } else {
      num = cfmac(num, uu, vv);
      den += nrm2(uu);
    }
  }
  xi[i] = den > 0.0 ? mk(num.x / den, num.y / den) : mk(0.0, 0.0);
}

// v = xi * u on X (real xi), written into the torus-embedded array
// out[f][l][py][px] (zeros outside the window must be set beforehand).
template <typename TI, typename T>
__global__ __launch_bounds__(256) void k_current(const double* __restrict__ xi,
                                                 const cx<TI>* __restrict__ u, int nx, int ny,
                                                 int nz, int F, int px, int py, int ox, int oy,
                                                 cx<T>* __restrict__ out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  long nvox = (long)nx * ny * nz;
  if (i >= nvox * F) return;
  int f = (int)(i / nvox);
  long v = i - (long)f * nvox;
  int l = (int)(v / ((long)nx * ny));
  long r = v - (long)l * nx * ny;
  int iy = (int)(r / nx), ix = (int)(r - (long)iy * nx);
  cx<TI> uu = u[i];
  double x = xi[v];
  out[(((long)f * nz + l) * py + iy + oy) * px + ix + ox] = mk((T)(x * uu.x), (T)(x * uu.y));
}

// W^[f][j][m] = sum_l gtab[f][j - l + nz - 1][m] V^[f][l][m] (every m)
template <typename T>
__global__ __launch_bounds__(256) void k_apply_systems(const cx<T>* __restrict__ gtab,
                                                       const cx<T>* __restrict__ Vh, int nd, int nz,
                                                       long N, int F, int thin,
                                                       cx<T>* __restrict__ Wh) {
  long fm = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (fm >= (long)F * N) return;
  int f = (int)(fm / N);
  long m = fm - (long)f * N;
  // table index of (j, l): j - l + nz - 1 on X's lattice, j nz + l otherwise
  const int nzeta = thin ? nd * nz : nd + nz - 1;
  const int sj = thin ? nz : 1, sl = thin ? 1 : -1, d0 = thin ? 0 : nz - 1;
  const cx<T>* g = gtab + (long)f * nzeta * N + m;
  const cx<T>* v = Vh + (long)f * nz * N + m;
  for (int j = 0; j < nd; ++j) {
    z64 acc = mk(0.0, 0.0);
    for (int l = 0; l < nz; ++l)
      acc = cfma(acc, cast<double>(g[(long)(j * sj + l * sl + d0) * N]), cast<double>(v[(long)l * N]));
    Wh[((long)f * nd + j) * N + m] = cast<T>(acc);
  }
}

// The same on X's lattice (nd = nz, table entry j - l + nz - 1), nz a
// multiple of JB: one thread per (f, m) takes JB rows j at a time. The JB
// table entries those rows need at one l are the ones of the previous l
// shifted by one, so they stay in registers as a circular buffer (one new
// entry per l): every v^ entry and table entry is loaded once per row block
// instead of once per row.
template <int JB>
__global__ __launch_bounds__(256) void k_apply_toeplitz(const z64* __restrict__ gtab,
                                                        const z64* __restrict__ Vh, int nz, long N,
                                                        int F, z64* __restrict__ Wh) {
  const long fm = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (fm >= (long)F * N) return;
  const int f = (int)(fm / N);
  const long m = fm - (long)f * N;
  const z64* g = gtab + (long)f * (2 * nz - 1) * N + m;
  const z64* v = Vh + (long)f * nz * N + m;
  for (int j0 = 0; j0 < nz; j0 += JB) {
    // slot (i - l) mod JB holds entry j0 + i - l + nz - 1 at step l
    z64 c[JB], acc[JB];
#pragma unroll
    for (int i = 0; i < JB; ++i) {
      c[i] = g[(long)(j0 + i + nz - 1) * N];
      acc[i] = mk(0.0, 0.0);
    }
    for (int l0 = 0; l0 < nz; l0 += JB) {
#pragma unroll
      for (int lp = 0; lp < JB; ++lp) {
        const int l = l0 + lp;
        const z64 vl = v[(long)l * N];
#pragma unroll
        for (int i = 0; i < JB; ++i) acc[i] = cfma(acc[i], c[(i - lp) & (JB - 1)], vl);
        // step l + 1 needs entry j0 - l + nz - 2 for row j0, in the slot row
        // j0 + JB - 1 has just finished with
        if (l + 1 < nz) c[(JB - 1 - lp) & (JB - 1)] = g[(long)(j0 + nz - 2 - l) * N];
      }
    }
#pragma unroll
    for (int i = 0; i < JB; ++i) Wh[((long)f * nz + j0 + i) * N + m] = acc[i];
  }
}

}  // namespace fl

namespace fl {

// ---------------------------------------------------------------- BiCGSTAB
// Stabilized biconjugate gradients (van der Vorst) for the second-kind
// equation u - omega^2 K(xi u) = u0 in X (system (2), first line), every
// frequency at once: vectors are [F][nvox] complex128, scalars per frequency.

// out[f][v] = -xi[v] y[f][v]
__global__ __launch_bounds__(256) void k_neg_xi(const double* __restrict__ xi, const z64* __restrict__ y,
                                                long nvox, int F, z64* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * F) return;
  const double x = xi[i % nvox];
  out[i] = mk(-x * y[i].x, -x * y[i].y);
}

// partial[f][blk] = sum conj(a) b over frequency f's block-strided segment
__global__ __launch_bounds__(256) void k_cdot(const z64* __restrict__ a, const z64* __restrict__ b,
                                              long n, z64* __restrict__ partial) {
  __shared__ double rx[4], ry[4];
  const int f = blockIdx.y, nb = gridDim.x;
  const z64* af = a + (long)f * n;
  const z64* bf = b + (long)f * n;
  z64 s = mk(0.0, 0.0);
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)nb * blockDim.x)
    s = cfmac(s, af[i], bf[i]);
  s.x = group_sum<64>(s.x);
  s.y = group_sum<64>(s.y);
  if ((threadIdx.x & 63) == 0) {
    rx[threadIdx.x >> 6] = s.x;
    ry[threadIdx.x >> 6] = s.y;
  }
  __syncthreads();
  if (threadIdx.x == 0)
    partial[f * nb + blockIdx.x] = mk((rx[0] + rx[1]) + (rx[2] + rx[3]), (ry[0] + ry[1]) + (ry[2] + ry[3]));
}

__global__ void k_cdot_finish(const z64* __restrict__ partial, int nb, int F, z64* __restrict__ out) {
  const int f = blockIdx.x;
  if (f >= F) return;
  z64 s = mk(0.0, 0.0);
  for (int b = threadIdx.x; b < nb; b += 64) s = s + partial[f * nb + b];
  s.x = group_sum<64>(s.x);
  s.y = group_sum<64>(s.y);
  if (threadIdx.x == 0) out[f] = s;
}

struct BicgScalars {
  z64 *rho, *alpha, *omega, *beta;
  double* bn2;
  int* active;
};

__device__ __forceinline__ z64 cdiv(z64 a, z64 b) {
  const double d = nrm2(b);
  if (!(d > 0.0)) return mk(0.0, 0.0);
  return mk((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

// alpha = rho / <rh, v>
__global__ void k_bicg_alpha(BicgScalars S, const z64* __restrict__ d, int F) {
  const int f = threadIdx.x;
  if (f < F && S.active[f]) S.alpha[f] = cdiv(S.rho[f], d[f]);
}

// omega = <t, s> / <t, t>, or 0 when ||s|| already meets the tolerance
__global__ void k_bicg_omega(BicgScalars S, const z64* __restrict__ ts, const z64* __restrict__ tt,
                             const z64* __restrict__ ss, double tol2, int F) {
  const int f = threadIdx.x;
  if (f < F && S.active[f]) S.omega[f] = ss[f].x <= tol2 * S.bn2[f] ? mk(0.0, 0.0) : cdiv(ts[f], tt[f]);
}

// beta = (rho' / rho)(alpha / omega), rho = rho'
__global__ void k_bicg_beta(BicgScalars S, const z64* __restrict__ rho_new, int F) {
  const int f = threadIdx.x;
  if (f < F && S.active[f]) {
    S.beta[f] = cdiv(rho_new[f], S.rho[f]) * cdiv(S.alpha[f], S.omega[f]);
    S.rho[f] = rho_new[f];
  }
}

// s = r - alpha v
__global__ __launch_bounds__(256) void k_bicg_s(BicgScalars S, const z64* __restrict__ r,
                                                const z64* __restrict__ v, long nvox, int F,
                                                z64* __restrict__ s) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * F) return;
  const int f = (int)(i / nvox);
  if (!S.active[f]) return;
  s[i] = cfms(r[i], S.alpha[f], v[i]);
}

// x += alpha p + omega s; r = s - omega t
__global__ __launch_bounds__(256) void k_bicg_xr(BicgScalars S, const z64* __restrict__ p,
                                                 const z64* __restrict__ s, const z64* __restrict__ t,
                                                 long nvox, int F, z64* __restrict__ x,
                                                 z64* __restrict__ r) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * F) return;
  const int f = (int)(i / nvox);
  if (!S.active[f]) return;
  const z64 a = S.alpha[f], w = S.omega[f];
  x[i] = cfma(cfma(x[i], a, p[i]), w, s[i]);
  r[i] = cfms(s[i], w, t[i]);
}

// One step of the fixed point u <- u0 + omega^2 K(xi u) (Algorithm 1) for the
// frequencies still iterating: t holds u - omega^2 K(xi u), so the new u is
// u + (u0 - t); d receives the change u0 - t (zero for frozen frequencies).
__global__ __launch_bounds__(256) void k_fp_step(const z64* __restrict__ b, const z64* __restrict__ t,
                                                 long nvox, int F, const int* __restrict__ active,
                                                 z64* __restrict__ x, z64* __restrict__ d) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * F) return;
  const int f = (int)(i / nvox);
  if (!active[f]) {
    d[i] = mk(0.0, 0.0);
    return;
  }
  const z64 di = b[i] - t[i];
  x[i] = x[i] + di;
  d[i] = di;
}

// p = r + beta (p - omega v)
__global__ __launch_bounds__(256) void k_bicg_p(BicgScalars S, const z64* __restrict__ r,
                                                const z64* __restrict__ v, long nvox, int F,
                                                z64* __restrict__ p) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox * F) return;
  const int f = (int)(i / nvox);
  if (!S.active[f]) return;
  p[i] = cfma(r[i], S.beta[f], cfms(p[i], S.omega[f], v[i]));
}

}  // namespace fl
