// Reverse (VJP) and tangent (JVP) derivatives of the inversion map W -> xi.
//
// Per solved system (M = A^H A + alpha I, v^ = M^-1 A^H w):
//   VJP  w^bar = A M^-1 v^bar, and for a discrepancy-chosen alpha the
//        implicit term w^bar -= (s / phi_a) q, Tbar += s / phi_a with
//        s = -Re(v^bar^H M^-1 v^), phi_a = 2 alpha v^H M^-1 v^,
//        q = 2 (-alpha A M^-1 v^ - r), r = A v^ - w;
//   JVP  alpha' = (T' - Re(q^H w')) / phi_a, v^' = M^-1 (A^H w' - alpha' v^).
// M^-1 is applied through the forward factorization: A = U D_L B' D_R^H V^H
// (Householder reflectors V, phases D_R, real bidiagonal B'), so
// M^-1 x = V D_R (B'^T B' + alpha I)^-1 D_R^H V^H x, and the tridiagonal
// solve uses R^T R = B'^T B' + alpha I from the Givens QR of [B'; sqrt(alpha) I].
// A and A^H are applied directly from the system's Toeplitz table row. With
// shared factorizations (one per symmetry orbit of the wavenumbers) the
// system's factorization is its orbit's: the reflectors of the orbit slot,
// and B', D_R from the slot's complex bidiagonal by the same phase scaling
// as the forward solve.
#pragma once
#include "common.hpp"
#include "solver.hpp"

namespace fl {

struct AdjArgs {
  const z64* gsys;      // [F][N][tpitch] Toeplitz table rows
  int tpitch;
  const int* list;
  const int* count;
  int C, n;
  int chunk0;           // first compacted system of the resident chunk
  long N;
  const double* alpha;  // [F*N]
  const signed char* branch;
  const double* bd_d;   // [C][n] real bidiagonal and phases from the forward
  const double* bd_e;
  const z64* bd_dr;
  const z64* refl;      // [C][tri_size(n, 1)] packed right reflectors
  const double* gam;    // [C][n]
  const void* What;     // [F][n][N] forward W^ (complex128)
  const void* Vh;       // [F][n][N] forward v^
  const void* X;        // VJP: v^bar [F][n][N]; JVP: W^' [F][n][N]
  int single;           // 1: Vh (and the JVP's Y) hold complex64
  int x_single;         // 1: X holds complex64
  const double* Tdot;   // JVP: per frequency T'
  void* Y;              // VJP: w^bar [F][n][N] complex128; JVP: v^' (type of Vh)
  double* cm;           // VJP: [F*N] implicit-alpha coefficients s / phi_a
  // shared factorizations (NULL: one per system): system (f, m) uses slot
  // oslot[f N + orep[m]] of refl, gam and of the complex bidiagonal dg, sp
  const int* oslot;
  const int* orep;
  const z64* dg;
  const z64* sp;
  // orbit chunks (NULL: every active orbit has a slot): the systems of
  // compacted orbits [slot0, slot0 + OC), factorizations in slots
  // oslot - slot0
  const int* osys0;
  const int* ocount;
  int slot0, OC;
};

template <typename T>
__device__ __forceinline__ z64 ld(const void* p, long i) {
  return cast<double>(((const cx<T>*)p)[i]);
}

__device__ __forceinline__ z64 ldx(const void* p, long i, int single) {
  return single ? ld<float>(p, i) : ld<double>(p, i);
}

// complex dot conj(a) . b over the wave's two-slot distribution
__device__ __forceinline__ z64 wdot(z64 a0, z64 a1, z64 b0, z64 b1) {
  z64 s = cmulc(a0, b0);
  s = cfmac(s, a1, b1);
  s.x = lanes_sum<64>(s.x);
  s.y = lanes_sum<64>(s.y);
  return s;
}

// A shared slot's complex bidiagonal (cy, cs) is needed only by the phase
// scaling, before vec, irho and off are first written: it shares their
// storage (less LDS per workgroup, more resident waves).
template <int NMAX>
struct AdjShared {
  z64 t[2 * NMAX];
  union {
    z64 vec[NMAX];
    z64 cy[NMAX];
  };
  double d[NMAX], e[NMAX];
  union {
    struct {
      double irho[NMAX], off[NMAX];
    };
    z64 cs[NMAX];
  };
  z64 dr[NMAX];
};

// y = M^-1 x for the wave-distributed x (entries lane, lane + 64)
template <int NMAX>
__device__ void minv(const AdjArgs& a, AdjShared<NMAX>& S, int sl, z64& x0, z64& x1) {
  constexpr int E = NMAX / 64;  // elements per lane: lane, lane + 64
  constexpr int RG = E == 1 ? 8 : 2;  // reflector rows loaded ahead
  const int n = a.n, lane = threadIdx.x;
  const z64* R = a.refl + (long)sl * tri_size(n, 1);
  const double* G = a.gam + (long)sl * n;
  z64 x[E];
  // z = V^H x = P_{n-3} ... P_0 x (reflector k has entries k + 1 .. n - 1)
  x[0] = x0;
  if constexpr (E > 1) x[1] = x1;
  group_reflect<64, E, RG>(x, R, G, n, lane, 0, n - 2, 1, 1);
  x0 = x[0];
  if constexpr (E > 1) x1 = x[1];
  // D_R^H, then (R^T R)^-1 sequentially on lane 0
  if (lane < n) S.vec[lane] = cmulc(S.dr[lane], x0);
  if (lane + 64 < n) S.vec[lane + 64] = cmulc(S.dr[lane + 64], x1);
  __syncthreads();
  if (lane == 0) {
    z64 tp = mk(0.0, 0.0);
    for (int i = 0; i < n; ++i) {  // R^T t = z
      z64 t = S.vec[i];
      if (i > 0) t = t - S.off[i - 1] * tp;
      t = S.irho[i] * t;
      S.vec[i] = t;
      tp = t;
    }
    z64 yn = mk(0.0, 0.0);
    for (int i = n - 1; i >= 0; --i) {  // R y = t
      z64 y = S.vec[i];
      if (i < n - 1) y = y - S.off[i] * yn;
      y = S.irho[i] * y;
      S.vec[i] = y;
      yn = y;
    }
  }
  __syncthreads();
  x[0] = lane < n ? S.dr[lane] * S.vec[lane] : mk(0.0, 0.0);
  if constexpr (E > 1) x[1] = lane + 64 < n ? S.dr[lane + 64] * S.vec[lane + 64] : mk(0.0, 0.0);
  __syncthreads();
  // V y = P_0 (P_1 (... P_{n-3} y))
  group_reflect<64, E, RG>(x, R, G, n, lane, n - 3, -1, -1, 1);
  x0 = x[0];
  x1 = E > 1 ? x[E - 1] : mk(0.0, 0.0);
}

// (A x)_j = sum_l t[j - l + n - 1] x_l, or (A^H x)_l = sum_j conj(t[j - l + n - 1]) x_j,
// each sum in P partial sums (l mod P) so that consecutive products do not
// wait for each other; the last n mod P terms go to the first
template <int NMAX, bool HERM, int P>
__device__ void toeplitz(AdjShared<NMAX>& S, int n, z64& x0, z64& x1) {
  const int lane = threadIdx.x;
  if (lane < n) S.vec[lane] = x0;
  if (lane + 64 < n) S.vec[lane + 64] = x1;
  __syncthreads();
  z64 o[2] = {mk(0.0, 0.0), mk(0.0, 0.0)};
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int j = lane + 64 * h;
    if (j < n) {
      z64 acc[P];
#pragma unroll
      for (int q = 0; q < P; ++q) acc[q] = mk(0.0, 0.0);
      const int nP = n & ~(P - 1);  // P a power of two
      for (int l0 = 0; l0 < nP; l0 += P) {
#pragma unroll
        for (int q = 0; q < P; ++q) {
          const int l = l0 + q;
          if (HERM)
            acc[q] = cfmac(acc[q], S.t[l - j + n - 1], S.vec[l]);
          else
            acc[q] = cfma(acc[q], S.t[j - l + n - 1], S.vec[l]);
        }
      }
      for (int l = nP; l < n; ++l) {
        if (HERM)
          acc[0] = cfmac(acc[0], S.t[l - j + n - 1], S.vec[l]);
        else
          acc[0] = cfma(acc[0], S.t[j - l + n - 1], S.vec[l]);
      }
      if constexpr (P == 4)
        o[h] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
      else if constexpr (P == 2)
        o[h] = acc[0] + acc[1];
      else
        o[h] = acc[0];
    }
  }
  __syncthreads();
  x0 = o[0];
  x1 = o[1];
}

// MODE 0: VJP, MODE 1: JVP. One single-wave workgroup per solved system.
template <int NMAX, int MODE>
__global__ __launch_bounds__(64) void k_sys_adjoint(AdjArgs a) {
  __shared__ AdjShared<NMAX> S;
  // partial sums per Toeplitz product (more would cost a wave per SIMD)
  constexpr int TP = 2;
  const int lane = threadIdx.x;
  const int n = a.n;
  const int total = *a.count;
  int c0;
  const int nsys = launch_range(a.osys0, a.ocount, a.slot0, a.OC, a.chunk0, a.C, total, &c0);
  for (int sl = blockIdx.x; sl < nsys; sl += gridDim.x) {
    const int fm = a.list[c0 + sl];
    const int f = (int)(fm / a.N);
    const long m = fm - (long)f * a.N;
    const double al = a.alpha[fm];
    const bool root = a.branch[fm] == 2;
    const z64* trow = a.gsys + ((long)f * a.N + m) * a.tpitch;
    for (int i = lane; i < 2 * n - 1; i += 64) S.t[i] = trow[i];
    // factorization slot: the system's own, or its orbit's
    const int fs = a.oslot ? a.oslot[(long)f * a.N + a.orep[m]] - a.slot0 : sl;
    if (a.oslot) {
      for (int i = lane; i < n; i += 64) {
        S.cy[i] = a.dg[(long)fs * n + i];
        S.cs[i] = a.sp[(long)fs * n + i];
      }
      __syncthreads();
      dp_phase_scale<NMAX>(n, lane, S.d, S.e, nullptr, S.cs, S.cy, S.dr);
    } else {
      for (int i = lane; i < n; i += 64) {
        S.d[i] = a.bd_d[(long)sl * n + i];
        S.e[i] = a.bd_e[(long)sl * n + i];
        S.dr[i] = a.bd_dr[(long)sl * n + i];
      }
    }
    __syncthreads();
    if (lane == 0) {
      // R of the Givens QR of [B'; sqrt(alpha) I] (rhs not needed)
      const double mu = sqrt(al);
      double mt = mu;
      for (int i = 0; i < n; ++i) {
        const double di = S.d[i];
        const double p2 = di * di + mt * mt;
        const double ip = p2 > 0.0 ? rsq_nr(p2) : 0.0;
        S.irho[i] = ip;
        if (i < n - 1) {
          const double cs = p2 > 0.0 ? di * ip : 1.0;
          const double sn = mt * ip;
          S.off[i] = cs * S.e[i];
          const double fz = -sn * S.e[i];
          const double q2 = mu * mu + fz * fz;
          mt = q2 > 0.0 ? q2 * rsq_nr(q2) : 0.0;
        }
      }
    }
    __syncthreads();
    const long base = (long)f * n * a.N + m;
    auto at = [&](const void* p, int i, int sgl) {
      return i < n ? ldx(p, base + (long)i * a.N, sgl) : mk(0.0, 0.0);
    };
    const z64 vh0 = at(a.Vh, lane, a.single), vh1 = at(a.Vh, lane + 64, a.single);
    const z64 w0 = at(a.What, lane, 0), w1 = at(a.What, lane + 64, 0);
    const z64 x0i = at(a.X, lane, a.x_single), x1i = at(a.X, lane + 64, a.x_single);
    // pieces of the implicit alpha derivative
    z64 q0 = mk(0.0, 0.0), q1 = mk(0.0, 0.0);
    double phia = 1.0, sx2 = 0.0;
    if (root) {
      z64 m0 = vh0, m1 = vh1;
      minv<NMAX>(a, S, fs, m0, m1);                   // x2 = M^-1 v^
      phia = 2.0 * al * wdot(vh0, vh1, m0, m1).x;
      if (MODE == 0) sx2 = -wdot(x0i, x1i, m0, m1).x; // s = -Re(v^bar^H x2)
      z64 a0 = m0, a1 = m1;
      toeplitz<NMAX, false, TP>(S, n, a0, a1);            // A x2
      z64 r0 = vh0, r1 = vh1;
      toeplitz<NMAX, false, TP>(S, n, r0, r1);            // A v^
      r0 = r0 - w0;
      r1 = r1 - w1;
      q0 = 2.0 * ((-al) * a0 - r0);
      q1 = 2.0 * ((-al) * a1 - r1);
    }
    if (MODE == 0) {
      z64 y0 = x0i, y1 = x1i;
      minv<NMAX>(a, S, fs, y0, y1);
      toeplitz<NMAX, false, TP>(S, n, y0, y1);            // A M^-1 v^bar
      double c = 0.0;
      if (root) {
        c = sx2 / phia;
        y0 = y0 - c * q0;
        y1 = y1 - c * q1;
      }
      z64* out = (z64*)a.Y + base;
      if (lane < n) out[(long)lane * a.N] = y0;
      if (lane + 64 < n) out[(long)(lane + 64) * a.N] = y1;
      if (lane == 0) a.cm[fm] = c;
    } else {
      z64 b0 = x0i, b1 = x1i;
      toeplitz<NMAX, true, TP>(S, n, b0, b1);             // A^H w'
      if (root) {
        const double ad = (a.Tdot[f] - wdot(q0, q1, x0i, x1i).x) / phia;
        b0 = b0 - ad * vh0;
        b1 = b1 - ad * vh1;
      }
      minv<NMAX>(a, S, fs, b0, b1);
      if (a.single) {
        z32* out = (z32*)a.Y + base;
        if (lane < n) out[(long)lane * a.N] = cast<float>(b0);
        if (lane + 64 < n) out[(long)(lane + 64) * a.N] = cast<float>(b1);
      } else {
        z64* out = (z64*)a.Y + base;
        if (lane < n) out[(long)lane * a.N] = b0;
        if (lane + 64 < n) out[(long)(lane + 64) * a.N] = b1;
      }
    }
    __syncthreads();
  }
}

// (d) reversed: vbar_f = g u_f / den, ubar_f = (conj(g)(v_f - xi u_f) - g conj(xi) u_f) / den
__global__ __launch_bounds__(256) void k_xi_vjp(const z64* __restrict__ g, const z64* __restrict__ xi,
                                                const z64* __restrict__ u, const z64* __restrict__ v,
                                                long nvox, int F, const double* __restrict__ fw,
                                                z64* __restrict__ vbar, z64* __restrict__ ubar) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox) return;
  double den = 0.0;
  for (int f = 0; f < F; ++f) den += (fw ? fw[f] : 1.0) * nrm2(u[(long)f * nvox + i]);
  const double inv = den > 0.0 ? 1.0 / den : 0.0;
  const z64 gg = g[i], x = xi[i];
  for (int f = 0; f < F; ++f) {
    const double wi = fw ? fw[f] * inv : inv;
    const z64 uu = u[(long)f * nvox + i], vv = v[(long)f * nvox + i];
    vbar[(long)f * nvox + i] = wi * (gg * uu);
    const z64 t = cj(gg) * (vv - x * uu) - gg * (cj(x) * uu);
    ubar[(long)f * nvox + i] = wi * t;
  }
}

// (d) tangent: xi' = sum_f [conj(u) v' + conj(u')(v - xi u) - xi conj(u) u'] / den
__global__ __launch_bounds__(256) void k_xi_jvp(const z64* __restrict__ xi, const z64* __restrict__ u,
                                                const z64* __restrict__ v, const z64* __restrict__ vd,
                                                const z64* __restrict__ ud, long nvox, int F,
                                                const double* __restrict__ fw,
                                                z64* __restrict__ out) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nvox) return;
  double den = 0.0;
  z64 acc = mk(0.0, 0.0);
  const z64 x = xi[i];
  for (int f = 0; f < F; ++f) {
    const long o = (long)f * nvox + i;
    const z64 uu = u[o], vv = v[o], dv = vd[o], du = ud[o];
    if (fw) {
      den += fw[f] * nrm2(uu);
      acc = acc + fw[f] * (cmulc(uu, dv) + cmulc(du, vv - x * uu) - x * cmulc(uu, du));
    } else {
      den += nrm2(uu);
      acc = acc + cmulc(uu, dv) + cmulc(du, vv - x * uu) - x * cmulc(uu, du);
    }
  }
  out[i] = den > 0.0 ? (1.0 / den) * acc : mk(0.0, 0.0);
}

// Tbar[f] = sum_m cm[f * N + m] (fixed order), one block per frequency
__global__ __launch_bounds__(1024) void k_sum_rows(const double* __restrict__ x, long N,
                                                   double* __restrict__ out) {
  // 1024 threads, four independent partial sums each (four loads in flight),
  // then the waves' totals in a fixed order
  __shared__ double red[16];
  const int f = blockIdx.x;
  const double* xf = x + (long)f * N;
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  long i = threadIdx.x;
  for (; i + 3 * 1024 < N; i += 4 * 1024) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s4[u] += xf[i + u * 1024];
  }
  for (; i < N; i += 1024) s4[0] += xf[i];
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  s = lanes_sum<64>(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < 16; ++w) t += red[w];
    out[f] = t;
  }
}

// gW[f] += c * Tbar[f] * W[f]
template <typename TI>
__global__ __launch_bounds__(256) void k_add_noise_term(z64* __restrict__ gW, const cx<TI>* __restrict__ W,
                                                        const double* __restrict__ Tbar, double c,
                                                        long per_f, int F) {
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= per_f * F) return;
  const int f = (int)(i / per_f);
  gW[i] = gW[i] + (c * Tbar[f]) * cast<double>(W[i]);
}

// per-frequency partial sums of Re(conj(a) b): grid (nb, F)
template <typename TI>
__global__ __launch_bounds__(256) void k_dotre(const cx<TI>* __restrict__ a, const cx<TI>* __restrict__ b,
                                               long per_f, double* __restrict__ partial) {
  __shared__ double red[4];
  const int f = blockIdx.y, nb = gridDim.x;
  // four independent partial sums per thread (four loads of each operand in
  // flight)
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  const long step = (long)nb * blockDim.x;
  long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const cx<TI>* af = a + (long)f * per_f;
  const cx<TI>* bf = b + (long)f * per_f;
  for (; i + 3 * step < per_f; i += 4 * step) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const cx<TI> x = af[i + u * step], y = bf[i + u * step];
      s4[u] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
    }
  }
  for (; i < per_f; i += step) {
    const cx<TI> x = af[i], y = bf[i];
    s4[0] += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
  }
  double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  s = lanes_sum<64>(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) partial[f * nb + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void k_finish_dot(const double* __restrict__ partial, int nb, int F, double c,
                             double* __restrict__ out) {
  for (int f = threadIdx.x; f < F; f += blockDim.x) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += partial[f * nb + b];
    out[f] = c * s;
  }
}

}  // namespace fl
