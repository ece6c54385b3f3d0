// Truncated SVD of the square systems (Algorithm 2, item 1, with the TSVD
// regularization the paper reports as its best; the truncation index by the
// discrepancy principle), on the shared factorizations of the wavenumber
// orbits:
//
//   k_tsvd_svd
//       one workgroup per factorization: phase-scale the complex bidiagonal
//       B = D_L B' D_R^H to a real one, then one-sided (Hestenes) Jacobi on
//       the dense B' (pairs of columns both far below the truncation floor
//       left unrotated): its columns converge to P Sigma, B' = P Sigma Q^T, and
//       Q = B'^T P Sigma^{-1} (relative error u sigma_1 / sigma_j in column
//       j, which matters only for the triplets that are kept). So
//       A = (U D_L P) Sigma (V D_R Q)^H.
//   k_tsvd_solve
//       one wave per system: q = U^H w from the orbit's left reflectors,
//       beta = P^T D_L^H q, the truncation index k from the ranks of the
//       singular values and the tails of |beta|^2, and
//       v^ = V D_R Q (beta_j / sigma_j over the k largest sigma_j).
#pragma once
#include "solver.hpp"

namespace fl {

constexpr int TSVD_NMAX = 128;  // largest n (the kernels are instantiated for 64 and 128)

struct TsvdOut {
  double* sig;  // [slots][n] singular values of B' (unsorted)
  double* P;    // [slots][n][n] left singular vectors of B', P[r * n + j]
  double* Qc;   // [slots][n][n] right singular vectors of B', Qc[j * n + r]
  z64* cdl;     // [slots][n] conj(D_L)
  z64* dr;      // [slots][n] D_R
};

// Pair p of round r of a round-robin over m2 (even) columns: column 0 stays,
// the others turn on a circle of m2 - 1 places; every pair meets once in
// m2 - 1 rounds.
__device__ __forceinline__ void rr_pair(int m2, int r, int p, int& i, int& j) {
  const int m = m2 - 1;
  if (p == 0) {
    i = 0;
    j = 1 + r % m;
  } else {
    i = 1 + (r + p) % m;
    j = 1 + (r - p + m) % m;
  }
  if (i > j) {
    const int t = i;
    i = j;
    j = t;
  }
}

// grid-stride over the factorization slots [slot0, min(*count, slot0 + C))
// into workspace slots 0..; 4 NMAX threads: the eight threads of pair p
// (lanes 8p .. 8p + 7) share its column dot products and rotations, rows
// h, h + 8, ... each. The dense B' (NMAX x NMAX + 1 doubles: 33 KB at 64,
// 132 KB at 128) lives in LDS.
template <int NMAX>
__global__ __launch_bounds__(4 * NMAX) void k_tsvd_svd(const z64* __restrict__ dg,
                                                       const z64* __restrict__ sp,
                                                       const int* __restrict__ count, int slot0,
                                                       int C, int n, double eta, TsvdOut o) {
  constexpr int PITCH = NMAX + 1;  // LDS column pitch (bank spread)
  constexpr int NT = 4 * NMAX, NWV = NT / 64;
  __shared__ double M[NMAX * PITCH];  // column c at M[c * PITCH + r]
  __shared__ double sd[NMAX], se[NMAX];
  __shared__ z64 sq[NMAX], srr[NMAX], sy[NMAX], sdr[NMAX];
  __shared__ double sth;
  __shared__ double cn[NMAX];  // squared column norms of M
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int total = min(*count - slot0, C);
  const int m2 = n + (n & 1);  // a zero column pads an odd n
  const double tol = 2.2e-16 * n;
  for (int sl = blockIdx.x; sl < total; sl += gridDim.x) {
    if (wv == 0) {
      for (int i = lane; i < n; i += 64) {
        sy[i] = dg[(long)sl * n + i];
        srr[i] = sp[(long)sl * n + i];
        sq[i] = mk(1.0, 0.0);
      }
    }
    __syncthreads();
    // sq becomes conj(D_L), sdr D_R
    if (wv == 0) dp_phase_scale<NMAX>(n, lane, sd, se, sq, srr, sy, sdr);
    __syncthreads();
    if (wv == 0) {
      double f = 0.0;
      for (int i = lane; i < n; i += 64) f += sd[i] * sd[i] + (i + 1 < n ? se[i] * se[i] : 0.0);
      f = lanes_sum<64>(f);
      if (lane == 0) sth = eta * f / n;
    }
    for (int t = tid; t < m2 * PITCH; t += NT) {
      const int c = t / PITCH, r = t - c * PITCH;
      double b = 0.0;
      if (c < n && r < n) b = (r == c) ? sd[c] : (r + 1 == c ? se[r] : 0.0);
      M[t] = b;
    }
    __syncthreads();
    for (int cc = tid; cc < m2; cc += NT) {
      double f = 0.0;
      for (int r = 0; r < n; ++r) f = fma(M[cc * PITCH + r], M[cc * PITCH + r], f);
      cn[cc] = f;
    }
    __syncthreads();
    // Pairs of columns whose squared norms are both below th = eta ||B'||_F^2 / n
    // are not rotated: at convergence every other pair is orthogonal, so the
    // columns below th span a subspace whose largest singular value squared
    // is below their summed squared norms, < n th, the floor under which no
    // triplet is kept; the kept triplets are unchanged and their sweeps end
    // in about half the count. The squared column norms are kept in cn (exact
    // sums over the column after every load or rotation), so such a pair is
    // not even loaded: most pairs of a sweep are (about ten of the 128 columns
    // of a bench orbit lie above the floor). The margin keeps a column whose
    // kept norm rounds just below th in the exact test.
    const double th = sth, thm = th * (1.0 - 1e-9);
    const int p = tid >> 3, h = tid & 7;
    // rows h + 8 s of both columns: the rows past n are zero in M, so
    // every thread handles its eight rows with no bound test and all loads of
    // a round are in flight together
    constexpr int RPT = NMAX / 8;
    for (int sweep = 0; sweep < 40; ++sweep) {
      int rot = 0;
      for (int rd = 0; rd < m2 - 1; ++rd) {
        int i = 0, j = 0;
        if (p < m2 / 2) rr_pair(m2, rd, p, i, j);
        if (p < m2 / 2 && (cn[i] >= thm || cn[j] >= thm)) {
          double* Mi = M + i * PITCH + h;
          double* Mj = M + j * PITCH + h;
          double x[RPT], y[RPT];
#pragma unroll
          for (int s2 = 0; s2 < RPT; ++s2) {
            x[s2] = Mi[8 * s2];
            y[s2] = Mj[8 * s2];
          }
          double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
          for (int s2 = 0; s2 < RPT; ++s2) {
            a = fma(x[s2], x[s2], a);
            b = fma(y[s2], y[s2], b);
            c = fma(x[s2], y[s2], c);
          }
          // sums over the pair's eight lanes by DPP moves (partners lane ^ 1,
          // lane ^ 2, then the other four of the eight), not through the LDS
          // crossbar, which the column loads already keep busy
          a += dpp_d<0xB1>(a);
          b += dpp_d<0xB1>(b);
          c += dpp_d<0xB1>(c);
          a += dpp_d<0x4E>(a);
          b += dpp_d<0x4E>(b);
          c += dpp_d<0x4E>(c);
          a += dpp_d<0x141>(a);
          b += dpp_d<0x141>(b);
          c += dpp_d<0x141>(c);
          if (a > 0.0 && b > 0.0 && c * c > tol * tol * (a * b) && (a >= th || b >= th)) {
            rot = 1;
            // the smaller root t of t^2 + 2 z t - 1 = 0, cos = 1 / sqrt(1 + t^2)
            const double z = (b - a) * rcp_nr(2.0 * c);
            const double z2 = fma(z, z, 1.0);
            const double t = copysign(rcp_nr(fabs(z) + z2 * rsq_nr(z2)), z);
            const double cs = rsq_nr(fma(t, t, 1.0)), sn = cs * t;
            double a2 = 0.0, b2 = 0.0;
#pragma unroll
            for (int s2 = 0; s2 < RPT; ++s2) {
              const double xr = cs * x[s2] - sn * y[s2], yr = sn * x[s2] + cs * y[s2];
              Mi[8 * s2] = xr;
              Mj[8 * s2] = yr;
              a2 = fma(xr, xr, a2);
              b2 = fma(yr, yr, b2);
            }
            a2 += dpp_d<0xB1>(a2);
            b2 += dpp_d<0xB1>(b2);
            a2 += dpp_d<0x4E>(a2);
            b2 += dpp_d<0x4E>(b2);
            a2 += dpp_d<0x141>(a2);
            b2 += dpp_d<0x141>(b2);
            a = a2;
            b = b2;
          }
          if (h == 0) {
            cn[i] = a;
            cn[j] = b;
          }
        }
        __syncthreads();
      }
      if (!__syncthreads_or(rot)) break;
    }
    // sigma_j = ||M_j||, P_j = M_j / sigma_j, Q_j = B'^T M_j / sigma_j^2 (zero
    // for a zero column)
    for (int j = wv; j < n; j += NWV) {
      const double* Mj = M + j * PITCH;
      double s = 0.0;
      for (int r = lane; r < n; r += 64) s = fma(Mj[r], Mj[r], s);
      s = lanes_sum<64>(s);
      const double sg = sqrt(s);
      const double is = sg > 0.0 ? 1.0 / sg : 0.0;
      if (lane == 0) o.sig[(long)sl * n + j] = sg;
      double* P = o.P + (long)sl * n * n;
      double* Qc = o.Qc + (long)sl * n * n;
      for (int r = lane; r < n; r += 64) {
        P[(long)r * n + j] = Mj[r] * is;
        const double bt = sd[r] * Mj[r] + (r > 0 ? se[r - 1] * Mj[r - 1] : 0.0);
        Qc[(long)j * n + r] = bt * is * is;
      }
    }
    if (wv == 0) {
      for (int i = lane; i < n; i += 64) {
        o.cdl[(long)sl * n + i] = sq[i];
        o.dr[(long)sl * n + i] = sdr[i];
      }
    }
    __syncthreads();
  }
}

struct TsvdArgs {
  const z64* What;     // [F][n][N]
  const int* list;     // active systems grouped by orbit
  const int* count;
  const int* oslot;    // [F N] factorization slot of (f, representative)
  const int* orep;     // [N]
  const z64* refl_l;   // left reflectors per slot
  const double* gam_l;
  const z64* refl;     // right reflectors per slot
  const double* gam;
  const double* fro;   // ||A||_F^2 per slot
  TsvdOut s;
  const double* thr2;  // per frequency (tau delta_m)^2, < 0 for noise-free data
  double eta;
  int n;
  int nd, nzv;         // data planes and X planes (n for square Toeplitz systems)
  long N;
  void* Vh;            // [F][nzv][N] output
  int vh_single;
  double* alpha;       // [F N]: the truncation index k
  signed char* branch; // [F N]: 0
  // orbit chunks (NULL: every active orbit has a slot)
  const int* osys0;
  const int* ocount;
  int slot0, OC;
};

// One wave per system, each lane holding entries lane + 64 e (E of them);
// with orbit chunks (osys0 not NULL) the systems of compacted orbits
// [slot0, slot0 + OC), factorizations in workspace slots oslot - slot0.
template <int NMAX>
__global__ __launch_bounds__(64) void k_tsvd_solve(TsvdArgs a) {
  constexpr int E = NMAX / 64;
  __shared__ z64 sqp[NMAX];
  __shared__ z64 sc[NMAX], sbeta[NMAX];
  __shared__ double ssig[NMAX], sb2[NMAX];
  __shared__ int slead[NMAX];
  const int lane = threadIdx.x, n = a.n;
  const int total = *a.count;
  int c0;
  const int nsys = launch_range(a.osys0, a.ocount, a.slot0, a.OC, 0, total, total, &c0);
  bool on[E];
#pragma unroll
  for (int e = 0; e < E; ++e) on[e] = lane + 64 * e < n;
  for (int sl = blockIdx.x; sl < nsys; sl += gridDim.x) {
    const int fm = a.list[c0 + sl];
    const int f = (int)(fm / a.N);
    const long m = fm - (long)f * a.N;
    const long fs = a.oslot[(long)f * a.N + a.orep[m]] - a.slot0;
    // q = U^H w
    z64 x[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
      x[e] = lane + 64 * e < a.nd ? a.What[((long)f * a.nd + lane + 64 * e) * a.N + m]
                                  : mk(0.0, 0.0);
    group_reflect<64, E, 4>(x, a.refl_l + fs * tri_size(n, 0), a.gam_l + fs * n, n, lane, 0, n - 1,
                            1, 0);
    z64 qp[E];
    double sg[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = lane + 64 * e;
      qp[e] = on[e] ? a.s.cdl[fs * n + i] * x[e] : mk(0.0, 0.0);
      sg[e] = on[e] ? a.s.sig[fs * n + i] : 0.0;
      if (on[e]) {
        sqp[i] = qp[e];
        ssig[i] = sg[e];
      }
    }
    __syncthreads();
    // beta_j = sum_r P[r][j] q'_r (j = lane + 64 e)
    const double* P = a.s.P + fs * n * n;
    z64 beta[E];
    double b2[E];
    int rank[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int j = lane + 64 * e;
      z64 bt = mk(0.0, 0.0);
      if (on[e])
        for (int r = 0; r < n; ++r) {
          const double pr = P[(long)r * n + j];
          const z64 qr = sqp[r];
          bt.x = fma(pr, qr.x, bt.x);
          bt.y = fma(pr, qr.y, bt.y);
        }
      beta[e] = bt;
      b2[e] = on[e] ? nrm2(bt) : 0.0;
      // rank of sigma_j in decreasing order (ties by index)
      int rk = 0;
      if (on[e])
        for (int i = 0; i < n; ++i) {
          const double si = ssig[i];
          rk += (si > sg[e] || (si == sg[e] && i < j)) ? 1 : 0;
        }
      rank[e] = rk;
      if (on[e]) sb2[rk] = b2[e];
    }
    const double fro = a.fro[fs];
    int kmax = 0, nb = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      kmax += __popcll(__ballot(on[e] && sg[e] * sg[e] > a.eta * fro));
      // the nb columns with sigma^2 >= 2 eta ||A||_F^2 / n (at least the
      // factorization's threshold for rotating a pair) are orthonormal to
      // every other column
      nb += __popcll(__ballot(on[e] && sg[e] * sg[e] >= 2.0 * a.eta * fro / n));
    }
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (on[e]) {
        sbeta[lane + 64 * e] = beta[e];
        slead[lane + 64 * e] = rank[e] < nb;
      }
    __syncthreads();
    // The other columns, zero columns included, may not be orthogonal among
    // themselves, so their share of ||q'||^2 (with the part outside the
    // range) is taken as a whole, as the squared norm of the residual
    // r = q' - sum_lead beta_j P_j (formed explicitly: a difference of
    // squared norms would carry an error of u ||q'||^2, far above
    // (tau delta_m)^2 for small delta).
    double gs = 0.0;
    if (nb < n) {
      double rr = 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        z64 r = qp[e];
        if (on[e])
          for (int j = 0; j < n; ++j)
            if (slead[j]) {
              const double pr = P[(long)(lane + 64 * e) * n + j];
              const z64 bj = sbeta[j];
              r.x = fma(-pr, bj.x, r.x);
              r.y = fma(-pr, bj.y, r.y);
            }
        rr += on[e] ? nrm2(r) : 0.0;
      }
      gs = lanes_sum<64>(rr);
    }
    // residual after keeping the k leading triplets (k = lane + 64 e): the
    // |beta|^2 of the rest of the leading nb summed from the smallest
    // singular value up, plus that share (kmax <= nb, so every count that
    // can be chosen sees the leading terms one by one)
    // noise-free data: the residual must vanish
    const double T = fmax(a.thr2[f], 0.0);
    int k = n;
#pragma unroll
    for (int e = E - 1; e >= 0; --e) {
      const int kk = lane + 64 * e;
      double acc = 0.0;
      for (int t = nb - 1; t >= kk; --t) acc += sb2[t];
      const unsigned long long okb = __ballot(kk < n && acc + gs <= T);
      if (okb) k = 64 * e + __ffsll((long long)okb) - 1;
    }
    k = min(k, kmax);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (on[e]) {
        const bool keep = rank[e] < k;
        sc[lane + 64 * e] =
            (keep && sg[e] > 0.0) ? mk(beta[e].x / sg[e], beta[e].y / sg[e]) : mk(0.0, 0.0);
      }
    __syncthreads();
    // y = D_R Q c (entry r = lane + 64 e), then v^ = V y
    z64 y[E];
    const double* Qc = a.s.Qc + fs * n * n;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int r = lane + 64 * e;
      y[e] = mk(0.0, 0.0);
      if (on[e]) {
        for (int j = 0; j < n; ++j) {
          const double qj = Qc[(long)j * n + r];
          const z64 cj_ = sc[j];
          y[e].x = fma(qj, cj_.x, y[e].x);
          y[e].y = fma(qj, cj_.y, y[e].y);
        }
        y[e] = a.s.dr[fs * n + r] * y[e];
      }
    }
    group_reflect<64, E, 4>(y, a.refl + fs * tri_size(n, 1), a.gam + fs * n, n, lane, n - 3, -1,
                            -1, 1);
#pragma unroll
    for (int e = 0; e < E; ++e)
      if (lane + 64 * e < a.nzv) {
        const long o = ((long)f * a.nzv + lane + 64 * e) * a.N + m;
        if (a.vh_single)
          ((z32*)a.Vh)[o] = cast<float>(y[e]);
        else
          ((z64*)a.Vh)[o] = y[e];
      }
    if (lane == 0) {
      a.alpha[fm] = (double)k;
      a.branch[fm] = 0;
    }
    __syncthreads();
  }
}

}  // namespace fl
