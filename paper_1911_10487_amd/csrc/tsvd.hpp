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

constexpr int TSVD_NMAX = 64;
constexpr int TSVD_PITCH = TSVD_NMAX + 1;  // LDS column pitch (bank spread)

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

// grid-stride over the factorization slots [0, *count); 256 threads: the
// eight threads of pair p (lanes 8p .. 8p + 7) share its column dot products
// and rotations, rows h, h + 8, ... each
__global__ __launch_bounds__(256) void k_tsvd_svd(const z64* __restrict__ dg,
                                                  const z64* __restrict__ sp,
                                                  const int* __restrict__ count, int C, int n,
                                                  double eta, TsvdOut o) {
  __shared__ double M[TSVD_NMAX * TSVD_PITCH];  // column c at M[c * PITCH + r]
  __shared__ double sd[TSVD_NMAX], se[TSVD_NMAX];
  __shared__ z64 sq[TSVD_NMAX], srr[TSVD_NMAX], sy[TSVD_NMAX], sdr[TSVD_NMAX];
  __shared__ double sth;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int total = min(*count, C);
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
    if (wv == 0) dp_phase_scale<TSVD_NMAX>(n, lane, sd, se, sq, srr, sy, sdr);
    __syncthreads();
    if (wv == 0) {
      double f = 0.0;
      for (int i = lane; i < n; i += 64) f += sd[i] * sd[i] + (i + 1 < n ? se[i] * se[i] : 0.0);
      f = lanes_sum<64>(f);
      if (lane == 0) sth = eta * f / n;
    }
    for (int t = tid; t < m2 * TSVD_PITCH; t += 256) {
      const int c = t / TSVD_PITCH, r = t - c * TSVD_PITCH;
      double b = 0.0;
      if (c < n && r < n) b = (r == c) ? sd[c] : (r + 1 == c ? se[r] : 0.0);
      M[t] = b;
    }
    __syncthreads();
    // Pairs of columns whose squared norms are both below th = eta ||B'||_F^2 / n
    // are not rotated: at convergence every other pair is orthogonal, so the
    // columns below th span a subspace whose largest singular value squared
    // is below their summed squared norms, < n th, the floor under which no
    // triplet is kept; the kept triplets are unchanged and their sweeps end
    // in about half the count
    const double th = sth;
    const int p = tid >> 3, h = tid & 7;
    // rows h + 8 s of both columns: the rows past n are zero in M, so
    // every thread handles its eight rows with no bound test and all loads of
    // a round are in flight together
    constexpr int RPT = TSVD_NMAX / 8;
    for (int sweep = 0; sweep < 40; ++sweep) {
      int rot = 0;
      for (int rd = 0; rd < m2 - 1; ++rd) {
        if (p < m2 / 2) {
          int i, j;
          rr_pair(m2, rd, p, i, j);
          double* Mi = M + i * TSVD_PITCH + h;
          double* Mj = M + j * TSVD_PITCH + h;
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
          a += __shfl_xor(a, 1);
          b += __shfl_xor(b, 1);
          c += __shfl_xor(c, 1);
          a += __shfl_xor(a, 2);
          b += __shfl_xor(b, 2);
          c += __shfl_xor(c, 2);
          a += __shfl_xor(a, 4);
          b += __shfl_xor(b, 4);
          c += __shfl_xor(c, 4);
          if (a > 0.0 && b > 0.0 && c * c > tol * tol * (a * b) && (a >= th || b >= th)) {
            rot = 1;
            // the smaller root t of t^2 + 2 z t - 1 = 0, cos = 1 / sqrt(1 + t^2)
            const double z = (b - a) * rcp_nr(2.0 * c);
            const double z2 = fma(z, z, 1.0);
            const double t = copysign(rcp_nr(fabs(z) + z2 * rsq_nr(z2)), z);
            const double cs = rsq_nr(fma(t, t, 1.0)), sn = cs * t;
#pragma unroll
            for (int s2 = 0; s2 < RPT; ++s2) {
              Mi[8 * s2] = cs * x[s2] - sn * y[s2];
              Mj[8 * s2] = sn * x[s2] + cs * y[s2];
            }
          }
        }
        __syncthreads();
      }
      if (!__syncthreads_or(rot)) break;
    }
    // sigma_j = ||M_j||, P_j = M_j / sigma_j, Q_j = B'^T M_j / sigma_j^2 (zero
    // for a zero column)
    for (int j = wv; j < n; j += 4) {
      const double* Mj = M + j * TSVD_PITCH;
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
  long N;
  void* Vh;            // [F][n][N] output
  int vh_single;
  double* alpha;       // [F N]: the truncation index k
  signed char* branch; // [F N]: 0
};

// grid-stride over the active systems, one wave each
__global__ __launch_bounds__(64) void k_tsvd_solve(TsvdArgs a) {
  __shared__ z64 sqp[TSVD_NMAX];
  __shared__ z64 sc[TSVD_NMAX];
  __shared__ double ssig[TSVD_NMAX], sb2[TSVD_NMAX];
  const int lane = threadIdx.x, n = a.n;
  const int total = *a.count;
  const bool on = lane < n;
  for (int sl = blockIdx.x; sl < total; sl += gridDim.x) {
    const int fm = a.list[sl];
    const int f = (int)(fm / a.N);
    const long m = fm - (long)f * a.N;
    const long fs = a.oslot[(long)f * a.N + a.orep[m]];
    // q = U^H w
    z64 x[1];
    x[0] = on ? a.What[((long)f * n + lane) * a.N + m] : mk(0.0, 0.0);
    group_reflect<64, 1, 4>(x, a.refl_l + fs * tri_size(n, 0), a.gam_l + fs * n, n, lane, 0, n - 1, 1, 0);
    const z64 qp = on ? a.s.cdl[fs * n + lane] * x[0] : mk(0.0, 0.0);
    const double sg = on ? a.s.sig[fs * n + lane] : 0.0;
    sqp[lane] = qp;
    ssig[lane] = sg;
    __syncthreads();
    // beta_j = sum_r P[r][j] q'_r (lane j)
    z64 beta = mk(0.0, 0.0);
    const double* P = a.s.P + fs * n * n;
    if (on)
      for (int r = 0; r < n; ++r) {
        const double pr = P[(long)r * n + lane];
        const z64 qr = sqp[r];
        beta.x = fma(pr, qr.x, beta.x);
        beta.y = fma(pr, qr.y, beta.y);
      }
    const double b2 = on ? nrm2(beta) : 0.0;
    // rank of sigma_j in decreasing order (ties by index)
    int rank = 0;
    if (on)
      for (int i = 0; i < n; ++i) {
        const double si = ssig[i];
        rank += (si > sg || (si == sg && i < lane)) ? 1 : 0;
      }
    if (on) sb2[rank] = b2;
    const double wn = lanes_sum<64>(nrm2(qp));
    const double fro = a.fro[fs];
    const int kmax = __popcll(__ballot(on && sg * sg > a.eta * fro));
    // the nb columns with sigma^2 >= 2 eta ||A||_F^2 / n (at least the
    // factorization's threshold for rotating a pair) are orthonormal to
    // every other column; the rest, zero columns included, may not be
    // orthogonal among themselves, so their share of ||q'||^2 (with the part
    // outside the range) is taken as a whole: ||q'||^2 minus the leading share
    const int nb = __popcll(__ballot(on && sg * sg >= 2.0 * a.eta * fro / n));
    const double bh = lanes_sum<64>((on && rank < nb) ? b2 : 0.0);
    const double gs = nb < n ? fmax(0.0, wn - bh) : 0.0;
    __syncthreads();
    // residual after keeping the k = lane leading triplets: the |beta|^2 of
    // the rest of the leading nb summed from the smallest singular value up,
    // plus that share (kmax <= nb, so every count that can be chosen sees
    // the leading terms one by one)
    double acc = 0.0;
    for (int t = nb - 1; t >= lane; --t) acc += sb2[t];
    const double tail = acc + gs;
    // noise-free data: the residual must vanish
    const double T = fmax(a.thr2[f], 0.0);
    const unsigned long long okb = __ballot(on && tail <= T);
    int k = okb ? __ffsll((long long)okb) - 1 : n;
    k = min(k, kmax);
    const bool keep = on && rank < k;
    sc[lane] = (keep && sg > 0.0) ? mk(beta.x / sg, beta.y / sg) : mk(0.0, 0.0);
    __syncthreads();
    // y = D_R Q c (lane r), then v^ = V y
    z64 y[1];
    y[0] = mk(0.0, 0.0);
    const double* Qc = a.s.Qc + fs * n * n;
    if (on) {
      for (int j = 0; j < n; ++j) {
        const double qj = Qc[(long)j * n + lane];
        const z64 cj_ = sc[j];
        y[0].x = fma(qj, cj_.x, y[0].x);
        y[0].y = fma(qj, cj_.y, y[0].y);
      }
      y[0] = a.s.dr[fs * n + lane] * y[0];
    }
    group_reflect<64, 1, 4>(y, a.refl + fs * tri_size(n, 1), a.gam + fs * n, n, lane, n - 3, -1, -1, 1);
    if (on) {
      const long o = ((long)f * n + lane) * a.N + m;
      if (a.vh_single)
        ((z32*)a.Vh)[o] = cast<float>(y[0]);
      else
        ((z64*)a.Vh)[o] = y[0];
    }
    if (lane == 0) {
      a.alpha[fm] = (double)k;
      a.branch[fm] = 0;
    }
    __syncthreads();
  }
}

}  // namespace fl
