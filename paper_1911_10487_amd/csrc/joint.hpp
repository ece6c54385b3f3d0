// Item 1 of Algorithm 2 solved as one system over the frequencies (Section 4,
// comment c; fl_opts.alpha_rule = 2): for a wavenumber m the frequencies'
// systems form the block-diagonal system diag(A_1m, ..., A_Fm) v = w, which
// is regularized as one system: one Tikhonov parameter alpha_m, chosen by the
// discrepancy principle on the stacked data,
//   sum_f ||A_fm v_f - w_fm||^2 = tau^2 sum_f delta_fm^2,
// alpha_m >= eta sum_f ||A_fm||_F^2, and v = 0 at every frequency when
// sum_f ||w_fm||^2 <= tau^2 sum_f delta_fm^2. Block diagonal: v_f is
// frequency f's Tikhonov solution at alpha_m.
//
//   k_joint_classify
//       per wavenumber: the stacked data norm against the stacked noise
//       level; flags every selected frequency's system of an active m (and
//       zeroes v^ of the systems it unflags) and m itself.
//   k_joint_solve
//       one wave per active wavenumber: q = U^H w and the phase scaling of
//       each frequency's system on its orbit's factorization, the discrepancy
//       search on the summed discrepancy (the per-system search with a
//       different phi), then every frequency's Elden solve at the common
//       alpha (one lane each) and back-transform v^ = V y.
#pragma once
#include "solver.hpp"

namespace fl {

constexpr int JOINT_FMAX = 8;  // frequencies of one stacked system

// thread per wavenumber m; wn2 and flag from k_classify run with every
// nonzero system flagged
__global__ __launch_bounds__(256) void k_joint_classify(const double* __restrict__ wn2, long N,
                                                        int F, const double* __restrict__ thr2,
                                                        const double* __restrict__ fw,
                                                        int* __restrict__ flag,
                                                        int* __restrict__ mflag, void* __restrict__ Vh,
                                                        int vh_single, int nz) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  double S = 0.0, T = 0.0;
  bool noise_free = false;
  for (int f = 0; f < F; ++f) {
    if (fw && fw[f] == 0.0) continue;
    S += wn2[(long)f * N + m];
    if (thr2[f] < 0.0)
      noise_free = true;
    else
      T += thr2[f];
  }
  const int act = noise_free ? (S > 0.0) : (S > T);
  mflag[m] = act;
  for (int f = 0; f < F; ++f) {
    const long fm = (long)f * N + m;
    const int a = act && !(fw && fw[f] == 0.0);
    if (!a && flag[fm]) {
      const long o0 = (long)f * nz * N + m;
      if (vh_single)
        for (int j = 0; j < nz; ++j) ((z32*)Vh)[o0 + (long)j * N] = mk(0.f, 0.f);
      else
        for (int j = 0; j < nz; ++j) ((z64*)Vh)[o0 + (long)j * N] = mk(0.0, 0.0);
    }
    flag[fm] = a;
  }
}

struct JointArgs {
  const int* mlist;   // active wavenumbers, compacted
  const int* mcount;
  const int* flag;    // [F N] systems taking part
  int F, n;
  int nd, nzv;        // data planes and X planes (n for square Toeplitz systems)
  long N;
  const double* thr2;
  double eta;
  // orbit factorizations (every active orbit resident): slot
  // oslot[f N + orep[m]] of dg, sp, fro, the packed reflectors and gammas
  const int* oslot;
  const int* orep;
  const z64* dg;
  const z64* sp;
  const double* fro;
  const z64* refl;
  const double* gam;
  const z64* refl_l;
  const double* gam_l;
  const z64* What;    // [F][nd][N]
  void* Vh;           // [F][nzv][N] output
  int vh_single;
  double* alpha;      // [F N]
  signed char* branch;
};

template <int NMAX>
__global__ __launch_bounds__(64) void k_joint_solve(JointArgs a) {
  constexpr int E = NMAX / 64;
  constexpr int RG = E >= 2 ? 2 : 4;
  // per frequency of the stack: real bidiagonal (overwritten by the Elden
  // factors), q', right phases, the Elden right-hand side and solution; the
  // complex bidiagonal of the system being phase-scaled
  __shared__ double sd[JOINT_FMAX][NMAX], se[JOINT_FMAX][NMAX];
  __shared__ z64 sq[JOINT_FMAX][NMAX], sdr[JOINT_FMAX][NMAX];
  __shared__ z64 srr[JOINT_FMAX][NMAX], sy[JOINT_FMAX][NMAX];
  __shared__ z64 cy[NMAX], cs[NMAX];
  const int lane = threadIdx.x, n = a.n;
  const int count = *a.mcount;
  for (int g = blockIdx.x; g < count; g += gridDim.x) {
    const int m = a.mlist[g];
    int fl[JOINT_FMAX];
    int nf = 0;
    double T = 0.0, fro = 0.0;
    bool noise_free = false;
    for (int f = 0; f < a.F; ++f)
      if (a.flag[(long)f * a.N + m]) {
        fl[nf++] = f;
        const int slot = a.oslot[(long)f * a.N + a.orep[m]];
        fro += a.fro[slot];
        if (a.thr2[f] < 0.0)
          noise_free = true;
        else
          T += a.thr2[f];
      }
    if (noise_free) T = -1.0;
    // q = U^H w and the phase scaling, one frequency after another
    for (int k = 0; k < nf; ++k) {
      const int f = fl[k];
      const long slot = a.oslot[(long)f * a.N + a.orep[m]];
      for (int i = lane; i < n; i += 64) {
        cy[i] = a.dg[slot * n + i];
        cs[i] = a.sp[slot * n + i];
      }
      z64 x[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        x[e] = i < a.nd ? a.What[((long)f * a.nd + i) * a.N + m] : mk(0.0, 0.0);
      }
      group_reflect<64, E, RG>(x, a.refl_l + slot * tri_size(n, 0), a.gam_l + slot * n, n, lane, 0,
                               n - 1, 1, 0);
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        if (i < n) sq[k][i] = x[e];
      }
      __syncthreads();
      dp_phase_scale<NMAX>(n, lane, sd[k], se[k], sq[k], cs, cy, sdr[k]);
      __syncthreads();
    }
    // one alpha for the stack: the summed discrepancy, the stacked floor
    double al = 0.0;
    const int br = dp_choose_alpha_f<64>(
        lane,
        [&](double x) {
          double s = 0.0;
          for (int k = 0; k < nf; ++k) s += phi_fwd(sd[k], se[k], sq[k], n, x);
          return s;
        },
        T, fro, a.eta, &al);
    __syncthreads();
    // every frequency's Elden solve at alpha, one lane each
    if (lane < nf) elden_solve(sd[lane], se[lane], sq[lane], n, al, sd[lane], se[lane], srr[lane],
                               sy[lane]);
    __syncthreads();
    for (int k = 0; k < nf; ++k) {
      const int f = fl[k];
      const long slot = a.oslot[(long)f * a.N + a.orep[m]];
      // v^ = V (D_R y), V = P_0 P_1 ... P_{n-3}: apply P_{n-3} first
      z64 y[E];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        y[e] = i < n ? sdr[k][i] * sy[k][i] : mk(0.0, 0.0);
      }
      group_reflect<64, E, RG>(y, a.refl + slot * tri_size(n, 1), a.gam + slot * n, n, lane, n - 3,
                               -1, -1, 1);
      const long o0 = (long)f * a.nzv * a.N + m;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        if (i < a.nzv) {
          if (a.vh_single)
            ((z32*)a.Vh)[o0 + (long)i * a.N] = cast<float>(y[e]);
          else
            ((z64*)a.Vh)[o0 + (long)i * a.N] = y[e];
        }
      }
      if (lane == 0) {
        a.alpha[(long)f * a.N + m] = al;
        a.branch[(long)f * a.N + m] = (signed char)br;
      }
    }
    __syncthreads();
  }
}

}  // namespace fl
