// Item 1 of Algorithm 2 on the shared factorization of a symmetry orbit,
// orbit by orbit: the members of an orbit (at one frequency) are the systems
// A_m v = w_m with the same A (Section 5's kernel is radial, so every member
// of the orbit of m under the torus symmetries has the same table row), each
// with its own data, noise level and discrepancy-chosen alpha. Three launches
// per orbit chunk, all on the factorizations the bidiagonalization left in
// the workspace:
//
//   k_dpo_prep    one wave per orbit: the phase scaling of the orbit's
//                 complex bidiagonal to the real B' (kept per slot with the
//                 right phases), then q = U^H w for every member at once
//                 (one pass over the left reflectors; each reflector is
//                 loaded once and its inner products with all members are
//                 summed over the wave together) and q' = D_L^H q.
//   k_dpo_search  SPW systems per wave, each in a group of 64 / SPW lanes:
//                 the multisection discrepancy search on B' and q' (the
//                 same search as k_dp_solve), the Elden solve, D_R y.
//   k_dpo_back    one wave per orbit: v^ = V (D_R y) for every member at
//                 once (one pass over the right reflectors), v^ = 0 for the
//                 members whose data lie within the noise level.
#pragma once
#include "solver.hpp"

namespace fl {

constexpr int DPO_MEMBERS = 8;  // members of an orbit (torus symmetries of m)

// Householder reflectors applied to VP vectors at once by one wave (element
// i of vector j held by lane i % 64 in slot i / 64): x_j <- H_k x_j for
// k = k0, k0 + dk, ... while k has not reached kend, H_k = I - g_k h_k h_k^H
// with h_k the packed reflector k of R (entries k + off .. n - 1). The VP
// inner products with a reflector are summed over the wave together
// (group_sums), so a reflector row is fetched once for all vectors. The
// reflectors go in batches of RG; the next batch is loaded while the current
// one is applied, so that its latency overlaps the work.
template <int RG, int E>
__device__ __forceinline__ void wave_reflect_load(z64 (&h)[RG][E], double (&gg)[RG],
                                                  const z64* __restrict__ R,
                                                  const double* __restrict__ gam, int n, int lane,
                                                  int kb, int kend, int dk, int off) {
#pragma unroll
  for (int g = 0; g < RG; ++g) {
    const int k = kb + dk * g;
    const bool ok = dk > 0 ? k < kend : k > kend;
    gg[g] = ok ? gam[k] : 0.0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = lane + 64 * e;
      h[g][e] = (ok && i >= k + off && i < n) ? R[tri_start(k, n, off) + (i - k - off)]
                                               : mk(0.0, 0.0);
    }
  }
}

template <int VP, int E, int RG>
__device__ __forceinline__ void wave_reflect(z64 (&x)[VP][E], const z64* __restrict__ R,
                                             const double* __restrict__ gam, int n, int lane,
                                             int k0, int kend, int dk, int off, z64* gat) {
  if (!(dk > 0 ? k0 < kend : k0 > kend)) return;
  z64 hn[RG][E];
  double gn[RG];
  wave_reflect_load<RG, E>(hn, gn, R, gam, n, lane, k0, kend, dk, off);
  for (int kb = k0; dk > 0 ? kb < kend : kb > kend; kb += dk * RG) {
    z64 h[RG][E];
    double gg[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      gg[g] = gn[g];
#pragma unroll
      for (int e = 0; e < E; ++e) h[g][e] = hn[g][e];
    }
    const int kn = kb + dk * RG;
    if (dk > 0 ? kn < kend : kn > kend)
      wave_reflect_load<RG, E>(hn, gn, R, gam, n, lane, kn, kend, dk, off);
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      z64 d[VP];
#pragma unroll
      for (int j = 0; j < VP; ++j) {
        z64 t = mk(0.0, 0.0);
#pragma unroll
        for (int e = 0; e < E; ++e) t = cfmac(t, h[g][e], x[j][e]);
        d[j] = t;
      }
      group_sums<64, VP>(d, gat, lane);
#pragma unroll
      for (int j = 0; j < VP; ++j) {
        const z64 s = gg[g] * d[j];
#pragma unroll
        for (int e = 0; e < E; ++e) x[j][e] = cfms(x[j][e], h[g][e], s);
      }
    }
  }
}

// reflector rows loaded ahead per batch (register budget of three waves per
// SIMD)
template <int NMAX, int VP>
constexpr int dpo_rg() {
  return NMAX > 64 ? (VP >= 8 ? 2 : 4) : (VP >= 8 ? 4 : 8);
}

// members [p0, p0 + c) of the orbit in slot s: q' = D_L^H U^H w into qy
template <int NMAX, int VP>
__device__ __forceinline__ void dpo_q(const DpArgs& a, int s, int p0, int c, int c0,
                                      const z64* sdl, z64* gat, int lane) {
  constexpr int E = NMAX / 64;
  const int n = a.n;
  z64 x[VP][E];
#pragma unroll
  for (int j = 0; j < VP; ++j) {
    long f = 0, m = 0;
    if (j < c) {
      const int fm = a.list[p0 + j];
      f = fm / a.N;
      m = fm - f * a.N;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = lane + 64 * e;
      x[j][e] = (j < c && i < a.nd) ? a.What[(f * a.nd + i) * a.N + m] : mk(0.0, 0.0);
    }
  }
  wave_reflect<VP, E, dpo_rg<NMAX, VP>()>(x, a.refl_l + (long)s * tri_size(n, 0),
                                          a.gam_l + (long)s * n, n, lane, 0, n - 1, 1, 0, gat);
#pragma unroll
  for (int j = 0; j < VP; ++j) {
    if (j < c) {
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        if (i < n) a.qy[(long)(p0 + j - c0) * n + i] = cmulc(sdl[i], x[j][e]);
      }
    }
  }
}

// the launch's orbit of this workgroup: slot s, members [*p0, *p0 + c), and
// the launch's first system c0; false when the slot holds no active orbit
__device__ __forceinline__ bool dpo_orbit(const DpArgs& a, int s, int* p0, int* c, int* c0) {
  const int oc = *a.ocount;
  const int o = a.slot0 + s;
  if (s >= a.OC || o >= oc) return false;
  *c0 = a.osys0[min(a.slot0, oc)];
  *p0 = a.osys0[o];
  *c = min(a.osys0[o + 1] - *p0, DPO_MEMBERS);
  return *c > 0;
}

template <int NMAX>
__global__ __launch_bounds__(64) void k_dpo_prep(DpArgs a) {
  __shared__ double sd[NMAX], se[NMAX];
  __shared__ z64 sy[NMAX], srr[NMAX], sdr[NMAX], sdl[NMAX];
  __shared__ z64 gat[DPO_MEMBERS];
  const int lane = threadIdx.x, n = a.n, s = blockIdx.x;
  int p0, c, c0;
  if (!dpo_orbit(a, s, &p0, &c, &c0)) return;
  for (int i = lane; i < n; i += 64) {
    sy[i] = a.dg[(long)s * n + i];
    srr[i] = a.sp[(long)s * n + i];
  }
  __syncthreads();
  dp_phase_scale<NMAX>(n, lane, sd, se, nullptr, srr, sy, sdr, sdl);
  __syncthreads();
  for (int i = lane; i < n; i += 64) {
    a.bd_d[(long)s * n + i] = sd[i];
    a.bd_e[(long)s * n + i] = se[i];
    a.bd_dr[(long)s * n + i] = sdr[i];
  }
  if (c <= 1)
    dpo_q<NMAX, 1>(a, s, p0, c, c0, sdl, gat, lane);
  else if (c <= 2)
    dpo_q<NMAX, 2>(a, s, p0, c, c0, sdl, gat, lane);
  else if (c <= 4)
    dpo_q<NMAX, 4>(a, s, p0, c, c0, sdl, gat, lane);
  else
    dpo_q<NMAX, 8>(a, s, p0, c, c0, sdl, gat, lane);
}

// SPW systems per single-wave workgroup, each in a group of G = 64 / SPW
// lanes: the discrepancy search (G trial alphas per round), the Elden solve
// by the group's first lane, and D_R y back into qy.
template <int NMAX, int SPW>
__global__ __launch_bounds__(64) void k_dpo_search(DpArgs a) {
  constexpr int G = 64 / SPW;
  __shared__ double sd[SPW][NMAX], se[SPW][NMAX];
  __shared__ z64 sq[SPW][NMAX];
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  const int n = a.n;
  const int oc = *a.ocount;
  const int c0 = a.osys0[min(a.slot0, oc)];
  const int nsys = a.osys0[min(a.slot0 + a.OC, oc)] - c0;
  const int nact = nsys > 0 ? (nsys + SPW - 1) / SPW : 0;
  // Workgroups go to the eight XCDs in turn: XCD x (of V = min(8, grid))
  // takes the contiguous group range [x per, (x + 1) per), so that the
  // members of an orbit (consecutive systems) share an L2.
  const int NG = gridDim.x, V = NG < 8 ? NG : 8;
  const int xcd = blockIdx.x % V, nbx = (NG - xcd + V - 1) / V;
  const int per = (nact + V - 1) / V;
  for (int k = blockIdx.x / V; k < per; k += nbx) {
    const int sg = xcd * per + k;
    if (sg >= nact) break;
    const int sl = sg * SPW + grp;  // the group's system, relative to c0
    const bool live = sl < nsys;
    int fm = 0, f = 0;
    long fs = 0;
    if (live) {
      fm = a.list[c0 + sl];
      f = (int)(fm / a.N);
      const long m = fm - (long)f * a.N;
      fs = a.oslot[(long)f * a.N + a.orep[m]] - a.slot0;
      for (int i = gl; i < n; i += G) {
        sd[grp][i] = a.bd_d[fs * n + i];
        se[grp][i] = a.bd_e[fs * n + i];
        sq[grp][i] = a.qy[(long)sl * n + i];
      }
    }
    __syncthreads();
    double al = 0.0;
    int br = 0;
    if (live)
      br = dp_choose_alpha<G>(n, lane, sd[grp], se[grp], sq[grp], a.thr2[f], a.fro[fs], a.eta, &al);
    __syncthreads();
    // rho, off, the rotated right-hand side and y overwrite d, e and q' in place
    if (live && br != 0 && gl == 0)
      elden_solve(sd[grp], se[grp], sq[grp], n, al, sd[grp], se[grp], sq[grp], sq[grp]);
    __syncthreads();
    if (live) {
      if (br != 0)
        for (int i = gl; i < n; i += G) a.qy[(long)sl * n + i] = a.bd_dr[fs * n + i] * sq[grp][i];
      if (gl == 0) {
        a.alpha[fm] = br != 0 ? al : INFINITY;
        a.branch[fm] = (signed char)br;
      }
    }
    __syncthreads();
  }
}

// members [p0, p0 + c) of the orbit in slot s: v^ = V (D_R y), or 0 for a
// member within the noise level
template <int NMAX, int VP>
__device__ __forceinline__ void dpo_v(const DpArgs& a, int s, int p0, int c, int c0, z64* gat,
                                      int lane) {
  constexpr int E = NMAX / 64;
  const int n = a.n;
  z64 x[VP][E];
  long fj[VP], mj[VP];
#pragma unroll
  for (int j = 0; j < VP; ++j) {
    bool on = false;
    fj[j] = 0;
    mj[j] = 0;
    if (j < c) {
      const int fm = a.list[p0 + j];
      fj[j] = fm / a.N;
      mj[j] = fm - fj[j] * a.N;
      on = a.branch[fm] != 0;
    }
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int i = lane + 64 * e;
      x[j][e] = (on && i < n) ? a.qy[(long)(p0 + j - c0) * n + i] : mk(0.0, 0.0);
    }
  }
  // V = P_0 P_1 ... P_{n-3}: apply P_{n-3} first
  wave_reflect<VP, E, dpo_rg<NMAX, VP>()>(x, a.refl + (long)s * tri_size(n, 1), a.gam + (long)s * n,
                                          n, lane, n - 3, -1, -1, 1, gat);
#pragma unroll
  for (int j = 0; j < VP; ++j) {
    if (j < c) {
      const long o0 = fj[j] * a.nzv * a.N + mj[j];
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = lane + 64 * e;
        if (i < a.nzv) {
          if (a.vh_single)
            ((z32*)a.Vh)[o0 + (long)i * a.N] = cast<float>(x[j][e]);
          else
            ((z64*)a.Vh)[o0 + (long)i * a.N] = x[j][e];
        }
      }
    }
  }
}

template <int NMAX>
__global__ __launch_bounds__(64) void k_dpo_back(DpArgs a) {
  __shared__ z64 gat[DPO_MEMBERS];
  const int lane = threadIdx.x, s = blockIdx.x;
  int p0, c, c0;
  if (!dpo_orbit(a, s, &p0, &c, &c0)) return;
  if (c <= 1)
    dpo_v<NMAX, 1>(a, s, p0, c, c0, gat, lane);
  else if (c <= 2)
    dpo_v<NMAX, 2>(a, s, p0, c, c0, gat, lane);
  else if (c <= 4)
    dpo_v<NMAX, 4>(a, s, p0, c, c0, gat, lane);
  else
    dpo_v<NMAX, 8>(a, s, p0, c, c0, gat, lane);
}

}  // namespace fl
