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
//   k_dp_solve
//       one wave per 1, 2 or 4 systems, each in its own group of lanes:
//       phase-scale B to a real bidiagonal, pick alpha by the discrepancy
//       principle with a multisection on log(alpha) (each lane evaluates the
//       discrepancy at its own alpha in one O(n) pass), solve at the chosen
//       alpha by Elden's Givens QR of [B; sqrt(alpha) I], and back-transform
//       v^ = V y into the plane-major array.
#pragma once
#include "common.hpp"

namespace fl {

// ---------------------------------------------------------------- classify

// thread per (f, m): wn2 = sum_j |W^[f][j][m]|^2; flag = system needs a solve.
// v^ of a system without a solve is zero: the plan starts with v^ = 0 and
// flag = 0, the solvers write v^ of every flagged system, and this kernel
// zeroes v^ of a system flagged by the previous call and not by this one.
template <typename T>
__global__ __launch_bounds__(256) void k_classify(const cx<T>* __restrict__ What, int nd, long N,
                                                  int F, const double* __restrict__ thr2,
                                                  int solve_all, const double* __restrict__ fw,
                                                  double* __restrict__ wn2,
                                                  int* __restrict__ flag, void* __restrict__ Vh,
                                                  int vh_single, int nz) {
  long fm = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (fm >= (long)F * N) return;
  int f = (int)(fm / N);
  long m = fm - (long)f * N;
  const cx<T>* w = What + (long)f * nd * N + m;
  // eight loads in flight, four partial sums
  double s4[4] = {0.0, 0.0, 0.0, 0.0};
  int j = 0;
  for (; j + 8 <= nd; j += 8) {
    cx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = w[(long)(j + u) * N];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      s4[u & 3] = fma((double)v[u].x, (double)v[u].x, fma((double)v[u].y, (double)v[u].y, s4[u & 3]));
  }
  for (; j < nd; ++j) {
    const cx<T> v = w[(long)j * N];
    s4[0] = fma((double)v.x, (double)v.x, fma((double)v.y, (double)v.y, s4[0]));
  }
  const double s = (s4[0] + s4[1]) + (s4[2] + s4[3]);
  wn2[fm] = s;
  // thr2[f] < 0 marks noise-free data, solve_all the rule with one alpha per
  // frequency: then every nonzero system is solved
  double t = thr2[f];
  // a frequency of weight 0 in the least-squares xi is not solved
  const int act = (fw && fw[f] == 0.0) ? 0 : (solve_all || t < 0.0) ? (s > 0.0) : (s > t);
  const int was = flag[fm];
  flag[fm] = act;
  if (!act && was) {
    const long o0 = (long)f * nz * N + m;
    if (vh_single)
      for (int j = 0; j < nz; ++j) ((cx<float>*)Vh)[o0 + (long)j * N] = mk(0.f, 0.f);
    else
      for (int j = 0; j < nz; ++j) ((cx<double>*)Vh)[o0 + (long)j * N] = mk(0.0, 0.0);
  }
}

// Inclusive scan of small ints over a 1024-thread block (wave shuffles, then
// the wave totals in wsum); returns the thread's inclusive sum, and wsum[15]
// holds the block's sum afterwards.
__device__ __forceinline__ int block_incl_sum_scan(int v, int* wsum) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d);
    if (lane >= d) v += u;
  }
  if (lane == 63) wsum[wv] = v;
  __syncthreads();
  if (wv == 0) {
    int w = lane < 16 ? wsum[lane] : 0;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      const int u = __shfl_up(w, d);
      if (lane >= d) w += u;
    }
    if (lane < 16) wsum[lane] = w;
  }
  __syncthreads();
  return v + (wv > 0 ? wsum[wv - 1] : 0);
}

// Wavenumbers related by the torus's mirror (and, on a square torus, swap)
// symmetries share A_m. Per block of 1024 (f, m): for a representative m
// (orep[m] = m), ocw[f N + m] counts the members of its orbit (omem[m][0..7],
// -1 padded) that need a solve, every other m gets 0; and the block's
// active orbits (cnt) and their active members (cntw).
__global__ __launch_bounds__(1024) void k_orbit_block_count(const int* __restrict__ flag,
                                                            const int* __restrict__ orep,
                                                            const int* __restrict__ omem, long N,
                                                            int* __restrict__ ocw, long n,
                                                            int* __restrict__ cnt,
                                                            int* __restrict__ cntw) {
  __shared__ int wsum[16];
  __shared__ int wcnt[16];
  const long i = (long)blockIdx.x * 1024 + threadIdx.x;
  int c = 0;
  if (i < n) {
    const int f = (int)(i / N);
    const long m = i - (long)f * N;
    if (orep[m] == m) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int mj = omem[m * 8 + j];
        if (mj >= 0) c += flag[(long)f * N + mj];
      }
    }
    ocw[i] = c;
  }
  const unsigned long long bal = __ballot(c > 0);
  if ((threadIdx.x & 63) == 0) wcnt[threadIdx.x >> 6] = __popcll(bal);
  block_incl_sum_scan(c, wsum);
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < 16; ++w) acc += wcnt[w];
    cnt[blockIdx.x] = acc;
    cntw[blockIdx.x] = wsum[15];
  }
}

// Compaction of the active orbits in increasing f N + m (olist, oslot; NULL
// keeps them, for factorizations made at plan creation) and of the active
// systems grouped by orbit (members in omem order) into list, from the
// exclusive block offsets cnt / cntw (k_scan of the block counts). osys0
// (with olist): the members of compacted orbit o are list[osys0[o] ..
// osys0[o + 1]), so that a range of orbits maps to a range of systems.
__global__ __launch_bounds__(1024) void k_orbit_scatter(const int* __restrict__ ocw, long n,
                                                        const int* __restrict__ omem,
                                                        const int* __restrict__ flag, long N,
                                                        const int* __restrict__ cnt,
                                                        const int* __restrict__ cntw,
                                                        int* __restrict__ olist,
                                                        int* __restrict__ oslot,
                                                        int* __restrict__ list,
                                                        int* __restrict__ osys0,
                                                        int* __restrict__ opos) {
  __shared__ int wsum[16];
  __shared__ int wpre[16];
  const long i = (long)blockIdx.x * 1024 + threadIdx.x;
  const int c = i < n ? ocw[i] : 0;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned long long bal = __ballot(c > 0);
  if (lane == 0) wpre[wv] = __popcll(bal);
  const int incl = block_incl_sum_scan(c, wsum);
  if (threadIdx.x == 0) {
    int acc = 0;
    for (int w = 0; w < 16; ++w) {
      const int t = wpre[w];
      wpre[w] = acc;
      acc += t;
    }
  }
  __syncthreads();
  // no active orbit at all still leaves an empty first range
  if (osys0 && blockIdx.x == 0 && threadIdx.x == 0) osys0[0] = 0;
  // first system of every position (orbits fixed at plan creation)
  if (opos && i < n) {
    const int pos0 = cntw[blockIdx.x] + incl - c;
    opos[i] = pos0;
    if (i == n - 1) opos[n] = pos0 + c;
  }
  if (c > 0) {
    const int pos0 = cntw[blockIdx.x] + incl - c;
    if (olist) {
      const int o = cnt[blockIdx.x] + wpre[wv] + __popcll(bal & ((1ull << lane) - 1ull));
      olist[o] = (int)i;
      oslot[i] = o;
      // orbit o's start and end (the next orbit writes the same end value
      // as its start)
      if (osys0) {
        osys0[o] = pos0;
        osys0[o + 1] = pos0 + c;
      }
    }
    const int f = (int)(i / N);
    const long m = i - (long)f * N;
    int pos = pos0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int mj = omem[m * 8 + j];
      if (mj >= 0 && flag[(long)f * N + mj]) list[pos++] = (int)((long)f * N + mj);
    }
  }
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

// block b: exclusive scan of the nb block counts cnt_b in place, the total to
// *count_b (block 0: cnt, count; block 1, if launched: cnt2, count2)
__global__ __launch_bounds__(1024) void k_scan(int* __restrict__ cnt0, int nb, int* __restrict__ count0,
                                               int* __restrict__ cnt2, int* __restrict__ count2) {
  __shared__ int wsum[16];
  __shared__ int total;
  int* cnt = blockIdx.x == 0 ? cnt0 : cnt2;
  int* count = blockIdx.x == 0 ? count0 : count2;
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
  z64* dg;      // [C][n] diagonal of B (complex)
  z64* sp;      // [C][n] superdiagonal of B (complex; entry n-1 unused)
  z64* q;       // [C][n] U^H w
  double* fro;  // [C] ||A||_F^2
  double* wn2;  // [C] ||w||^2
  z64* refl;    // [C][tri_size(n, 1)] right reflector k: entries k+1..n-1, packed
  double* gam;  // [C][n]
  z64* refl_l;  // [C][tri_size(n, 0)] left reflector k: entries k..n-1, packed; NULL: not kept
  double* gam_l;
};

constexpr int pow2ceil(int v) { return v <= 1 ? 1 : 2 * pow2ceil((v + 1) / 2); }

// Householder scalars of a vector x with s = |x|^2 and pivot entry x_k = piv:
// beta = -(x_k / |x_k|) |x|, the entry that replaces x_k, and
// g = 1 / (|x| (|x| + |x_k|)), so that I - g u u^H with u = x - beta e_k maps
// x to beta e_k. One reciprocal square root of P = s |x_k|^2 gives both
// |x| / |x_k| = s / sqrt(P) and |x| |x_k| = P / sqrt(P). A zero (or
// negligible: P below the normal range) pivot takes phase 1; s = 0 gives
// beta = 0 and g = 0 (no reflection).
__device__ __forceinline__ void hh_scalars(double s, z64 piv, z64& beta, double& g) {
  const double P = s * nrm2(piv);
  const bool phased = P > 1e-290;
  const double Pv = phased ? P : s;
  const double rp = Pv > 0.0 ? rsq_nr(Pv) : 0.0;
  const double xa = s * rp;  // |x| / |x_k|, or |x| when the pivot has no phase
  beta = phased ? mk(-piv.x * xa, -piv.y * xa) : mk(-xa, 0.0);
  const double den = phased ? s + P * rp : s;
  g = den > 0.0 ? rcp_nr(den) : 0.0;
}

// Pairwise sum of v[B..E) (E > B): a tree of depth log2(E - B) instead of a
// chain of E - B - 1 dependent additions.
template <int B, int E, int N>
__device__ __forceinline__ double range_sum(const double (&v)[N]) {
  if constexpr (E - B == 1) {
    return v[B];
  } else {
    constexpr int M = (B + E) / 2;
    return range_sum<B, M>(v) + range_sum<M, E>(v);
  }
}

// threads per row for summing the wave partials of z: the largest power of
// two P <= min(NW, 8) with n P <= NT
constexpr int bd_rows_threads(int n, int NT, int NW, int P = 8) {
  return (P <= NW && n * P <= NT) || P == 1 ? P : bd_rows_threads(n, NT, NW, P / 2);
}

// Sums of the VP complex values v over each aligned group of TR lanes (TR =
// 16, 32 or 64; VP a power of two): reduce-scatter over the group's lane bits
// 5..2 while a lane carries more than one value (each sum is formed once), a
// full butterfly over the remaining bits, then every lane of the group reads
// the VP totals from the group's VP slots gat of LDS. A wave's LDS accesses
// complete in order, so the exchange needs no barrier.
template <int TR, int VP>
__device__ __forceinline__ void group_sums(z64 (&v)[VP], z64* gat, int lane) {
  double d[2 * VP];
#pragma unroll
  for (int i = 0; i < VP; ++i) {
    d[2 * i] = v[i].x;
    d[2 * i + 1] = v[i].y;
  }
  int idx = 0;  // first of the values this lane carries
  // bit 5 (i ^ 32)
  constexpr int C5 = (TR == 64 && VP >= 2) ? VP / 2 : VP;
  if constexpr (TR == 64) {
    if constexpr (VP >= 2) {
#pragma unroll
      for (int i = 0; i < 2 * C5; ++i) d[i] = rs_xor32(d[i], d[i + 2 * C5]);
      if (lane & 32) idx += C5;
    } else {
#pragma unroll
      for (int i = 0; i < 2 * C5; ++i) d[i] = add_xor32(d[i]);
    }
  }
  // bit 4 (i ^ 16)
  constexpr int C4 = (TR >= 32 && C5 >= 2) ? C5 / 2 : C5;
  if constexpr (TR >= 32) {
    if constexpr (C5 >= 2) {
#pragma unroll
      for (int i = 0; i < 2 * C4; ++i) d[i] = rs_xor16(d[i], d[i + 2 * C4]);
      if (lane & 16) idx += C4;
    } else {
#pragma unroll
      for (int i = 0; i < 2 * C4; ++i) d[i] = add_xor16(d[i]);
    }
  }
  // bit 3 (row_mirror, i <-> 15 - i)
  constexpr int C3 = C4 >= 2 ? C4 / 2 : C4;
  if constexpr (C4 >= 2) {
#pragma unroll
    for (int i = 0; i < 2 * C3; ++i) d[i] = rs_dpp<0x140, 0x3>(d[i], d[i + 2 * C3]);
    if (lane & 8) idx += C3;
  } else {
#pragma unroll
    for (int i = 0; i < 2 * C3; ++i) d[i] += dpp_d<0x140>(d[i]);
  }
  // bit 2 (row_half_mirror, i <-> 7 - i within eight)
  constexpr int C2 = C3 >= 2 ? C3 / 2 : C3;
  if constexpr (C3 >= 2) {
#pragma unroll
    for (int i = 0; i < 2 * C2; ++i) d[i] = rs_dpp<0x141, 0x5>(d[i], d[i + 2 * C2]);
    if (lane & 4) idx += C2;
  } else {
#pragma unroll
    for (int i = 0; i < 2 * C2; ++i) d[i] += dpp_d<0x141>(d[i]);
  }
  // bits 1 and 0 (quad_perm [2,3,0,1], [1,0,3,2])
#pragma unroll
  for (int i = 0; i < 2 * C2; ++i) {
    d[i] += dpp_d<0x4E>(d[i]);
    d[i] += dpp_d<0xB1>(d[i]);
  }
#pragma unroll
  for (int i = 0; i < C2; ++i) gat[idx + i] = mk(d[2 * i], d[2 * i + 1]);
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
#pragma unroll
  for (int i = 0; i < VP; ++i) v[i] = gat[i];
}

// Exchange areas of one bidiagonalization workgroup (index = step parity).
template <int n, int NW>
struct BdShared {
  z64 tb[2 * n];
  z64 ul[2][n];       // left reflector u (entries k..n-1)
  z64 xr[2][n];       // row k after the left update (entries k+1..n-1)
  z64 zp[2][NW][n];   // per-wave partial z = A v
  z64 zs[n];          // g z, summed over the waves (when they are many)
  double lg[2];       // left gamma
  z64 dg[n], sp[n];
  z64 qv[n];          // q = U^H w (row i kept by the column-class-0 thread of row class i % TR)
  double gm[n];
  double gl[n];       // left gamma of every step
  double red[2][NW];
  alignas(16) double rn[2][NW];  // per wave: its part of |row k beyond the diagonal|^2
  z64 cg[NW][64];     // per wave: the column sums of its lane groups
};

// One Householder step k (left reflector from column k, right reflector
// from row k). Row slots a < SA and column slots b < SB hold only finished
// rows / columns for every k of the current block and are skipped at compile
// time; in the partially finished slots the finished rows and columns are
// masked per element (by selects, so that the step is straight-line code).
template <int TR, int TC, int NA, int NB, int SA, int SB>
__device__ __forceinline__ void bd_step(z64 (&A)[NA][NB], BdShared<TR * NA, (TR * TC + 63) / 64>& S,
                                        int k, int r, int c, int tid, int lane, int wv, bool doq) {
  constexpr int n = TR * NA;
  constexpr int NW = (TR * TC + 63) / 64;
  const int par = k & 1;
  const int ka = k / TR, kr = k % TR;  // row k: row class kr, slot ka
  const int kb = k / TC, kc = k % TC;  // column k: column class kc, slot kb
  // ---------- A. left reflector from column k (holders: column class kc)
  if (n - k >= 2) {
    if (c == kc) {
      z64 col[NA];
#pragma unroll
      for (int a = SA; a < NA; ++a) {
        col[a] = mk(0.0, 0.0);
#pragma unroll
        for (int b = SB; b < NB; ++b)
          if (b == kb) col[a] = A[a][b];
      }
      double sq[NA];
      z64 pc = mk(0.0, 0.0);
#pragma unroll
      for (int a = SA; a < NA; ++a) {
        const int i = r + TR * a;
        sq[a] = (i >= k) ? nrm2(col[a]) : 0.0;
        if (a == ka) pc = col[a];
      }
      const double s = lanes_sum<TR>(range_sum<SA, NA>(sq));
      // the pivot A(k, k) from its holder's lane of this wave
      const z64 piv = lane_read(pc, (kr + TR * kc) & 63);
      z64 beta;
      double gl;
      hh_scalars(s, piv, beta, gl);
      // rows above k are written too (B masks them), so the stores need no
      // branch
#pragma unroll
      for (int a = SA; a < NA; ++a) {
        const int i = r + TR * a;
        S.ul[par][i] = (i == k) ? (col[a] - beta) : col[a];
      }
      if (r == kr) {
        S.lg[par] = gl;
        S.gl[k] = gl;
        S.dg[k] = beta;
      }
    }
  } else if (c == kc && r == kr) {
#pragma unroll
    for (int a = SA; a < NA; ++a)
#pragma unroll
      for (int b = SB; b < NB; ++b)
        if (a == ka && b == kb) S.dg[k] = A[a][b];
  }
  __syncthreads();
  // ---------- B. A <- (I - g u u^H) A on columns > k, and q likewise
  if (n - k >= 2) {
    const double g = S.lg[par];
    z64 ur[NA];
#pragma unroll
    for (int a = SA; a < NA; ++a) {
      // loads without a branch (every index is in range), so that they can
      // be issued early; the rows above k are masked afterwards
      const int i = r + TR * a;
      const z64 u = S.ul[par][i];
      ur[a] = (i >= k) ? u : mk(0.0, 0.0);
    }
    // u^H A for the live column slots, summed over the row classes of each
    // column class at once
    constexpr int V = NB - SB, VP = pow2ceil(V);
    z64 sm[VP];
#pragma unroll
    for (int b = 0; b < VP; ++b) {
      z64 t = mk(0.0, 0.0);
      if (b < V) {
#pragma unroll
        for (int a = SA; a < NA; ++a) t = cfmac(t, ur[a], A[a][SB + b]);
      }
      sm[b] = t;
    }
    group_sums<TR, VP>(sm, &S.cg[wv][(lane / TR) * VP], lane);
#pragma unroll
    for (int b = SB; b < NB; ++b) {
      // columns up to k take w = 0, which leaves them unchanged
      const int j = c + TC * b;
      const z64 w = (j > k) ? g * sm[b - SB] : mk(0.0, 0.0);
#pragma unroll
      for (int a = SA; a < NA; ++a) A[a][b] = cfms(A[a][b], ur[a], w);
    }
    if (doq && c == 0) {
      z64 qa[NA];
#pragma unroll
      for (int a = SA; a < NA; ++a) qa[a] = S.qv[r + TR * a];
      z64 sm = mk(0.0, 0.0);
#pragma unroll
      for (int a = SA; a < NA; ++a) sm = cfmac(sm, ur[a], qa[a]);
      sm.x = lanes_sum<TR>(sm.x);
      sm.y = lanes_sum<TR>(sm.y);
      sm = g * sm;
#pragma unroll
      for (int a = SA; a < NA; ++a) S.qv[r + TR * a] = cfms(qa[a], ur[a], sm);
    }
  }
  const int rk = n - k - 1;
  if (rk >= 2) {
    // row k beyond the diagonal: its holders publish it, and each wave
    // publishes the part of its squared norm that the wave holds
    // (entries up to column k are written too: C masks them)
    double rs = 0.0;
#pragma unroll
    for (int a = SA; a < NA; ++a) {
      if (a == ka) {
#pragma unroll
        for (int b = SB; b < NB; ++b) {
          const int j = c + TC * b;
          rs += (j > k) ? nrm2(A[a][b]) : 0.0;
          if (r == kr) S.xr[par][j] = A[a][b];
        }
      }
    }
    rs = strided_sum<TR>(rs);
    if (lane == kr) S.rn[par][wv] = rs;
    __syncthreads();
    // ---------- C. right reflector from row k (every wave computes it, from
    // the same partial norms in the same order)
    double rn[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) rn[w] = S.rn[par][w];
    const double s = range_sum<0, NW>(rn);
    z64 beta;
    double g;
    hh_scalars(s, cj(S.xr[par][k + 1]), beta, g);
    z64 vr[NB];
#pragma unroll
    for (int b = SB; b < NB; ++b) {
      const int j = c + TC * b;
      const z64 x = cj(S.xr[par][j]);
      vr[b] = (j > k) ? ((j == k + 1) ? x - beta : x) : mk(0.0, 0.0);
    }
    if (tid == 0) {
      S.gm[k] = g;
      S.sp[k] = cj(beta);
    }
    // z = A v on the live row slots; the column classes of this wave are
    // summed with each row sum formed once, and a lane writes the rows it
    // ends with
    {
      constexpr int V = NA - SA, VP = pow2ceil(V);
      z64 t[VP];
#pragma unroll
      for (int a = 0; a < VP; ++a) {
        z64 x = mk(0.0, 0.0);
        if (a < V) {
#pragma unroll
          for (int b = SB; b < NB; ++b) x = cfma(x, A[SA + a][b], vr[b]);
        }
        t[a] = x;
      }
      // reduce-scatter over the 2 VP doubles (real and imaginary parts as
      // separate values), so that at small VP the last levels still halve
      // the values a lane carries instead of summing both parts in full
      constexpr bool L5 = TR <= 32, L4 = TR <= 16;
      constexpr int D0 = 2 * VP;
      constexpr int D1 = L5 ? D0 / 2 : D0;
      constexpr int D2 = (L4 && D1 >= 2) ? D1 / 2 : D1;
      double d[D0];
#pragma unroll
      for (int i = 0; i < VP; ++i) {
        d[2 * i] = t[i].x;
        d[2 * i + 1] = t[i].y;
      }
      int idx = 0;  // first of the doubles this lane ends with
      if constexpr (L5) {
#pragma unroll
        for (int j = 0; j < D1; ++j) d[j] = rs_xor32(d[j], d[j + D1]);
        if (lane & 32) idx += D1;
      }
      if constexpr (L4) {
        if constexpr (D1 >= 2) {
#pragma unroll
          for (int j = 0; j < D2; ++j) d[j] = rs_xor16(d[j], d[j + D2]);
          if (lane & 16) idx += D2;
        } else {
          d[0] = add_xor16(d[0]);
        }
      }
      if constexpr (D2 >= 2) {
#pragma unroll
        for (int e = 0; e < D2 / 2; ++e) {
          const int ci = idx / 2 + e;
          if (ci < V) S.zp[par][wv][r + TR * (SA + ci)] = mk(d[2 * e], d[2 * e + 1]);
        }
      } else {
        const int ci = idx / 2;
        if (ci < V) reinterpret_cast<double*>(&S.zp[par][wv][r + TR * (SA + ci)])[idx & 1] = d[0];
      }
    }
    __syncthreads();
    // With eight or more waves the wave partials of z are summed once per
    // row, by P consecutive threads (NW / P partials each, then a butterfly
    // over the P lanes), instead of by every holder of the row.
    constexpr bool COOP = NW >= 8;
    if constexpr (COOP) {
      constexpr int P = bd_rows_threads(n, TR * TC, NW), WP = NW / P;
      if (tid < n * P) {
        const int i = tid / P, part = tid % P;
        z64 z = S.zp[par][part * WP][i];
#pragma unroll
        for (int w = 1; w < WP; ++w) z = z + S.zp[par][part * WP + w][i];
        if constexpr (P >= 2) z = mk(z.x + dpp_d<0xB1>(z.x), z.y + dpp_d<0xB1>(z.y));
        if constexpr (P >= 4) z = mk(z.x + dpp_d<0x4E>(z.x), z.y + dpp_d<0x4E>(z.y));
        if constexpr (P >= 8) z = mk(z.x + dpp_d<0x141>(z.x), z.y + dpp_d<0x141>(z.y));
        if (part == 0) S.zs[i] = g * z;
      }
      __syncthreads();
    }
    // ---------- D. A <- A (I - g v v^H) on rows > k, columns > k
#pragma unroll
    for (int a = SA; a < NA; ++a) {
      // rows up to k take z = 0, which leaves them unchanged
      const int i = r + TR * a;
      z64 z;
      if constexpr (COOP) {
        z = S.zs[i];
      } else {
        z = S.zp[par][0][i];
#pragma unroll
        for (int w = 1; w < NW; ++w) z = z + S.zp[par][w][i];
        z = g * z;
      }
      z = (i > k) ? z : mk(0.0, 0.0);
#pragma unroll
      for (int b = SB; b < NB; ++b) A[a][b] = cfmsc(A[a][b], z, vr[b]);
    }
    // row k is finished: keep the right reflector in its place (LAPACK
    // style); entries j <= k keep the left reflectors of columns j
#pragma unroll
    for (int a = SA; a < NA; ++a) {
      if (r + TR * a == k) {
#pragma unroll
        for (int b = SB; b < NB; ++b)
          if (c + TC * b > k) A[a][b] = vr[b];
      }
    }
  } else {
    if (rk == 1) {
      const int jb = (k + 1) / TC, jc = (k + 1) % TC;
      if (r == kr && c == jc) {
#pragma unroll
        for (int a = SA; a < NA; ++a)
#pragma unroll
          for (int b = SB; b < NB; ++b)
            if (a == ka && b == jb) S.sp[k] = A[a][b];
      }
    }
    if (tid == 0) S.gm[k] = 0.0;
  }
}

// Steps of k-block Q (KB = max(TR, TC) consecutive k), then the next block.
template <int TR, int TC, int NA, int NB, int Q>
__device__ __forceinline__ void bd_blocks(z64 (&A)[NA][NB],
                                          BdShared<TR * NA, (TR * TC + 63) / 64>& S, int r, int c,
                                          int tid, int lane, int wv, bool doq) {
  constexpr int n = TR * NA;
  constexpr int KB = TR < TC ? TR : TC;
  if constexpr (Q * KB < n) {
    constexpr int SA = Q * KB / TR, SB = Q * KB / TC;
    for (int k = Q * KB; k < (Q + 1) * KB && k < n; ++k)
      bd_step<TR, TC, NA, NB, SA, SB>(A, S, k, r, c, tid, lane, wv, doq);
    bd_blocks<TR, TC, NA, NB, Q + 1>(A, S, r, c, tid, lane, wv, doq);
  }
}

// WPE: minimum waves per SIMD requested from the register allocator
template <int TR, int TC, int NA, int NB, typename TW, int WPE>
__global__ __launch_bounds__(TR* TC, WPE) void k_bidiag(const z64* __restrict__ gsys, int tpitch,
                                                   const cx<TW>* __restrict__ What, long N,
                                                   const int* __restrict__ list,
                                                   const int* __restrict__ count, int chunk0, int C,
                                                   BidiagOut o, const int* __restrict__ resident,
                                                   int nd, int nzv, int gen) {
  constexpr int n = TR * NA;
  static_assert(TR * NA == TC * NB, "square system");
  static_assert(TR == 16 || TR == 32 || TR == 64, "row classes form aligned lane groups");
  constexpr int NT = TR * TC;
  constexpr int NW = (NT + 63) / 64;
  __shared__ BdShared<n, NW> S;

  const int tid = threadIdx.x;
  const int r = tid % TR, c = tid / TR;
  const int lane = tid & 63, wv = tid >> 6;
  const int total = *count;
  const bool doq = o.refl_l == nullptr;
  // the workspace already holds this chunk's factorizations (the forward
  // solve made them from the same tables)
  if (resident && *resident == chunk0) return;

  // one factorization per workgroup: with no loop over slots the compiler
  // keeps the per-element index and address arithmetic of the epilogue out
  // of the step loops (hoisted out of a slot loop it spilled to scratch)
  {
    const int sl = blockIdx.x;
    const int gs = chunk0 + sl;
    if (sl >= C || gs >= total) return;
    const int fm = list[gs];
    const long m = fm % N;
    const int f = (int)(fm / N);
    const z64* trow = gsys + ((long)f * N + m) * tpitch;
    if (!gen)
      for (int t = tid; t < 2 * n - 1; t += NT) S.tb[t] = trow[t];
    __syncthreads();

    // A from the Toeplitz row (planes on X's lattice, nd = nz = n), or, for a
    // general plane set, entry (i, j) of the nd x nzv table row, zero padded
    // to n x n (zero rows and columns leave the regularized solution of the
    // unpadded system unchanged)
    z64 A[NA][NB];
    double fr = 0.0;
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = r + TR * a, j = c + TC * b;
        if (gen)
          A[a][b] = (i < nd && j < nzv) ? trow[(long)i * nzv + j] : mk(0.0, 0.0);
        else
          A[a][b] = S.tb[i - j + n - 1];
        fr += nrm2(A[a][b]);
      }
    // q = U^H w (starts as w), rows r + TR a kept by the column-class-0
    // threads; not formed when the left reflectors are kept instead
    double wq = 0.0;
    if (doq && c == 0) {
#pragma unroll
      for (int a = 0; a < NA; ++a) {
        const int row = r + TR * a;
        const z64 w = row < nd ? cast<double>(What[((long)f * nd + row) * N + m]) : mk(0.0, 0.0);
        S.qv[r + TR * a] = w;
        wq += nrm2(w);
      }
    }
    fr = lanes_sum<64>(fr);
    wq = lanes_sum<64>(wq);
    if (lane == 0) {
      S.red[0][wv] = fr;
      S.red[1][wv] = wq;
    }
    __syncthreads();
    if (tid == 0) {
      double s0 = 0.0, s1 = 0.0;
      for (int w = 0; w < NW; ++w) {
        s0 += S.red[0][w];
        s1 += S.red[1][w];
      }
      o.fro[sl] = s0;
      o.wn2[sl] = s1;
    }

    bd_blocks<TR, TC, NA, NB, 0>(A, S, r, c, tid, lane, wv, doq);

    __syncthreads();
    z64* refl = o.refl + (long)sl * tri_size(n, 1);
    double* gam = o.gam + (long)sl * n;
    // right reflector k: row k, columns k+1..n-1
#pragma unroll
    for (int a = 0; a < NA; ++a)
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const int i = r + TR * a, j = c + TC * b;
        if (j > i && i + 2 < n) refl[tri_start(i, n, 1) + (j - i - 1)] = A[a][b];
      }
    for (int t = tid; t < n; t += NT) {
      gam[t] = S.gm[t];
      o.dg[(long)sl * n + t] = S.dg[t];
      o.sp[(long)sl * n + t] = (t < n - 1) ? S.sp[t] : mk(0.0, 0.0);
    }
    if (doq && c == 0) {
#pragma unroll
      for (int a = 0; a < NA; ++a) o.q[(long)sl * n + r + TR * a] = S.qv[r + TR * a];
    }
    if (o.refl_l) {
      // left reflector j: column j from the diagonal down (the pivot minus
      // beta on the diagonal), as it was when step j formed it
      z64* rl = o.refl_l + (long)sl * tri_size(n, 0);
#pragma unroll
      for (int a = 0; a < NA; ++a)
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const int i = r + TR * a, j = c + TC * b;
          if (i >= j && j + 1 < n)
            rl[tri_start(j, n, 0) + (i - j)] = (i == j) ? A[a][b] - S.dg[j] : A[a][b];
        }
      for (int t = tid; t < n; t += NT) o.gam_l[(long)sl * n + t] = (t + 1 < n) ? S.gl[t] : 0.0;
    }
    __syncthreads();
  }
}

// Orbits fixed at plan creation (slot s = orbit olist[s], in position
// order): the systems of slot s are [osys0[s], osys0[s + 1]).
__global__ void k_slot_ranges(const int* __restrict__ olist, int FO, const int* __restrict__ opos,
                              int* __restrict__ osys0) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= FO) return;
  osys0[s] = opos[olist[s]];
  if (s == FO - 1) osys0[FO] = opos[olist[s] + 1];
}

// After the factorization of orbit chunk [chunk0, chunk0 + C): the
// workspace holds it if the chunk had an active orbit (a chunk past the
// last active orbit factorizes nothing and leaves the previous one).
// chunk0 < 0 clears the mark.
__global__ void k_mark_resident(int* __restrict__ resident, const int* __restrict__ ocount,
                                int chunk0) {
  if (chunk0 < 0)
    *resident = -1;
  else if (chunk0 < *ocount)
    *resident = chunk0;
}

// ---------------------------------------------------------------- dp

struct DpArgs {
  const z64* dg;       // [C][n] bidiagonal of A (complex)
  const z64* sp;
  const z64* q;        // [C][n] U^H w
  const double* fro;   // [C]
  const int* list;
  const int* count;
  int chunk0, C, n;
  int nd, nzv;         // data planes (rows of W^) and X planes (of V^); n for
                       // square Toeplitz systems, else n >= both (zero padding)
  long N;
  const double* thr2;  // per frequency: (tau delta_m)^2, < 0 for noise-free data
  double eta;
  const z64* refl;     // [C][tri_size(n, 1)] right reflectors
  const double* gam;   // [C][n]
  void* Vh;            // [F][n][N] output, plane-major (complex64 or complex128)
  int vh_single;       // 1: Vh holds complex64
  double* alpha;       // [F*N]
  signed char* branch; // [F*N]
  double* bd_d;        // [C][n] real bidiagonal and right phases, kept for
  double* bd_e;        //        the derivative kernels
  z64* bd_dr;
  const double* alpha_fixed;       // per frequency, or NULL: alpha given (one per
  const signed char* branch_fixed; // frequency) instead of the per-system search
  // shared factorizations (k_dpo_*): system (f, m) uses slot
  // oslot[f N + orep[m]] of dg, sp, fro, refl, gam, and q = U^H w from the
  // slot's left reflectors and w in What
  const int* oslot;
  const int* orep;
  const z64* What;
  const z64* refl_l;
  const double* gam_l;
  // orbit chunks (NULL: every active orbit has a slot): this launch solves
  // the systems of compacted orbits [slot0, slot0 + OC), whose
  // factorizations sit in slots oslot - slot0 of the workspace
  const int* osys0;
  const int* ocount;
  int slot0, OC;
  // orbit-batched solve (k_dpo_*): per system of the launch, q' and then
  // D_R y; bd_d, bd_e, bd_dr then hold each slot's B' and right phases
  z64* qy;
};

// The compacted systems [*first, *first + return value) that one solver
// launch takes: the chunk [chunk0, chunk0 + C) of a list of total systems,
// or, with orbit chunks, the members of compacted orbits
// [slot0, slot0 + OC).
__device__ __forceinline__ int launch_range(const int* osys0, const int* ocount, int slot0, int OC,
                                            int chunk0, int C, int total, int* first) {
  if (osys0) {
    const int oc = *ocount;
    const int b = osys0[min(slot0, oc)];
    *first = b;
    return osys0[min(slot0 + OC, oc)] - b;
  }
  *first = chunk0;
  return min(C, total - chunk0);
}

// phi(alpha) = ||B y - q||^2 of the Tikhonov solution for the real upper
// bidiagonal B (d, e; e[n-1] = 0), evaluated in one forward pass without storage:
// phi = -alpha^2 g'(alpha) with g = q^H (B B^T + alpha I)^{-1} q, g from the
// LDL^T recurrence of the tridiagonal B B^T + alpha I and g' by forward-mode
// differentiation of the same recurrence.
__device__ __forceinline__ double phi_fwd(const double* __restrict__ d, const double* __restrict__ e,
                                          const z64* __restrict__ q, int n, double alpha) {
  double D = d[0] * d[0] + e[0] * e[0] + alpha;
  double Dp = 1.0;
  z64 z = q[0], zp = mk(0.0, 0.0);
  double rD = rcp_nr(D);
  double gp = -nrm2(z) * Dp * rD * rD;
  for (int i = 1; i < n; ++i) {
    const double b = e[i - 1] * d[i];
    const double l = b * rD;
    const double ei = e[i];
    const double Dn = d[i] * d[i] + ei * ei + alpha - l * b;
    const double Dpn = 1.0 + l * l * Dp;
    const double c1 = l * Dp * rD;
    const z64 zn = q[i] - l * z;
    const z64 zpn = c1 * z - l * zp;
    D = Dn;
    Dp = Dpn;
    z = zn;
    zp = zpn;
    rD = rcp_nr(D);
    gp += 2.0 * (z.x * zp.x + z.y * zp.y) * rD - nrm2(z) * Dp * rD * rD;
  }
  return -alpha * alpha * gp;
}

// Elden: Givens QR of [B; sqrt(alpha) I], back substitution; writes y.
// rho and off may alias d and e (entry i is read before it is written).
__device__ void elden_solve(const double* d, const double* e, const z64* q, int n, double alpha,
                            double* rho, double* off, z64* rr, z64* y) {
  const double mu = sqrt(alpha);
  double mt = mu;
  z64 g = mk(0.0, 0.0);
  for (int i = 0; i < n; ++i) {
    const double di = d[i];
    const z64 qi = q[i];
    const double p2s = di * di + mt * mt;
    const double ip = p2s > 0.0 ? rsq_nr(p2s) : 0.0;
    const double p = p2s * ip;
    const double cs = p2s > 0.0 ? di * ip : 1.0;
    const double sn = mt * ip;
    rho[i] = p;
    rr[i] = cs * qi + sn * g;
    const z64 gp = (-sn) * qi + cs * g;
    if (i < n - 1) {
      const double ei = e[i];
      off[i] = cs * ei;
      const double fz = -sn * ei;
      const double q2 = mu * mu + fz * fz;
      const double iq = q2 > 0.0 ? rsq_nr(q2) : 0.0;
      mt = q2 * iq;
      g = (fz * iq) * gp;
    }
  }
  z64 yn = mk(0.0, 0.0);
  for (int i = n - 1; i >= 0; --i) {
    z64 t = rr[i];
    if (i < n - 1) t = t - off[i] * yn;
    const double p = rho[i];
    const double ip = p > 0.0 ? rcp_nr(p) : 0.0;
    const z64 yi = mk(t.x * ip, t.y * ip);
    y[i] = yi;
    yn = yi;
  }
}

// Phase scaling of one system's complex bidiagonal (sy: diagonal, srr:
// superdiagonal, sq: q in LDS) to B = D_L B' D_R^H with B' real and
// nonnegative: writes sd, se (B'), sdr (right phases) and q' = D_L^H q into sq
// (sq may be NULL), and the left phases D_L into sdl when it is given.
// One wave; the caller synchronizes afterwards.
template <int NMAX>
__device__ __forceinline__ void dp_phase_scale(int n, int lane, double* sd, double* se, z64* sq,
                                               const z64* srr, const z64* sy, z64* sdr,
                                               z64* sdl = nullptr) {
  // B = D_L B' D_R^H with B' real nonnegative. The right phases obey
  // r_i = rho_i r_{i-1} (or restart at a zero entry), an affine recurrence
  // evaluated by a parallel prefix over the lanes (elements lane, lane + 64).
  {
    constexpr int H = (NMAX + 63) / 64;  // elements per lane
    z64 ra[2], rb[2], pd[2];
    bool dz[2];
    ra[1] = mk(1.0, 0.0);
    rb[1] = mk(0.0, 0.0);
    pd[1] = mk(1.0, 0.0);
    dz[1] = true;
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int i = lane + 64 * h;
      z64 am = mk(1.0, 0.0), bm = mk(0.0, 0.0), ph = mk(1.0, 0.0);
      dz[h] = true;
      if (i < n) {
        const z64 dgi = sy[i];
        const double d2 = nrm2(dgi);
        const double idd = d2 > 0.0 ? rsq_nr(d2) : 0.0;
        sd[i] = d2 * idd;
        dz[h] = !(d2 > 0.0);
        if (d2 > 0.0) ph = mk(dgi.x * idd, dgi.y * idd);
        z64 cs = mk(1.0, 0.0);  // conj(phase(sp_i))
        double ei = 0.0;
        if (i < n - 1) {
          const z64 spi = srr[i];
          const double s2 = nrm2(spi);
          const double is = s2 > 0.0 ? rsq_nr(s2) : 0.0;
          ei = s2 * is;
          if (s2 > 0.0) cs = mk(spi.x * is, -spi.y * is);
          if (!(s2 > 0.0)) {
            am = mk(0.0, 0.0);
            bm = mk(1.0, 0.0);
          } else if (!(d2 > 0.0)) {
            am = mk(0.0, 0.0);
            bm = cs;
          } else {
            am = ph * cs;
          }
        }
        se[i] = ei;
      }
      pd[h] = ph;
      ra[h] = am;
      rb[h] = bm;
    }
    // inclusive scan of x -> a x + b within each half (Hillis-Steele)
#pragma unroll
    for (int h = 0; h < H; ++h) {
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const double ax = __shfl_up(ra[h].x, o), ay = __shfl_up(ra[h].y, o);
        const double bx = __shfl_up(rb[h].x, o), by = __shfl_up(rb[h].y, o);
        if (lane >= o) {
          // (a, b) o (a', b') = (a a', a b' + b)
          const z64 ap = mk(ax, ay), bp = mk(bx, by);
          rb[h] = cfma(rb[h], ra[h], bp);
          ra[h] = ra[h] * ap;
        }
      }
    }
    // right phase entering element i: x_{i-1}, with x_{-1} = 1
    const z64 x0 = ra[0] + rb[0];                       // x_lane
    const z64 end0 = mk(__shfl(x0.x, 63), __shfl(x0.y, 63));
    const z64 x1 = cfma(rb[1], ra[1], end0);            // x_{lane+64}
    z64 in0 = mk(__shfl_up(x0.x, 1), __shfl_up(x0.y, 1));
    z64 in1 = mk(__shfl_up(x1.x, 1), __shfl_up(x1.y, 1));
    if (lane == 0) {
      in0 = mk(1.0, 0.0);
      in1 = end0;
    }
    const z64 xin[2] = {in0, in1};
#pragma unroll
    for (int h = 0; h < H; ++h) {
      const int i = lane + 64 * h;
      if (i < n) {
        sdr[i] = xin[h];
        const z64 dl = dz[h] ? mk(1.0, 0.0) : pd[h] * xin[h];
        if (sq) sq[i] = cmulc(dl, sq[i]);
        if (sdl) sdl[i] = dl;
      }
    }
  }
}

// Discrepancy choice of alpha for one system per group of W lanes (W = 64:
// the whole wave; W = 32: each half-wave searches its own system, every lane
// passing its half's arrays and constants): round 0 tests the floor
// alpha_min = eta ||A||_F^2 (the group's lane 0) and spreads lanes 1..W-1
// over (log alpha_min, log ||A||_F^2 + 1]; then a multisection on the
// bracket with W points per round. T < 0 (noise-free data) keeps the floor.
// Returns the branch (1 floor, 2 root) and writes alpha, the same on every
// lane of the group. The groups' control flow may diverge; the evaluations
// are per lane, and ballots and shuffles stay inside the group.
// PHI: the discrepancy as a function of alpha (evaluated per lane); fro:
// ||A||_F^2 of the (stacked) system, which sets the floor eta ||A||_F^2 and
// the first spread.
template <int W, typename PHI>
__device__ __forceinline__ int dp_choose_alpha_f(int lane_w, PHI phi, double T, double fro,
                                                 double eta, double* alpha_out) {
  static_assert(W == 16 || W == 32 || W == 64, "a group is 16 or 32 lanes or the wave");
  const int lane = lane_w & (W - 1);  // lane within the group
  const int hb = lane_w & (64 - W);   // the group's first lane in the wave
  auto gballot = [&](bool pr) -> unsigned long long {
    const unsigned long long b = __ballot(pr);
    if constexpr (W == 64)
      return b;
    else
      return (b >> hb) & ((1ull << W) - 1ull);
  };
  auto gshfl = [&](double v, int src) -> double { return __shfl(v, hb + src); };
  const double amin = eta * fro;
  double al = amin;
  int br = 1;
  if (T >= 0.0) {
    // round 0: lane 0 tests the floor alpha_min; lanes 1..W-1 spread over
    // (log alpha_min, log ||A||_F^2 + 1], where the root almost always is
    const double h0 = log(fro) + 1.0;
    double lo = log(amin);
    const double st0 = (h0 - lo) / (double)(W - 1);
    double ph = phi(exp(lane == 0 ? lo : lo + st0 * lane));
    unsigned long long bal = gballot(ph >= T);
    if (!(bal & 1ull)) {
      br = 2;
      // bracket [lo, hi] on x = log(alpha) with phi(lo) < T <= phi(hi);
      // flo / fhi hold phi at the ends once known (NaN otherwise)
      const double nan = __longlong_as_double(0x7ff8000000000000ll);
      double hi, flo, fhi = nan;
      if (bal) {
        const int l1 = __ffsll((long long)bal) - 1;
        hi = lo + st0 * l1;
        fhi = gshfl(ph, l1);
        lo = lo + st0 * (l1 - 1);
        flo = gshfl(ph, l1 - 1);
      } else {
        // the root lies above: probe upward in steps of 4
        lo = h0;
        flo = gshfl(ph, W - 1);
        const double pu = phi(exp(h0 + 4.0 * (lane + 1)));
        const unsigned long long bu = gballot(pu >= T);
        if (bu) {
          const int l1 = __ffsll((long long)bu) - 1;
          hi = h0 + 4.0 * (l1 + 1);
          fhi = gshfl(pu, l1);
          if (l1 > 0) {
            lo = h0 + 4.0 * l1;
            flo = gshfl(pu, l1 - 1);
          }
        } else {
          hi = h0 + 4.0 * W;
          lo = hi;
        }
      }
      // Multisection with W points per round. Once phi is known at both
      // ends, the points are packed around the secant estimate of the
      // root (phi is smooth in log alpha, so the secant error shrinks like
      // the square of the bracket). A window that misses the root still
      // leaves a valid, smaller bracket; the round after a miss spreads
      // its points over the whole bracket again.
      // The search stops once the bracket is below 3e-8 in log(alpha): the
      // secant point is then within about curvature * 1e-16 of the root.
      bool miss = false;
      for (int round = 0; round < 24 && hi - lo > 3e-8; ++round) {
        const double wdt = hi - lo;
        double a0 = lo, a1 = hi;
        if (!miss && flo == flo && fhi == fhi && fhi > flo) {
          const double xs = lo + (T - flo) / (fhi - flo) * wdt;
          const double hw = fmax(0.25 * wdt * wdt, 1e-5 * wdt);
          a0 = fmax(lo, xs - hw);
          a1 = fmin(hi, xs + hw);
        }
        // W points in (a0, a1]: the last one is a1 unless a1 = hi (phi(hi) is known)
        const double step = (a1 - a0) / (a1 < hi ? (double)W : (double)(W + 1));
        const double pl = phi(exp(a0 + step * (lane + 1)));
        const unsigned long long b2 = gballot(pl >= T);
        if (b2) {
          const int l1 = __ffsll((long long)b2) - 1;
          if (l1 >= 1 && step <= 2e-3) {
            // The root lies between two points of this round's grid, spaced
            // at most 2e-3: the cubic through the four grid points around it
            // places the root within about step^4 |phi^(4) / phi'| / 24
            // (below 1e-12 in log alpha), so no further round is needed.
            // Newton on the cubic in t (grid index from j0), from the secant
            // point, kept inside the bracketing grid interval.
            const int j0 = min(max(l1 - 2, 0), W - 4);
            const double p0 = gshfl(pl, j0), p1 = gshfl(pl, j0 + 1);
            const double p2 = gshfl(pl, j0 + 2), p3 = gshfl(pl, j0 + 3);
            const double d1 = p1 - p0, d2 = p2 - 2.0 * p1 + p0;
            const double d3 = p3 - 3.0 * p2 + 3.0 * p1 - p0;
            const double pa = gshfl(pl, l1 - 1), pb = gshfl(pl, l1);
            const double ta = (double)(l1 - 1 - j0), tb = ta + 1.0;
            double t = ta + (pb > pa ? (T - pa) / (pb - pa) : 0.5);
#pragma unroll
            for (int it = 0; it < 3; ++it) {
              const double pt = p0 + t * (d1 + (t - 1.0) * (0.5 * d2 + (t - 2.0) * d3 / 6.0));
              const double dp = d1 + (2.0 * t - 1.0) * 0.5 * d2 +
                                (3.0 * t * t - 6.0 * t + 2.0) * d3 / 6.0;
              if (dp > 0.0) t = t - (pt - T) / dp;
              t = fmin(tb, fmax(ta, t));
            }
            *alpha_out = exp(a0 + step * ((double)j0 + t + 1.0));
            return br;
          }
          miss = l1 == 0 && a0 > lo;  // the root may lie left of the window
          hi = a0 + step * (l1 + 1);
          fhi = gshfl(pl, l1);
          if (l1 > 0) {
            lo = a0 + step * l1;
            flo = gshfl(pl, l1 - 1);
          }
        } else {
          miss = a1 < hi;             // the root lies right of the window
          lo = a0 + step * W;
          flo = gshfl(pl, W - 1);
        }
      }
      double xr = 0.5 * (lo + hi);
      if (flo == flo && fhi == fhi && fhi > flo)
        xr = fmin(hi, fmax(lo, lo + (T - flo) / (fhi - flo) * (hi - lo)));
      al = exp(xr);
    }
  }
  *alpha_out = al;
  return br;
}

template <int W>
__device__ __forceinline__ int dp_choose_alpha(int n, int lane_w, const double* sd, const double* se,
                                               const z64* sq, double T, double fro, double eta,
                                               double* alpha_out) {
  return dp_choose_alpha_f<W>(
      lane_w, [&](double al) { return phi_fwd(sd, se, sq, n, al); }, T, fro, eta, alpha_out);
}

// Householder reflectors applied to one vector by a group of G lanes
// (element i held by lane i % G in slot i / G): x <- H_k x for k = k0, k0 + dk,
// ..., with H_k = I - g_k h_k h_k^H and h_k the packed reflector k of R
// (entries k + off .. n - 1). Reflectors are loaded RG at a time so that
// their latency overlaps.
template <int G, int E, int RG>
__device__ __forceinline__ void group_reflect(z64 (&x)[E], const z64* __restrict__ R,
                                              const double* __restrict__ gam, int n, int gl,
                                              int k0, int kend, int dk, int off) {
  // reflector k has entries k + off .. n - 1
  for (int kb = k0; dk > 0 ? kb < kend : kb > kend; kb += dk * RG) {
    z64 v[RG][E];
    double gg[RG];
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      const int k = kb + dk * g;
      const bool ok = dk > 0 ? k < kend : k > kend;
      gg[g] = ok ? gam[k] : 0.0;
#pragma unroll
      for (int e = 0; e < E; ++e) {
        const int i = gl + G * e;
        v[g][e] = (ok && i >= k + off && i < n) ? R[tri_start(k, n, off) + (i - k - off)]
                                                 : mk(0.0, 0.0);
      }
    }
#pragma unroll
    for (int g = 0; g < RG; ++g) {
      z64 sm = mk(0.0, 0.0);
#pragma unroll
      for (int e = 0; e < E; ++e) sm = cfmac(sm, v[g][e], x[e]);
      sm.x = lanes_sum<G>(sm.x);
      sm.y = lanes_sum<G>(sm.y);
      sm = gg[g] * sm;
#pragma unroll
      for (int e = 0; e < E; ++e) x[e] = x[e] - v[g][e] * sm;
    }
  }
}

// One factorization per system (the shared orbit factorizations go through
// k_dpo_*): SPW systems per single-wave workgroup, each in a group of
// G = 64 / SPW lanes. The phase scaling uses the whole wave for one system at
// a time; the alpha searches (G trial alphas per round), the Elden solve and
// the back-transform v^ = V (D_R y) run for the SPW systems at once, each in
// its group, so their reductions span G lanes only.
template <int NMAX, int SPW>
__global__ __launch_bounds__(64, SPW == 2 ? 3 : 2) void k_dp_solve(DpArgs a) {
  constexpr int G = 64 / SPW;
  constexpr int E = (NMAX + G - 1) / G;
  // reflector rows loaded ahead in the passes
  // (two at four elements per lane for n > 64: four would take the kernel
  // past 256 registers, one wave per SIMD)
  constexpr int RG = (E >= 8 || (E >= 4 && NMAX > 64)) ? 2 : (E == 1 ? 8 : 4);
  // per system: real bidiagonal (sd, se; the Elden solve overwrites them
  // with its rho and off), q' (sq), the complex superdiagonal and then the
  // Elden right-hand side (srr), the complex diagonal and then y (sy), the
  // right phases (sdr)
  // (nothing else: at SPW = 4 and NMAX = 64 these are 20 KiB, so that eight
  // one-wave workgroups fit in a CU's 160 KiB)
  __shared__ double sd[SPW][NMAX], se[SPW][NMAX];
  __shared__ z64 sq[SPW][NMAX], srr[SPW][NMAX], sy[SPW][NMAX], sdr[SPW][NMAX];
  const int lane = threadIdx.x, grp = lane / G, gl = lane % G;
  const int n = a.n;
  const int total = *a.count;
  // groups of SPW systems that hold work in this launch
  int c0;
  const int nsys = launch_range(a.osys0, a.ocount, a.slot0, a.OC, a.chunk0, a.C, total, &c0);
  const int nact = nsys > 0 ? (nsys + SPW - 1) / SPW : 0;
  // Workgroups go to the eight XCDs in turn: XCD x (of V = min(8, grid))
  // takes the contiguous group range [x per, (x + 1) per).
  const int NG = gridDim.x, V = NG < 8 ? NG : 8;
  const int xcd = blockIdx.x % V, nbx = (NG - xcd + V - 1) / V;
  const int per = (nact + V - 1) / V;
  for (int k = blockIdx.x / V; k < per; k += nbx) {
    const int sg = xcd * per + k;
    if (sg >= nact) break;
    const int sl0 = sg * SPW;
    // this lane's group system
    const int sl = sl0 + grp, gs = c0 + sl;
    const bool live = sl < nsys;
    int f = 0;
    long m = 0, fs = 0;
    if (live) {
      const int fm = a.list[gs];
      f = (int)(fm / a.N);
      m = fm - (long)f * a.N;
      // the system's own factorization slot
      fs = sl;
      for (int e = 0; e < E; ++e) {
        const int i = gl + G * e;
        if (i < n) {
          sy[grp][i] = a.dg[fs * n + i];
          srr[grp][i] = a.sp[fs * n + i];
          sq[grp][i] = a.q[(long)sl * n + i];
        }
      }
    }
    __syncthreads();
    // phase scaling one system at a time over the whole wave; then the alpha
    // of every system at once, each group searching its own system with G
    // points per round (three rounds for all of them, against two for each
    // in turn with 64 points); with one system per wave the whole wave
    // searches. The group of system s keeps its alpha and branch (the same
    // on every lane).
    constexpr bool GROUPED = SPW == 2 || (SPW == 4 && NMAX <= 64);
    double gal = 0.0;
    int gbr = 0;
    for (int s = 0; s < SPW; ++s) {
      const int sls = sl0 + s, gss = c0 + sls;
      if (sls >= nsys) break;
      const int fms = a.list[gss];
      const int fsf = (int)(fms / a.N);
      const long fss = sls;
      dp_phase_scale<NMAX>(n, lane, sd[s], se[s], sq[s], srr[s], sy[s], sdr[s]);
      __syncthreads();
      // kept for the derivative kernels
      for (int i = lane; i < n; i += 64) {
        a.bd_d[(long)sls * n + i] = sd[s][i];
        a.bd_e[(long)sls * n + i] = se[s][i];
        a.bd_dr[(long)sls * n + i] = sdr[s][i];
      }
      if constexpr (!GROUPED) {
        double al;
        int br;
        if (a.alpha_fixed) {
          al = a.alpha_fixed[fsf];
          br = a.branch_fixed[fsf];
        } else {
          br = dp_choose_alpha<64>(n, lane, sd[s], se[s], sq[s], a.thr2[fsf], a.fro[fss], a.eta,
                                   &al);
        }
        if (grp == s) {
          gal = al;
          gbr = br;
        }
      }
      __syncthreads();
    }
    if constexpr (GROUPED) {
      if (live) {
        if (a.alpha_fixed) {
          gal = a.alpha_fixed[f];
          gbr = a.branch_fixed[f];
        } else {
          gbr = dp_choose_alpha<64 / SPW>(n, lane, sd[grp], se[grp], sq[grp], a.thr2[f],
                                          a.fro[fs], a.eta, &gal);
        }
      }
      __syncthreads();
    }
    // Elden solve of each group's system by the group's first lane
    const int br = live ? gbr : 0;
    const double al = live ? gal : 0.0;
    if (br != 0 && gl == 0)
      elden_solve(sd[grp], se[grp], sq[grp], n, al, sd[grp], se[grp], srr[grp], sy[grp]);
    __syncthreads();
    if (live) {
      const int fm = a.list[gs];
      if (br == 0) {
        // one alpha per frequency with the data inside the noise level: v^ = 0
        const long o0 = (long)f * a.nzv * a.N + m;
        for (int e = 0; e < E; ++e) {
          const int i = gl + G * e;
          if (i < a.nzv) {
            if (a.vh_single)
              ((z32*)a.Vh)[o0 + (long)i * a.N] = mk(0.f, 0.f);
            else
              ((z64*)a.Vh)[o0 + (long)i * a.N] = mk(0.0, 0.0);
          }
        }
        if (gl == 0) {
          a.alpha[fm] = INFINITY;
          a.branch[fm] = 0;
        }
      } else {
        // v^ = V (D_R y), V = P_0 P_1 ... P_{n-3}: apply P_{n-3} first
        z64 y[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int i = gl + G * e;
          y[e] = i < n ? sdr[grp][i] * sy[grp][i] : mk(0.0, 0.0);
        }
        group_reflect<G, E, RG>(y, a.refl + fs * tri_size(n, 1), a.gam + fs * n, n, gl, n - 3, -1, -1, 1);
        const long o0 = (long)f * a.nzv * a.N + m;
#pragma unroll
        for (int e = 0; e < E; ++e) {
          const int i = gl + G * e;
          if (i < a.nzv) {
            if (a.vh_single)
              ((z32*)a.Vh)[o0 + (long)i * a.N] = cast<float>(y[e]);
            else
              ((z64*)a.Vh)[o0 + (long)i * a.N] = y[e];
          }
        }
        if (gl == 0) {
          a.alpha[fm] = al;
          a.branch[fm] = (signed char)br;
        }
      }
    }
    __syncthreads();
  }
}

// ------------------------------------------------- one alpha per frequency

struct GlobalArgs {
  const z64* dg;        // chunk workspace as for k_dp_solve
  const z64* sp;
  const z64* q;
  const double* fro;
  const int* list;
  const int* count;
  int chunk0, C, n;
  long N;
  double* gd;           // [FN][n] phase-scaled real bidiagonal, by compacted index
  double* ge;
  z64* gq;              // [FN][n] q' = D_L^H U^H w
  double* gfro;         // [FN] ||A||_F^2
  int* gf;              // [FN] frequency
};

// Phase-scale every system of a chunk and keep its real bidiagonal, q' and
// ||A||_F^2 under its compacted index (one wave per system).
template <int NMAX>
__global__ __launch_bounds__(64) void k_global_prep(GlobalArgs a) {
  __shared__ double sd[NMAX], se[NMAX];
  __shared__ z64 sq[NMAX], srr[NMAX], sy[NMAX], sdr[NMAX];
  const int lane = threadIdx.x;
  const int n = a.n;
  const int total = *a.count;
  for (int sl = blockIdx.x; sl < a.C; sl += gridDim.x) {
    const int gs = a.chunk0 + sl;
    if (gs >= total) break;
    for (int i = lane; i < n; i += 64) {
      sy[i] = a.dg[(long)sl * n + i];
      srr[i] = a.sp[(long)sl * n + i];
      sq[i] = a.q[(long)sl * n + i];
    }
    __syncthreads();
    dp_phase_scale<NMAX>(n, lane, sd, se, sq, srr, sy, sdr);
    __syncthreads();
    for (int i = lane; i < n; i += 64) {
      a.gd[(long)gs * n + i] = sd[i];
      a.ge[(long)gs * n + i] = se[i];
      a.gq[(long)gs * n + i] = sq[i];
    }
    if (lane == 0) {
      a.gfro[gs] = a.fro[sl];
      a.gf[gs] = (int)(a.list[gs] / a.N);
    }
    __syncthreads();
  }
}

// start[f] = first compacted index of frequency f (systems are compacted in
// increasing f * N + m), start[F] = total
__global__ void k_global_ranges(const int* __restrict__ gf, const int* __restrict__ count, int F,
                                int* __restrict__ start) {
  const int total = *count;
  for (int gs = blockIdx.x * blockDim.x + threadIdx.x; gs < total; gs += gridDim.x * blockDim.x) {
    const int f = gf[gs];
    const int fp = gs > 0 ? gf[gs - 1] : -1;
    for (int g = fp + 1; g <= f; ++g) start[g] = gs;  // also frequencies with no system
    if (gs == total - 1)
      for (int g = f + 1; g <= F; ++g) start[g] = total;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && total == 0)
    for (int g = 0; g <= F; ++g) start[g] = 0;
}

// Search state of one frequency: the total discrepancy
// Phi(x) = sum_m phi_m(exp x) is evaluated at x0 + step (l + 1), l = 0..63,
// per round; [lo, hi] brackets the root of Phi = target.
struct GState {
  double lo, hi, flo, fhi;  // bracket and Phi at its ends (NaN: unknown)
  double x0, step, a1;      // this round's points and the window's right end
  double h0, target, amin;
  int phase;                // 0 first spread, 1 upward probe, 2 multisection, 3 done
  int miss;
};

// Per frequency (one wave): alpha_min = eta max_m ||A_m||_F^2, the target
// tau^2 N delta_m^2 = N thr2[f], and the cases settled without a search:
// no system, noise-free data (floor), or sum_m ||w_m||^2 <= target (v = 0).
__global__ __launch_bounds__(64) void k_global_init(const int* __restrict__ start,
                                                    const double* __restrict__ gfro,
                                                    const double* __restrict__ wn2,
                                                    const int* __restrict__ list,
                                                    const double* __restrict__ thr2, long N,
                                                    double eta, GState* __restrict__ S,
                                                    double* __restrict__ alpha_f,
                                                    signed char* __restrict__ branch_f) {
  const int f = blockIdx.x, lane = threadIdx.x;
  const int s0 = start[f], s1 = start[f + 1];
  double mx = 0.0, ws = 0.0;
  for (int gs = s0 + lane; gs < s1; gs += 64) {
    mx = fmax(mx, gfro[gs]);
    ws += wn2[list[gs]];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  ws = group_sum<64>(ws);
  if (lane != 0) return;
  const double nan = __longlong_as_double(0x7ff8000000000000ll);
  GState g;
  g.flo = g.fhi = nan;
  g.miss = 0;
  g.amin = eta * mx;
  g.target = thr2[f] < 0.0 ? -1.0 : thr2[f] * (double)N;
  g.h0 = mx > 0.0 ? log(mx) + 1.0 : 0.0;
  g.lo = g.hi = g.a1 = 0.0;
  g.x0 = g.step = 0.0;
  g.phase = 3;
  double al = INFINITY;
  signed char br = 0;
  if (s1 > s0 && mx > 0.0) {
    if (g.target < 0.0) {
      al = g.amin;
      br = 1;
    } else if (ws > g.target) {
      // lane 0 tests the floor; lanes 1..63 spread over (log alpha_min, h0]
      g.lo = log(g.amin);
      g.step = (g.h0 - g.lo) / 63.0;
      g.x0 = g.lo - g.step;
      g.phase = 0;
    }
  }
  S[f] = g;
  alpha_f[f] = al;
  branch_f[f] = br;
}

// Phi at this round's 64 points, partial sums per block: grid (B, F), one
// wave per block; block b takes a contiguous slice of frequency f's systems,
// one system after another, so the summation order is fixed.
template <int NMAX>
__global__ __launch_bounds__(64) void k_global_eval(const GState* __restrict__ S,
                                                    const int* __restrict__ start,
                                                    const double* __restrict__ gd,
                                                    const double* __restrict__ ge,
                                                    const z64* __restrict__ gq, int n,
                                                    double* __restrict__ part) {
  __shared__ double sd[NMAX], se[NMAX];
  __shared__ z64 sq[NMAX];
  const int f = blockIdx.y, b = blockIdx.x, B = gridDim.x, lane = threadIdx.x;
  if (S[f].phase == 3) return;
  const int s0 = start[f], s1 = start[f + 1];
  const int K = (s1 - s0 + B - 1) / B;
  const int a = s0 + b * K, e = min(a + K, s1);
  const double al = exp(S[f].x0 + S[f].step * (lane + 1));
  double acc = 0.0;
  for (int gs = a; gs < e; ++gs) {
    for (int i = lane; i < n; i += 64) {
      sd[i] = gd[(long)gs * n + i];
      se[i] = ge[(long)gs * n + i];
      sq[i] = gq[(long)gs * n + i];
    }
    __syncthreads();
    acc += phi_fwd(sd, se, sq, n, al);
    __syncthreads();
  }
  part[((long)f * B + b) * 64 + lane] = acc;
}

// One round of the search per frequency (one wave): Phi from the partial
// sums in block order, then the bracket update of the per-system search
// (first spread, upward probe in steps of 4, 64-point multisection with
// secant windows); a converged bracket, or the last round, fixes alpha at
// the secant point.
__global__ __launch_bounds__(64) void k_global_update(GState* __restrict__ S,
                                                      const double* __restrict__ part, int B,
                                                      int last, double* __restrict__ alpha_f,
                                                      signed char* __restrict__ branch_f) {
  const int f = blockIdx.x, lane = threadIdx.x;
  GState g = S[f];
  if (g.phase == 3) return;
  double ph = 0.0;
  for (int b = 0; b < B; ++b) ph += part[((long)f * B + b) * 64 + lane];
  const double T = g.target;
  const unsigned long long bal = __ballot(ph >= T);
  if (g.phase == 0) {
    if (bal & 1ull) {
      g.phase = 3;
      if (lane == 0) {
        S[f] = g;
        alpha_f[f] = g.amin;
        branch_f[f] = 1;
      }
      return;
    }
    if (bal) {
      const int l1 = __ffsll((long long)bal) - 1;
      g.hi = g.x0 + g.step * (l1 + 1);
      g.fhi = __shfl(ph, l1);
      g.lo = g.x0 + g.step * l1;
      g.flo = __shfl(ph, l1 - 1);
    } else {
      g.lo = g.h0;
      g.flo = __shfl(ph, 63);
      g.x0 = g.h0;
      g.step = 4.0;
      g.phase = 1;
      if (lane == 0) S[f] = g;
      return;
    }
  } else if (g.phase == 1) {
    if (bal) {
      const int l1 = __ffsll((long long)bal) - 1;
      g.hi = g.x0 + 4.0 * (l1 + 1);
      g.fhi = __shfl(ph, l1);
      if (l1 > 0) {
        g.lo = g.x0 + 4.0 * l1;
        g.flo = __shfl(ph, l1 - 1);
      }
    } else {
      g.hi = g.lo = g.h0 + 4.0 * 64;
    }
  } else {
    const double a0 = g.x0;
    if (bal) {
      const int l1 = __ffsll((long long)bal) - 1;
      g.miss = l1 == 0 && a0 > g.lo;
      g.hi = a0 + g.step * (l1 + 1);
      g.fhi = __shfl(ph, l1);
      if (l1 > 0) {
        g.lo = a0 + g.step * l1;
        g.flo = __shfl(ph, l1 - 1);
      }
    } else {
      g.miss = g.a1 < g.hi;
      g.lo = a0 + g.step * 64;
      g.flo = __shfl(ph, 63);
    }
  }
  const bool known = g.flo == g.flo && g.fhi == g.fhi && g.fhi > g.flo;
  const double wdt = g.hi - g.lo;
  if (last || !(wdt > 1e-13 * fmax(1.0, fabs(g.hi)))) {
    double xr = 0.5 * (g.lo + g.hi);
    if (known) xr = fmin(g.hi, fmax(g.lo, g.lo + (T - g.flo) / (g.fhi - g.flo) * wdt));
    g.phase = 3;
    if (lane == 0) {
      S[f] = g;
      alpha_f[f] = exp(xr);
      branch_f[f] = 2;
    }
    return;
  }
  double a0 = g.lo, a1 = g.hi;
  if (!g.miss && known) {
    const double xs = g.lo + (T - g.flo) / (g.fhi - g.flo) * wdt;
    const double hw = fmax(0.25 * wdt * wdt, 1e-5 * wdt);
    a0 = fmax(g.lo, xs - hw);
    a1 = fmin(g.hi, xs + hw);
  }
  g.x0 = a0;
  g.a1 = a1;
  g.step = (a1 - a0) / (a1 < g.hi ? 64.0 : 65.0);
  g.phase = 2;
  if (lane == 0) S[f] = g;
}

// ------------------------------------------------------- thin data layer

// Data in a thin layer: nd <= THIN_ND planes at any heights, nd <= nz, so
// every A_m is wide (nd x nz). With the Householder QR A^T = Q [R; 0]
// (lanes over the nz rows of A^T), A = R^T Q^T restricted to Q's first nd
// columns, and the minimum-norm Tikhonov solution is v = conj(Q [conj(y); 0])
// with y the Tikhonov solution of the nd x nd system R^T y = w. y comes from
// the one-sided Jacobi SVD of R^T, alpha from the discrepancy principle by
// 64-point multisection on log(alpha) down to a relative bracket of 1e-15
// (the misfit costs O(nd) per trial). One wave per active system; the small
// dense steps run redundantly on every lane.
constexpr int THIN_ND = 4;

struct ThinArgs {
  const z64* gsys;       // per system, row-major A [nd][nz] (pitch tpitch)
  int tpitch;
  const z64* What;       // [F][nd][N]
  const int* list;
  const int* count;
  int nd, nz;
  long N;
  const double* thr2;    // [F] (tau delta_m)^2, < 0 for noise-free data
  double eta;
  int tsvd;              // 1: truncated SVD instead of Tikhonov
  void* Vh;
  int vh_single;
  double* alpha;
  signed char* branch;
};

__device__ __forceinline__ z64 thin_phase(z64 a) {
  const double r = sqrt(nrm2(a));
  return r > 0.0 ? mk(a.x / r, a.y / r) : mk(1.0, 0.0);
}

template <int NMAX>
__global__ __launch_bounds__(64) void k_thin_solve(ThinArgs a) {
  __shared__ z64 sb[THIN_ND][NMAX];  // rows of A (columns of A^T), then reflectors
  __shared__ double sg[THIN_ND];
  __shared__ z64 sr[THIN_ND][THIN_ND];
  __shared__ z64 sw[THIN_ND];
  const int lane = threadIdx.x, nd = a.nd, nz = a.nz;
  const int total = *a.count;
  for (int gs = blockIdx.x; gs < total; gs += gridDim.x) {
    const int fm = a.list[gs];
    const int f = (int)(fm / a.N);
    const long m = fm - (long)f * a.N;
    const z64* row = a.gsys + (long)fm * a.tpitch;
    double fr = 0.0;
    for (int j = 0; j < nd; ++j)
      for (int l = lane; l < nz; l += 64) {
        const z64 v = row[j * nz + l];
        sb[j][l] = v;
        fr += nrm2(v);
      }
    fr = lanes_sum<64>(fr);
    if (lane < nd) sw[lane] = a.What[((long)f * nd + lane) * a.N + m];
    __syncthreads();
    // Householder QR of A^T, column by column
    for (int j = 0; j < nd; ++j) {
      double s = 0.0;
      for (int l = lane; l < nz; l += 64)
        if (l >= j) s += nrm2(sb[j][l]);
      s = lanes_sum<64>(s);
      const z64 piv = sb[j][j];
      const double xn = sqrt(s), a2 = sqrt(nrm2(piv));
      const z64 ph = thin_phase(piv);
      const z64 beta = mk(-ph.x * xn, -ph.y * xn);
      const double g = xn > 0.0 ? 1.0 / (xn * (xn + a2)) : 0.0;
      __syncthreads();
      if (lane == 0) {
        sb[j][j] = piv - beta;
        sg[j] = g;
        sr[j][j] = beta;
      }
      __syncthreads();
      for (int k = j + 1; k < nd; ++k) {
        z64 t = mk(0.0, 0.0);
        for (int l = lane; l < nz; l += 64)
          if (l >= j) t = cfmac(t, sb[j][l], sb[k][l]);
        t.x = lanes_sum<64>(t.x);
        t.y = lanes_sum<64>(t.y);
        t = g * t;
        for (int l = lane; l < nz; l += 64)
          if (l >= j) sb[k][l] = cfms(sb[k][l], sb[j][l], t);
        __syncthreads();
        if (lane == 0) sr[j][k] = sb[k][j];
        __syncthreads();
      }
    }
    // L = R^T (lower triangular) and its one-sided Jacobi SVD: M = L V = U S
    z64 M[THIN_ND][THIN_ND], V[THIN_ND][THIN_ND], w[THIN_ND];
#pragma unroll
    for (int i = 0; i < THIN_ND; ++i) {
      w[i] = i < nd ? sw[i] : mk(0.0, 0.0);
#pragma unroll
      for (int j = 0; j < THIN_ND; ++j) {
        M[i][j] = (i < nd && j < nd && i >= j) ? sr[j][i] : mk(0.0, 0.0);
        V[i][j] = mk(i == j ? 1.0 : 0.0, 0.0);
      }
    }
    for (int sweep = 0; sweep < 30; ++sweep) {
      bool off = false;
#pragma unroll
      for (int p = 0; p < THIN_ND; ++p)
#pragma unroll
        for (int q = p + 1; q < THIN_ND; ++q) {
          if (q >= nd) continue;
          double ap = 0.0, aq = 0.0;
          z64 c = mk(0.0, 0.0);
#pragma unroll
          for (int i = 0; i < THIN_ND; ++i) {
            ap += nrm2(M[i][p]);
            aq += nrm2(M[i][q]);
            c = cfmac(c, M[i][p], M[i][q]);
          }
          const double ac = sqrt(nrm2(c));
          if (!(ac > 1e-15 * sqrt(ap * aq))) continue;
          off = true;
          const z64 e = mk(c.x / ac, c.y / ac);
          const double zeta = (aq - ap) / (2.0 * ac);
          const double t = zeta != 0.0 ? copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta))
                                       : 1.0;
          const double cs = 1.0 / sqrt(1.0 + t * t), sn = cs * t;
#pragma unroll
          for (int i = 0; i < THIN_ND; ++i) {
            const z64 mp = M[i][p], mq = cmulc(e, M[i][q]);
            M[i][p] = cs * mp - sn * mq;
            M[i][q] = sn * mp + cs * mq;
            const z64 vp = V[i][p], vq = cmulc(e, V[i][q]);
            V[i][p] = cs * vp - sn * vq;
            V[i][q] = sn * vp + cs * vq;
          }
        }
      if (!off) break;
    }
    double sig[THIN_ND], b2[THIN_ND];
    z64 b[THIN_ND];
    double wn = 0.0, bn = 0.0, smax = 0.0;
    bool defic = false;
#pragma unroll
    for (int i = 0; i < THIN_ND; ++i) {
      double s2 = 0.0;
      z64 bi = mk(0.0, 0.0);
#pragma unroll
      for (int r = 0; r < THIN_ND; ++r) {
        s2 += nrm2(M[r][i]);
        bi = cfmac(bi, M[r][i], w[r]);
      }
      sig[i] = sqrt(s2);
      b[i] = sig[i] > 0.0 ? mk(bi.x / sig[i], bi.y / sig[i]) : mk(0.0, 0.0);
      defic = defic || (i < nd && !(s2 > 0.0));
      b2[i] = nrm2(b[i]);
      wn += nrm2(w[i]);
      bn += b2[i];
      smax = fmax(smax, s2);
    }
    // the square R^T spans C^nd unless a singular value is zero, so the
    // part of w outside its range is zero (wn - bn would only be rounding)
    const double rho2 = defic ? fmax(0.0, wn - bn) : 0.0;
    // phi(alpha) = sum_i (alpha / (s_i^2 + alpha))^2 |b_i|^2 + rho^2
    auto phi = [&](double al) {
      double s = rho2;
#pragma unroll
      for (int i = 0; i < THIN_ND; ++i) {
        const double q = al / (sig[i] * sig[i] + al);
        s += q * q * b2[i];
      }
      return s;
    };
    const double T = a.thr2[f];
    const double amin = a.eta * fr;
    double al = amin;
    int br = 1;
    // TSVD: keep the fewest leading triplets (s_i^2 > eta ||A||_F^2) whose
    // residual rho^2 + sum_{i >= k} |b_i|^2 is within T; alpha receives k
    double keep[THIN_ND];
#pragma unroll
    for (int i = 0; i < THIN_ND; ++i) keep[i] = 1.0;
    if (a.tsvd) {
      // rank of each singular value in decreasing order (ties by index)
      int rank[THIN_ND];
#pragma unroll
      for (int i = 0; i < THIN_ND; ++i) {
        int r = 0;
#pragma unroll
        for (int j = 0; j < THIN_ND; ++j)
          r += (j < nd) && (sig[j] > sig[i] || (sig[j] == sig[i] && j < i));
        rank[i] = r;
      }
      int kmax = 0;
      double sb2[THIN_ND];
#pragma unroll
      for (int k = 0; k < THIN_ND; ++k) {
        sb2[k] = 0.0;
#pragma unroll
        for (int i = 0; i < THIN_ND; ++i)
          if (i < nd && rank[i] == k) sb2[k] = b2[i];
        kmax += (k < nd) && (sig[k] * sig[k] > amin);
      }
      // tails sum_{i >= k} |b_i|^2 in decreasing-singular-value order,
      // accumulated from the smallest singular value up
      double tail[THIN_ND + 1];
      tail[THIN_ND] = 0.0;
#pragma unroll
      for (int k = THIN_ND - 1; k >= 0; --k) tail[k] = k < nd ? tail[k + 1] + sb2[k] : 0.0;
      int k = nd;
      bool found = false;
#pragma unroll
      for (int kk = 0; kk <= THIN_ND; ++kk)
        if (!found && kk <= nd && tail[kk] + rho2 <= T) {
          k = kk;
          found = true;
        }
      k = min(k, kmax);
#pragma unroll
      for (int i = 0; i < THIN_ND; ++i) keep[i] = (i < nd && rank[i] < k) ? 1.0 : 0.0;
      al = (double)k;
      br = 0;
    } else if (T >= 0.0 && phi(amin) < T) {
      br = 2;
      double lo = log(amin), hi = log(smax) + 1.0;
      for (int round = 0; round < 60 && hi - lo > 1e-15 * fmax(1.0, fabs(hi)); ++round) {
        const double x = lo + (hi - lo) * (lane + 1) / 64.0;
        const unsigned long long bal = __ballot(phi(exp(x)) >= T);
        if (!bal) {
          // the root lies above: look further up
          lo = hi;
          hi = hi + 256.0;
          continue;
        }
        const int l1 = __ffsll((long long)bal) - 1;
        const double nh = __shfl(x, l1);
        if (l1 > 0) lo = __shfl(x, l1 - 1);
        hi = nh;
      }
      al = exp(0.5 * (lo + hi));
    }
    // y = V diag(s / (s^2 + alpha)) b, then v = conj(H_0 ... H_{nd-1} [conj(y); 0])
    z64 y[THIN_ND];
#pragma unroll
    for (int j = 0; j < THIN_ND; ++j) {
      y[j] = mk(0.0, 0.0);
#pragma unroll
      for (int i = 0; i < THIN_ND; ++i) {
        // Tikhonov filter s / (s^2 + alpha), or 1 / s for a kept TSVD triplet
        const double c = !(sig[i] > 0.0) ? 0.0
                         : a.tsvd         ? keep[i] / sig[i]
                                          : sig[i] / (sig[i] * sig[i] + al);
        y[j] = cfma(y[j], V[j][i], c * b[i]);
      }
    }
    z64 t0 = mk(0.0, 0.0), t1 = mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j < THIN_ND; ++j) {
      if (lane == j && j < nd) t0 = cj(y[j]);
    }
    for (int j = nd - 1; j >= 0; --j) {
      const z64 u0 = (lane >= j && lane < nz) ? sb[j][lane] : mk(0.0, 0.0);
      const z64 u1 = (NMAX > 64 && lane + 64 < nz) ? sb[j][lane + 64] : mk(0.0, 0.0);
      z64 s = cmulc(u0, t0);
      if (NMAX > 64) s = cfmac(s, u1, t1);
      s.x = lanes_sum<64>(s.x);
      s.y = lanes_sum<64>(s.y);
      s = sg[j] * s;
      t0 = t0 - u0 * s;
      if (NMAX > 64) t1 = t1 - u1 * s;
    }
    const long o0 = (long)f * nz * a.N + m;
    if (lane < nz) {
      if (a.vh_single)
        ((z32*)a.Vh)[o0 + (long)lane * a.N] = cast<float>(cj(t0));
      else
        ((z64*)a.Vh)[o0 + (long)lane * a.N] = cj(t0);
    }
    if (NMAX > 64 && lane + 64 < nz) {
      if (a.vh_single)
        ((z32*)a.Vh)[o0 + (long)(lane + 64) * a.N] = cast<float>(cj(t1));
      else
        ((z64*)a.Vh)[o0 + (long)(lane + 64) * a.N] = cj(t1);
    }
    if (lane == 0) {
      a.alpha[fm] = al;
      a.branch[fm] = (signed char)br;
    }
    __syncthreads();
  }
}

}  // namespace fl
