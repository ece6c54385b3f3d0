// Host side of the flat-layer inversion library: plan construction, argument
// validation, table building and the launch sequence of Algorithm 2 on one
// HIP stream. The C ABI is declared in include/flayer.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/flayer.h"
#include "adjoint.hpp"
#include "dp_orbit.hpp"
#include "fft.hpp"
#include "joint.hpp"
#include "pointwise.hpp"
#include "solver.hpp"
#include "tsvd.hpp"

using namespace fl;

namespace {

thread_local std::string g_err;

fl_status fail(fl_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fl_status fail(fl_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define HIPCHK(expr)                                                                      \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? FL_ENOMEM : FL_EDEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

#define LAUNCHCHK()                                                                   \
  do {                                                                                \
    hipError_t e_ = hipGetLastError();                                                \
    if (e_ != hipSuccess)                                                             \
      return fail(FL_EDEVICE, "kernel launch: %s (%s:%d)", hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                \
  } while (0)

bool smooth235(int n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

unsigned nblk(long n, int t) { return (unsigned)((n + t - 1) / t); }

}  // namespace

// Workspaces of the derivative calls: the plan's own (allocated by its
// first derivative call), or carved from the library's static scratch array
// by fl_invert_vjp_noalloc.
struct AdjBufs {
  z64 *xi_tmp = nullptr, *vbar = nullptr, *ubar = nullptr, *vbar2 = nullptr;  // [F][nvox]
  void *Xb = nullptr, *Yb = nullptr;  // [F][max(nd, nz)][N] complex128
  double *cm = nullptr, *Tb = nullptr;  // [F N], [F]
};

struct fl_plan {
  int dev = 0;  // the device current at creation (the plan's memory lives there)
  int nx, ny, nz, nd, px, py, F;
  double h, c0;
  double hz;  // vertical cell size (h unless fl_opts.hz says otherwise)
  std::vector<double> planes, omegas;
  fl_opts opts;
  hipStream_t st;
  long N;
  int nzeta, TP, ox, oy, n;
  // tables (always FP64)
  z64 *tw_x = nullptr, *tw_y = nullptr, *tw_z = nullptr;
  z64* gtab = nullptr;  // [F][nzeta][N]
  z64* gsys = nullptr;  // [F][N][TP]
  z64* ktab = nullptr;  // [F][2nz][N]
  z64* ttab = nullptr;  // [F][2nz][N] z-transforms of the gtab rows (first fl_forward)
  // single-precision copies used by the mixed path
  z32 *tw_x32 = nullptr, *tw_y32 = nullptr, *tw_z32 = nullptr;
  z32* ktab32 = nullptr;
  int prec = 0;  // 0: FP64 throughout; 1: FP32 FFTs/convolution/storage
  // workspaces (complex64 or complex128 by precision)
  void *What = nullptr, *Vh = nullptr, *w1 = nullptr, *w2 = nullptr;
  z64 *vX = nullptr, *u = nullptr, *u0w = nullptr;
  double *wn2 = nullptr, *partial = nullptr, *thr2 = nullptr, *norm2 = nullptr;
  double* rowsq = nullptr;  // per row of W: sum of squares (stage (a) rows)
  // weights of the frequencies in the least-squares xi (fl_set_frequency_weights)
  double* fw = nullptr;
  std::vector<double> fw_host;
  int *flag = nullptr, *cnt = nullptr, *list = nullptr, *count = nullptr;
  int nb_scan = 0;
  // solver chunk
  int C = 0;
  // launch schedule (fl_tuning): bidiagonalization variant and grid sizes
  int bd_var = 0, bd_grid = 0, dp_grid = 0, dp_spw = 0;
  z64 *dg = nullptr, *sp = nullptr, *q = nullptr, *refl = nullptr;
  double *fro = nullptr, *wnc = nullptr, *gam = nullptr;
  double *bd_d = nullptr, *bd_e = nullptr;
  z64* bd_dr = nullptr;
  // one alpha per frequency (alpha_rule 1): phase-scaled bidiagonals of every
  // compacted system, the search state and per-block partial sums
  double *gd = nullptr, *ge = nullptr, *gfro = nullptr, *gpart = nullptr, *galpha = nullptr;
  z64* gq = nullptr;
  int *gf = nullptr, *gstart = nullptr;
  GState* gst = nullptr;
  signed char* gbranch = nullptr;
  int gB = 0;
  // shared factorizations: orbits of the wavenumber symmetries (orep [N]
  // representative, omem [N][8] members of a representative's orbit), the
  // active orbits compacted like the systems (oflag: active members per
  // representative), the active systems regrouped by orbit (ocnt: the
  // active members per block of 1024 representatives, then the blocks'
  // offsets), and the left reflectors
  bool orbits = false;
  int n_orb = 0;
  // thin data layer (nd <= THIN_ND planes at any heights): zt [nd][nz] the
  // height differences of the table planes
  bool thin = false;
  // a general plane set (planes off X's lattice, or nd != nz, more than
  // THIN_ND planes): table rows of nd x nz entries, systems zero padded to
  // the supported size n >= max(nd, nz)
  bool general = false;
  double* zt = nullptr;
  int *orep = nullptr, *omem = nullptr, *oflag = nullptr, *olist = nullptr, *ocount = nullptr,
      *oslot = nullptr, *ocnt = nullptr, *olist_sys = nullptr;
  // member ranges of the compacted orbits [F n_orb + 1]; the active orbits
  // are factorized C at a time (orbit chunks) when they may exceed C
  int* osys0 = nullptr;
  // first compacted orbit of the chunk whose factorizations the workspace
  // holds (-1: none known), so that the derivative pass after a forward
  // solve re-factorizes only the chunks it no longer holds
  int* oresident = nullptr;
  // one alpha per wavenumber over the frequencies (alpha_rule 2): the
  // wavenumbers whose stacked system needs a solve, and their compaction
  int *mflag = nullptr, *mlist = nullptr, *mcount = nullptr;
  z64* refl_l = nullptr;
  z64* qy = nullptr;  // orbit-batched solve: q', then D_R y, per system of a chunk
  int* opos = nullptr;  // plan-time orbits: first system of every (f, m) position
  double* gam_l = nullptr;
  // truncated SVD of the square systems (regularizer 1): per orbit slot the
  // SVD of the phase-scaled real bidiagonal
  bool tsvd_sq = false;
  TsvdOut tsv{};
  // derivative workspaces (allocated by the first fl_invert_vjp / _jvp)
  bool has_adj = false;
  AdjBufs adj;
  double* alpha = nullptr;
  signed char* branch = nullptr;
  // Lippmann-Schwinger solve (allocated by the first fl_forward with maxit > 0)
  bool has_ls = false;
  z64* bv[7] = {};          // x, r, r^, p, v, s, t  [F][nvox]
  z64 *lsw = nullptr, *dpart = nullptr, *dots = nullptr;
  z64 *b_rho = nullptr, *b_alpha = nullptr, *b_omega = nullptr, *b_beta = nullptr;
  double* b_bn2 = nullptr;
  int* b_active = nullptr;
  std::vector<void*> allocs;
  size_t bytes = 0;
  int last_active = -1, last_factorized = -1;
  bool last_shared = false;  // the last solve used orbit factorizations
  bool prefactored = false;  // every orbit factorized at plan creation
  // stage tracing
  bool prof = false;
  std::vector<hipEvent_t> ev_pool;
  size_t ev_used = 0;
  std::vector<std::pair<int, hipEvent_t>> marks;
};

namespace {

template <typename P>
fl_status dalloc(fl_plan* p, P** ptr, size_t count) {
  size_t b = count * sizeof(P);
  if (b == 0) b = 16;
  void* v = nullptr;
  hipError_t e = hipMalloc(&v, b);
  if (e != hipSuccess)
    return fail(e == hipErrorOutOfMemory ? FL_ENOMEM : FL_EDEVICE, "hipMalloc(%zu): %s", b,
                hipGetErrorString(e));
  p->allocs.push_back(v);
  p->bytes += b;
  *ptr = (P*)v;
  return FL_OK;
}

fl_status dalloc_bytes(fl_plan* p, void** ptr, size_t b) {
  unsigned char* v = nullptr;
  fl_status s = dalloc(p, &v, b);
  *ptr = v;
  return s;
}

#define ALLOC(ptr, cnt)                          \
  do {                                           \
    fl_status s_ = dalloc(p, &(ptr), (size_t)(cnt)); \
    if (s_ != FL_OK) return s_;                  \
  } while (0)

template <typename T>
fl_status make_twiddles(fl_plan* p, cx<T>** out, int L) {
  std::vector<cx<T>> h(L);
  for (int i = 0; i < L; ++i) {
    // exp(-2 pi i i / L) in extended precision, rounded once
    long double a = -2.0L * 3.14159265358979323846264338327950288L * (long double)i / (long double)L;
    h[i] = mk((T)cosl(a), (T)sinl(a));
  }
  ALLOC(*out, L);
  HIPCHK(hipMemcpy(*out, h.data(), L * sizeof(cx<T>), hipMemcpyHostToDevice));
  return FL_OK;
}

// FFT tiles: a twiddle table of L entries plus two buffers of CB transforms,
// within kFftLds bytes of LDS (the kernels opt in to that much dynamic LDS).
constexpr size_t kFftLds = 96 * 1024;

int pick_cb(int L, size_t esz) {
  long cb = (long)(kFftLds - L * esz) / (2L * (L + 1) * (long)esz);
  int r = 1;
  while (r * 2 <= cb && r < 16) r *= 2;
  return r;
}

size_t fft_lds(int L, int CB, size_t esz) { return ((size_t)L + 2 * (size_t)CB * (L + 1)) * esz; }

template <typename K>
void allow_lds(K kernel) {
  static bool done = false;
  if (!done) {
    (void)hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)kFftLds);
    done = true;
  }
}

template <typename TI, typename T, typename TO, int DIR, int L>
void launch_p2(const FftArgs& g, hipStream_t st) {
  constexpr int CB = p2_cb<L, T>(), NT = CB * (L / P2<L>::E);
  hipLaunchKernelGGL((k_fft_p2<TI, T, TO, DIR, L>), dim3(nblk(g.B, CB), g.planes), dim3(NT), 0, st, g);
}

template <typename TI, typename T, typename TO, int DIR>
fl_status run_fft(const FftArgs& g, hipStream_t st) {
  if (p2_supported(g.L) && g.in_kfast == g.out_kfast) {
    switch (g.L) {
      case 32: launch_p2<TI, T, TO, DIR, 32>(g, st); break;
      case 64: launch_p2<TI, T, TO, DIR, 64>(g, st); break;
      case 128: launch_p2<TI, T, TO, DIR, 128>(g, st); break;
      case 256: launch_p2<TI, T, TO, DIR, 256>(g, st); break;
      case 512: launch_p2<TI, T, TO, DIR, 512>(g, st); break;
      default: launch_p2<TI, T, TO, DIR, 1024>(g, st); break;
    }
    LAUNCHCHK();
    return FL_OK;
  }
  int CB = pick_cb(g.L, sizeof(cx<T>));
  size_t lds = fft_lds(g.L, CB, sizeof(cx<T>));
  dim3 grid(nblk(g.B, CB), g.planes);
  allow_lds(k_fft<TI, T, TO, DIR>);
  hipLaunchKernelGGL((k_fft<TI, T, TO, DIR>), grid, dim3(256), lds, st, g, CB);
  LAUNCHCHK();
  return FL_OK;
}

#define RUN(expr)                \
  do {                           \
    fl_status s_ = (expr);       \
    if (s_ != FL_OK) return s_;  \
  } while (0)

FftArgs rows_args(const void* in, void* out, const void* tw, int L, long rows) {
  FftArgs g{};
  g.in = in;
  g.out = out;
  g.tw = tw;
  g.L = L;
  g.lin = L;
  g.lout = L;
  g.in_sk = 1;
  g.in_sb = L;
  g.out_sk = 1;
  g.out_sb = L;
  g.B = (int)rows;
  g.planes = 1;
  g.in_kfast = 1;
  g.out_kfast = 1;
  g.scale = 1.0;
  return g;
}

// columns of planes laid out [plane][L][width] (unit stride across columns)
FftArgs cols_args(const void* in, void* out, const void* tw, int L, int width, int planes) {
  FftArgs g{};
  g.in = in;
  g.out = out;
  g.tw = tw;
  g.L = L;
  g.lin = L;
  g.lout = L;
  g.in_sk = width;
  g.in_sb = 1;
  g.in_sp = (long)L * width;
  g.out_sk = width;
  g.out_sb = 1;
  g.out_sp = (long)L * width;
  g.B = width;
  g.planes = planes;
  g.in_kfast = 0;
  g.out_kfast = 0;
  g.scale = 1.0;
  return g;
}

fl_status build_tables(fl_plan* p) {
  const long N = p->N;
  const int F = p->F;
  for (int f = 0; f < F; ++f) {
    const double om = p->omegas[f];
    const double k0 = om / p->c0;
    const double hz = p->hz;
    const double zeta0 = p->planes[0] - 0.5 * hz - (p->nz - 1) * hz;
    z64* gt = p->gtab + (long)f * p->nzeta * N;
    if (p->opts.kernel_mode == 1) {
      // closed-form transform of G at the torus wavenumbers, times omega^2 h
      hipLaunchKernelGGL(k_gclosed, dim3(nblk(N * p->nzeta, 256)), dim3(256), 0, p->st, gt, p->nzeta,
                         p->px, p->py, p->h, hz, zeta0, p->zt, k0, p->opts.damping, om * om * hz);
      LAUNCHCHK();
    } else {
      // sampled omega^2 h^3 G on every height plane, then FFT2 -> A's entries
      hipLaunchKernelGGL((k_gplanes<double>), dim3(nblk(N * p->nzeta, 256)), dim3(256), 0, p->st, gt,
                         p->nzeta, p->px, p->py, p->h, hz, zeta0, p->zt, k0,
                         om * om * p->h * p->h * hz);
      LAUNCHCHK();
      RUN((run_fft<double, double, double, -1>(
          rows_args(gt, gt, p->tw_x, p->px, (long)p->nzeta * p->py), p->st)));
      RUN((run_fft<double, double, double, -1>(cols_args(gt, gt, p->tw_y, p->py, p->px, p->nzeta),
                                               p->st)));
    }
    // volume kernel on (2nz, py, px), scaled by omega^2 / (2 nz px py): the
    // inverse transforms of the convolution are unnormalized
    const int nz2 = 2 * p->nz;
    z64* kt = p->ktab + (long)f * nz2 * N;
    hipLaunchKernelGGL((k_kappa<double>), dim3(nblk(N * nz2, 256)), dim3(256), 0, p->st, kt, nz2,
                       p->px, p->py, p->h, hz, k0, om * om / ((double)nz2 * (double)N));
    LAUNCHCHK();
    RUN((run_fft<double, double, double, -1>(rows_args(kt, kt, p->tw_x, p->px, (long)nz2 * p->py),
                                             p->st)));
    RUN((run_fft<double, double, double, -1>(cols_args(kt, kt, p->tw_y, p->py, p->px, nz2), p->st)));
    {
      FftArgs g{};
      g.in = kt;
      g.out = kt;
      g.tw = p->tw_z;
      g.L = nz2;
      g.lin = nz2;
      g.lout = nz2;
      g.in_sk = N;
      g.in_sb = 1;
      g.out_sk = N;
      g.out_sb = 1;
      g.B = (int)N;
      g.planes = 1;
      g.scale = 1.0;
      RUN((run_fft<double, double, double, -1>(g, p->st)));
    }
  }
  hipLaunchKernelGGL((k_to_sys<double>), dim3(nblk(N * p->nzeta, 256), F), dim3(256), 0, p->st,
                     p->gtab, p->gsys, p->nzeta, N, p->TP);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(p->st));
  return FL_OK;
}

// Record the start of stage `s` (s < 0: end of the call) when tracing.
fl_status mark(fl_plan* p, int s) {
  if (!p->prof) return FL_OK;
  if (p->ev_used == p->ev_pool.size()) {
    hipEvent_t e;
    HIPCHK(hipEventCreate(&e));
    p->ev_pool.push_back(e);
  }
  hipEvent_t e = p->ev_pool[p->ev_used++];
  HIPCHK(hipEventRecord(e, p->st));
  p->marks.emplace_back(s, e);
  return FL_OK;
}

// Bidiagonalization schedules per system size n: thread grid TR x TC (each
// thread holds an (n/TR) x (n/TC) block of the 2D-cyclic matrix layout) and
// the waves-per-SIMD hint given to the register allocator. Different grids
// sum in different orders, so results agree to rounding, not bitwise.
struct BdVariant {
  int tr, tc, wpe;
};
const std::vector<BdVariant>& bd_variants(int n) {
  static const std::vector<BdVariant> v16{{16, 4, 1}};
  static const std::vector<BdVariant> v32{{16, 8, 1}, {16, 4, 1}, {16, 4, 2}};
  static const std::vector<BdVariant> v48{{16, 8, 2}, {16, 16, 1}, {16, 8, 1}};
  static const std::vector<BdVariant> v64{{16, 8, 2}, {16, 16, 3}, {16, 16, 2}, {16, 8, 1}};
  static const std::vector<BdVariant> v80{{16, 16, 1}, {16, 8, 1}};
  static const std::vector<BdVariant> v96{{16, 16, 1}, {32, 16, 1}, {16, 32, 1}};
  static const std::vector<BdVariant> v128{{16, 32, 1}, {32, 16, 1}};
  static const std::vector<BdVariant> none{};
  switch (n) {
    case 16: return v16;
    case 32: return v32;
    case 48: return v48;
    case 64: return v64;
    case 80: return v80;
    case 96: return v96;
    case 128: return v128;
    default: return none;
  }
}

template <typename T>
fl_status launch_bidiag(fl_plan* p, const int* list, const int* count, int chunk0, int C,
                        BidiagOut& o, const int* resident = nullptr) {
  // one workgroup per slot of the chunk; slots past the active count end at once
  if (C <= 0) return FL_OK;
  const unsigned grid = (unsigned)C;
  const int n = p->n;
  const z64* What = (const z64*)p->What;
  const auto& vs = bd_variants(n);
  if (p->bd_var < 0 || p->bd_var >= (int)vs.size())
    return fail(FL_EUNSUPPORTED, "nz = %d has no solver schedule %d", n, p->bd_var);
  const BdVariant v = vs[p->bd_var];
#define BD(TR, TC, WPE)                                                                     \
  if (v.tr == TR && v.tc == TC && v.wpe == WPE) {                                           \
    hipLaunchKernelGGL((k_bidiag<TR, TC, NN / TR, NN / TC, double, WPE>), dim3(grid), dim3(TR * TC), 0, \
                       p->st, p->gsys, p->TP, What, p->N, list, count, chunk0, C, o, resident, \
                       p->nd, p->nz, (int)p->general);                                         \
    LAUNCHCHK();                                                                            \
    return FL_OK;                                                                           \
  }
  switch (n) {
    case 16: {
      constexpr int NN = 16;
      BD(16, 4, 1)
      break;
    }
    case 32: {
      constexpr int NN = 32;
      BD(16, 8, 1) BD(16, 4, 1) BD(16, 4, 2)
      break;
    }
    case 48: {
      constexpr int NN = 48;
      BD(16, 8, 2) BD(16, 16, 1) BD(16, 8, 1)
      break;
    }
    case 64: {
      constexpr int NN = 64;
      BD(16, 8, 2) BD(16, 16, 3) BD(16, 16, 2) BD(16, 8, 1)
      break;
    }
    case 80: {
      constexpr int NN = 80;
      BD(16, 16, 1) BD(16, 8, 1)
      break;
    }
    case 96: {
      constexpr int NN = 96;
      BD(16, 16, 1) BD(32, 16, 1) BD(16, 32, 1)
      break;
    }
    case 128: {
      constexpr int NN = 128;
      BD(16, 32, 1) BD(32, 16, 1)
      break;
    }
    default:
      break;
  }
#undef BD
  return fail(FL_EUNSUPPORTED, "nz = %d has no solver instance", n);
}

// The frequency weights of the least-squares xi (NULL when xi is per
// frequency).
const double* freq_weights(const fl_plan* p) {
  // always the device array (all ones by default; multiplying by 1 is
  // exact, so the unweighted results are unchanged), so that a captured
  // graph reads the weights set after its capture
  return p->opts.combine == 0 ? p->fw : nullptr;
}

// Classification (with v^ = 0 written for the systems without a solve) and,
// unless the systems are grouped by orbit afterwards, their compaction.
template <typename T>
fl_status solve_prepare(fl_plan* p, bool compact) {
  const long FN = (long)p->F * p->N;
  hipStream_t st = p->st;
  RUN(mark(p, FL_STAGE_CLASSIFY));
  hipLaunchKernelGGL(k_classify<double>, dim3(nblk(FN, 256)), dim3(256), 0, st, (const z64*)p->What,
                     p->nd, p->N, p->F, p->thr2, (int)(p->opts.alpha_rule != 0), freq_weights(p),
                     p->wn2, p->flag, p->Vh, (int)(sizeof(T) == 4), p->nz);
  LAUNCHCHK();
  if (!compact) return FL_OK;
  hipLaunchKernelGGL(k_block_count, dim3(p->nb_scan), dim3(1024), 0, st, p->flag, FN, p->cnt);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, p->cnt, p->nb_scan, p->count, nullptr,
                     nullptr);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scatter, dim3(p->nb_scan), dim3(1024), 0, st, p->flag, FN, p->cnt, p->list);
  LAUNCHCHK();
  return FL_OK;
}

// Bidiagonalization of compacted systems [c0, c0 + C) into the chunk
// workspace (reflectors, bidiagonal, q = U^H w, ||A||_F^2).
template <typename T>
fl_status run_bidiag(fl_plan* p, long c0) {
  BidiagOut o{p->dg, p->sp, p->q, p->fro, p->wnc, p->refl, p->gam, nullptr, nullptr};
  RUN(mark(p, FL_STAGE_BIDIAG));
  return launch_bidiag<T>(p, p->list, p->count, (int)c0, p->C, o);
}

// Systems per wave of the per-system discrepancy kernel
// (fl_tuning.dp_systems_per_wave; 0 = 4 for n <= 64, else 2; 4 is taken as 2
// above n = 64). The orbit-by-orbit search kernel takes the value as given
// (0 = 4).
int dp_spw_of(const fl_plan* p) {
  const int w = p->dp_spw > 0 ? p->dp_spw : (p->n <= 64 ? 4 : 2);
  return (w == 4 && p->n > 64) ? 2 : w;
}

// Discrepancy root, Tikhonov solve and back-transform of the same chunk;
// fixed: take alpha and the branch per frequency from the global search.
template <typename T>
fl_status run_dp(fl_plan* p, long c0, bool fixed = false, bool shared = false) {
  DpArgs a{};
  a.dg = p->dg;
  a.sp = p->sp;
  a.q = p->q;
  a.fro = p->fro;
  a.list = p->list;
  a.count = p->count;
  a.C = p->C;
  a.n = p->n;
  a.nd = p->nd;
  a.nzv = p->nz;
  a.N = p->N;
  a.thr2 = p->thr2;
  a.eta = p->opts.eta;
  a.refl = p->refl;
  a.gam = p->gam;
  a.Vh = p->Vh;
  a.vh_single = sizeof(T) == 4;
  a.alpha = p->alpha;
  a.branch = p->branch;
  a.bd_d = p->bd_d;
  a.bd_e = p->bd_e;
  a.bd_dr = p->bd_dr;
  a.chunk0 = (int)c0;
  a.alpha_fixed = fixed ? p->galpha : nullptr;
  a.branch_fixed = fixed ? p->gbranch : nullptr;
  if (shared) {
    // the active systems grouped by orbit, factorizations by orbit slot: the
    // members of the orbits whose factorizations the workspace holds
    // (orbits [c0, c0 + C) of the compacted list; every orbit when they
    // were factorized at plan creation)
    a.list = p->olist_sys;
    a.C = (int)((long)p->F * p->N);
    a.chunk0 = 0;
    a.oslot = p->oslot;
    a.orep = p->orep;
    a.What = (const z64*)p->What;
    a.refl_l = p->refl_l;
    a.gam_l = p->gam_l;
    // orbits [c0, c0 + C) of the compacted list in slots 0..; with plan-time
    // factorizations every orbit holds its own slot (c0 = 0)
    a.osys0 = p->osys0;
    a.ocount = p->ocount;
    a.slot0 = (int)c0;
    a.OC = p->C;
  }
  const int spw = dp_spw_of(p);
  const long ngr = ((long)a.C + spw - 1) / spw;
  const unsigned gd = (unsigned)std::min<long>(ngr, p->dp_grid > 0 ? p->dp_grid : 16384);
  RUN(mark(p, FL_STAGE_DP));
  if (a.osys0 && !fixed) {
    // orbit by orbit: phase scaling and q' per orbit, the searches per
    // system, the back-transforms per orbit; B' and the right phases per
    // slot in bd_d, bd_e, bd_dr
    a.qy = p->qy;
    const unsigned go = (unsigned)a.OC;
    const int ospw = p->dp_spw > 0 ? p->dp_spw : 4;
    const unsigned gs = (unsigned)std::min<long>(((long)DPO_MEMBERS * a.OC + ospw - 1) / ospw,
                                                 p->dp_grid > 0 ? p->dp_grid : 16384);
#define DPO(NM)                                                                        \
  hipLaunchKernelGGL((k_dpo_prep<NM>), dim3(go), dim3(64), 0, p->st, a);               \
  LAUNCHCHK();                                                                         \
  if (ospw == 4)                                                                       \
    hipLaunchKernelGGL((k_dpo_search<NM, 4>), dim3(gs), dim3(64), 0, p->st, a);        \
  else if (ospw == 2)                                                                  \
    hipLaunchKernelGGL((k_dpo_search<NM, 2>), dim3(gs), dim3(64), 0, p->st, a);        \
  else                                                                                 \
    hipLaunchKernelGGL((k_dpo_search<NM, 1>), dim3(gs), dim3(64), 0, p->st, a);        \
  LAUNCHCHK();                                                                         \
  hipLaunchKernelGGL((k_dpo_back<NM>), dim3(go), dim3(64), 0, p->st, a);               \
  LAUNCHCHK();
    if (p->n <= 64) {
      DPO(64)
    } else {
      DPO(128)
    }
#undef DPO
    return FL_OK;
  }
  if (p->n <= 64) {
    if (spw == 4)
      hipLaunchKernelGGL((k_dp_solve<64, 4>), dim3(gd), dim3(64), 0, p->st, a);
    else if (spw == 2)
      hipLaunchKernelGGL((k_dp_solve<64, 2>), dim3(gd), dim3(64), 0, p->st, a);
    else
      hipLaunchKernelGGL((k_dp_solve<64, 1>), dim3(gd), dim3(64), 0, p->st, a);
  } else {
    if (spw == 2)
      hipLaunchKernelGGL((k_dp_solve<128, 2>), dim3(gd), dim3(64), 0, p->st, a);
    else
      hipLaunchKernelGGL((k_dp_solve<128, 1>), dim3(gd), dim3(64), 0, p->st, a);
  }
  LAUNCHCHK();
  return FL_OK;
}

// Both solver launches for compacted systems [c0, c0 + C); leaves their
// factorization in the chunk workspace.
template <typename T>
fl_status solve_chunk(fl_plan* p, long c0) {
  RUN(run_bidiag<T>(p, c0));
  return run_dp<T>(p, c0);
}

// Rounds of the per-frequency search: first spread, upward probe and the
// multisection rounds of the per-system search.
constexpr int kGlobalRounds = 26;

// One alpha per frequency: factorize every compacted system and keep its
// phase-scaled bidiagonal, search alpha on the summed discrepancy of each
// frequency on the device (a fixed number of rounds; finished frequencies
// skip theirs), then solve every system at its frequency's alpha,
// re-factorizing chunk by chunk when the systems span several chunks.
template <typename T>
fl_status solve_global(fl_plan* p) {
  const long FN = (long)p->F * p->N;
  hipStream_t st = p->st;
  const int F = p->F, n = p->n;
  for (long c0 = 0; c0 < FN; c0 += p->C) {
    RUN(run_bidiag<T>(p, c0));
    GlobalArgs g{p->dg, p->sp, p->q, p->fro, p->list, p->count, (int)c0, p->C, n, p->N,
                 p->gd, p->ge, p->gq, p->gfro, p->gf};
    RUN(mark(p, FL_STAGE_DP));
    const unsigned gp = (unsigned)std::min<long>(p->C, 16384);
    if (n <= 64)
      hipLaunchKernelGGL(k_global_prep<64>, dim3(gp), dim3(64), 0, st, g);
    else
      hipLaunchKernelGGL(k_global_prep<128>, dim3(gp), dim3(64), 0, st, g);
    LAUNCHCHK();
  }
  hipLaunchKernelGGL(k_global_ranges, dim3(std::min<unsigned>(nblk(FN, 256), 1024)), dim3(256), 0,
                     st, p->gf, p->count, F, p->gstart);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_global_init, dim3(F), dim3(64), 0, st, p->gstart, p->gfro, p->wn2, p->list,
                     p->thr2, p->N, p->opts.eta, p->gst, p->galpha, p->gbranch);
  LAUNCHCHK();
  for (int r = 0; r < kGlobalRounds; ++r) {
    if (n <= 64)
      hipLaunchKernelGGL(k_global_eval<64>, dim3(p->gB, F), dim3(64), 0, st, p->gst, p->gstart,
                         p->gd, p->ge, p->gq, n, p->gpart);
    else
      hipLaunchKernelGGL(k_global_eval<128>, dim3(p->gB, F), dim3(64), 0, st, p->gst, p->gstart,
                         p->gd, p->ge, p->gq, n, p->gpart);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_global_update, dim3(F), dim3(64), 0, st, p->gst, p->gpart, p->gB,
                       (int)(r == kGlobalRounds - 1), p->galpha, p->gbranch);
    LAUNCHCHK();
  }
  const bool refactor = FN > p->C;
  for (long c0 = 0; c0 < FN; c0 += p->C) {
    if (refactor) RUN(run_bidiag<T>(p, c0));
    RUN(run_dp<T>(p, c0, true));
  }
  return FL_OK;
}

// Orbits with an active member, compacted in increasing f N + r (olist,
// oslot, ocount; kept as they are when every orbit was factorized at plan
// creation), and the active systems grouped by orbit (olist_sys, count), so
// that the systems sharing a factorization are solved side by side.
fl_status group_by_orbit(fl_plan* p) {
  const long FN = (long)p->F * p->N;
  hipStream_t st = p->st;
  hipLaunchKernelGGL(k_orbit_block_count, dim3(p->nb_scan), dim3(1024), 0, st, p->flag, p->orep,
                     p->omem, p->N, p->oflag, FN, p->cnt, p->ocnt);
  LAUNCHCHK();
  // member offsets (and, unless the orbits were compacted at plan creation,
  // orbit offsets) in one launch
  hipLaunchKernelGGL(k_scan, dim3(p->prefactored ? 1 : 2), dim3(1024), 0, st, p->ocnt, p->nb_scan,
                     p->count, p->prefactored ? nullptr : p->cnt,
                     p->prefactored ? nullptr : p->ocount);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_orbit_scatter, dim3(p->nb_scan), dim3(1024), 0, st, p->oflag, FN, p->omem,
                     p->flag, p->N, p->cnt, p->ocnt, p->prefactored ? nullptr : p->olist,
                     p->prefactored ? nullptr : p->oslot, p->olist_sys,
                     p->prefactored ? nullptr : p->osys0, p->prefactored ? p->opos : nullptr);
  LAUNCHCHK();
  if (p->prefactored) {
    // every orbit holds a slot: the slots' member ranges for the
    // orbit-by-orbit solve
    const int fo = (int)((long)p->F * p->n_orb);
    hipLaunchKernelGGL(k_slot_ranges, dim3(nblk(fo, 256)), dim3(256), 0, st, p->olist, fo, p->opos,
                       p->osys0);
    LAUNCHCHK();
  }
  return FL_OK;
}

// Active orbits of the compacted list that may need a slot (every orbit of
// every frequency), and the orbit chunks that cover them.
long orbit_bound(const fl_plan* p) { return (long)p->F * p->n_orb; }
long orbit_chunks(const fl_plan* p) { return (orbit_bound(p) + p->C - 1) / p->C; }

// Bidiagonalization of the compacted orbit representatives [o0, o0 + C)
// into slots 0.. of the workspace, keeping their left reflectors.
// reuse: skip a chunk that the workspace still holds from the forward solve.
template <typename T>
fl_status run_bidiag_orbits(fl_plan* p, long o0 = 0, bool reuse = false) {
  const long FO = orbit_bound(p);
  const int C = (int)std::min<long>(p->C, FO - o0);
  BidiagOut o{p->dg, p->sp, p->q, p->fro, p->wnc, p->refl, p->gam, p->refl_l, p->gam_l};
  RUN(mark(p, FL_STAGE_BIDIAG));
  RUN(launch_bidiag<T>(p, p->olist, p->ocount, (int)o0, C, o,
                       reuse ? p->oresident : nullptr));
  if (p->prefactored) return FL_OK;
  hipLaunchKernelGGL(k_mark_resident, dim3(1), dim3(1), 0, p->st, p->oresident, p->ocount, (int)o0);
  LAUNCHCHK();
  return FL_OK;
}

// One factorization per active orbit: flag the orbits with an active
// member, compact them, factorize each representative's A keeping its left
// reflectors, then solve every active system against its orbit's
// factorization (q = U^H w from the left reflectors). When the active
// orbits may exceed the workspace, they are taken C at a time (launches
// past the last active orbit find no work and end at once).
template <typename T>
fl_status solve_orbits(fl_plan* p) {
  RUN(group_by_orbit(p));
  hipLaunchKernelGGL(k_mark_resident, dim3(1), dim3(1), 0, p->st, p->oresident, p->ocount, -1);
  LAUNCHCHK();
  for (long o0 = 0; o0 < orbit_bound(p); o0 += p->C) {
    RUN(run_bidiag_orbits<T>(p, o0));
    RUN(run_dp<T>(p, o0, false, true));
  }
  return FL_OK;
}

// Plan-time factorization of every orbit representative of every frequency
// (A_m does not depend on the data): slot f * n_orb + r in the orbit
// workspace, so that fl_invert only classifies and solves.
fl_status prefactor(fl_plan* p, const std::vector<int>& reps) {
  const long N = p->N, F = p->F, FO = F * p->n_orb;
  std::vector<int> list(FO), slot(F * N, 0);
  for (long f = 0; f < F; ++f)
    for (int r = 0; r < p->n_orb; ++r) {
      list[f * p->n_orb + r] = (int)(f * N + reps[r]);
      slot[f * N + reps[r]] = (int)(f * p->n_orb + r);
    }
  const int fo = (int)FO;
  HIPCHK(hipMemcpy(p->olist, list.data(), FO * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->oslot, slot.data(), F * N * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(p->ocount, &fo, sizeof(int), hipMemcpyHostToDevice));
  // the bidiagonalization also transforms the representative's own data
  // column (unused here): give it zeros
  hipLaunchKernelGGL(k_zero<double>, dim3(nblk(F * p->nd * N, 256)), dim3(256), 0, p->st,
                     (z64*)p->What, F * p->nd * N);
  LAUNCHCHK();
  RUN(run_bidiag_orbits<double>(p));
  HIPCHK(hipStreamSynchronize(p->st));
  p->prefactored = true;
  return FL_OK;
}

// The thin-layer solves of the compacted systems, one wave each.
template <typename T>
fl_status run_thin(fl_plan* p) {
  ThinArgs a{};
  a.gsys = p->gsys;
  a.tpitch = p->TP;
  a.What = (const z64*)p->What;
  a.list = p->list;
  a.count = p->count;
  a.nd = p->nd;
  a.nz = p->nz;
  a.N = p->N;
  a.thr2 = p->thr2;
  a.eta = p->opts.eta;
  a.tsvd = p->opts.regularizer == 1;
  a.Vh = p->Vh;
  a.vh_single = sizeof(T) == 4;
  a.alpha = p->alpha;
  a.branch = p->branch;
  const unsigned g = (unsigned)std::min<long>((long)p->F * p->N, 16384);
  RUN(mark(p, FL_STAGE_DP));
  if (p->nz <= 64)
    hipLaunchKernelGGL(k_thin_solve<64>, dim3(g), dim3(64), 0, p->st, a);
  else
    hipLaunchKernelGGL(k_thin_solve<128>, dim3(g), dim3(64), 0, p->st, a);
  LAUNCHCHK();
  return FL_OK;
}

// Truncated SVD of the square systems on the orbits' factorizations, C
// orbits at a time: the bidiagonalization, the SVD of each factorization's
// real bidiagonal, then every member system's truncated solve.
template <typename T>
fl_status solve_tsvd(fl_plan* p) {
  RUN(group_by_orbit(p));
  hipLaunchKernelGGL(k_mark_resident, dim3(1), dim3(1), 0, p->st, p->oresident, p->ocount, -1);
  LAUNCHCHK();
  const long FN = (long)p->F * p->N;
  for (long o0 = 0; o0 < orbit_bound(p); o0 += p->C) {
    RUN(run_bidiag_orbits<T>(p, o0));
    const int C = (int)std::min<long>(p->C, orbit_bound(p) - o0);
    RUN(mark(p, FL_STAGE_DP));
    const unsigned gs = (unsigned)std::min<long>(C, 4096);
    if (p->n <= 64)
      hipLaunchKernelGGL((k_tsvd_svd<64>), dim3(gs), dim3(256), 0, p->st, p->dg, p->sp, p->ocount,
                         (int)o0, C, p->n, p->opts.eta, p->tsv);
    else
      hipLaunchKernelGGL((k_tsvd_svd<128>), dim3(gs), dim3(512), 0, p->st, p->dg, p->sp,
                         p->ocount, (int)o0, C, p->n, p->opts.eta, p->tsv);
    LAUNCHCHK();
    TsvdArgs a{};
    a.What = (const z64*)p->What;
    a.list = p->olist_sys;
    a.count = p->count;
    a.oslot = p->oslot;
    a.orep = p->orep;
    a.refl_l = p->refl_l;
    a.gam_l = p->gam_l;
    a.refl = p->refl;
    a.gam = p->gam;
    a.fro = p->fro;
    a.s = p->tsv;
    a.thr2 = p->thr2;
    a.eta = p->opts.eta;
    a.n = p->n;
    a.nd = p->nd;
    a.nzv = p->nz;
    a.N = p->N;
    a.Vh = p->Vh;
    a.vh_single = sizeof(T) == 4;
    a.alpha = p->alpha;
    a.branch = p->branch;
    a.osys0 = p->osys0;
    a.ocount = p->ocount;
    a.slot0 = (int)o0;
    a.OC = p->C;
    const unsigned gv = (unsigned)std::min<long>(FN, 16384);
    if (p->n <= 64)
      hipLaunchKernelGGL((k_tsvd_solve<64>), dim3(gv), dim3(64), 0, p->st, a);
    else
      hipLaunchKernelGGL((k_tsvd_solve<128>), dim3(gv), dim3(64), 0, p->st, a);
    LAUNCHCHK();
  }
  return FL_OK;
}

// Item 1 with one alpha per wavenumber for the stacked systems of all
// frequencies: the stacked classification, one factorization per active
// orbit (all resident), the active wavenumbers compacted, then one wave per
// wavenumber searches its alpha and solves its frequencies' systems.
template <typename T>
fl_status solve_joint(fl_plan* p) {
  hipStream_t st = p->st;
  const long N = p->N;
  hipLaunchKernelGGL(k_joint_classify, dim3(nblk(N, 256)), dim3(256), 0, st, p->wn2, N, p->F,
                     p->thr2, freq_weights(p), p->flag, p->mflag, p->Vh, (int)(sizeof(T) == 4),
                     p->nz);
  LAUNCHCHK();
  RUN(group_by_orbit(p));
  hipLaunchKernelGGL(k_mark_resident, dim3(1), dim3(1), 0, st, p->oresident, p->ocount, -1);
  LAUNCHCHK();
  RUN(run_bidiag_orbits<T>(p, 0));
  const int nbm = (int)nblk(N, 1024);
  hipLaunchKernelGGL(k_block_count, dim3(nbm), dim3(1024), 0, st, p->mflag, N, p->cnt);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(1024), 0, st, p->cnt, nbm, p->mcount, nullptr, nullptr);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_scatter, dim3(nbm), dim3(1024), 0, st, p->mflag, N, p->cnt, p->mlist);
  LAUNCHCHK();
  JointArgs a{};
  a.mlist = p->mlist;
  a.mcount = p->mcount;
  a.flag = p->flag;
  a.F = p->F;
  a.n = p->n;
  a.nd = p->nd;
  a.nzv = p->nz;
  a.N = N;
  a.thr2 = p->thr2;
  a.eta = p->opts.eta;
  a.oslot = p->oslot;
  a.orep = p->orep;
  a.dg = p->dg;
  a.sp = p->sp;
  a.fro = p->fro;
  a.refl = p->refl;
  a.gam = p->gam;
  a.refl_l = p->refl_l;
  a.gam_l = p->gam_l;
  a.What = (const z64*)p->What;
  a.Vh = p->Vh;
  a.vh_single = sizeof(T) == 4;
  a.alpha = p->alpha;
  a.branch = p->branch;
  RUN(mark(p, FL_STAGE_DP));
  const unsigned g = (unsigned)std::min<long>(N, 16384);
  if (p->n <= 64)
    hipLaunchKernelGGL((k_joint_solve<64>), dim3(g), dim3(64), 0, st, a);
  else
    hipLaunchKernelGGL((k_joint_solve<128>), dim3(g), dim3(64), 0, st, a);
  LAUNCHCHK();
  return FL_OK;
}

// Item 1 for every active system: one factorization per active orbit when
// the plan has them (alpha_rule 0, factor_per_system 0), else per system in
// chunks; the regularizer and alpha rule pick the solver.
template <typename T>
fl_status solve_systems(fl_plan* p) {
  const long FN = (long)p->F * p->N;
  p->last_shared = p->opts.alpha_rule != 1 && p->orbits;
  RUN(solve_prepare<T>(p, !p->last_shared));
  if (p->thin) return run_thin<T>(p);
  if (p->tsvd_sq) return solve_tsvd<T>(p);
  if (p->opts.alpha_rule == 1) return solve_global<T>(p);
  if (p->opts.alpha_rule == 2) return solve_joint<T>(p);
  if (p->last_shared && p->prefactored) {
    RUN(group_by_orbit(p));
    return run_dp<T>(p, 0, false, true);
  }
  if (p->last_shared) return solve_orbits<T>(p);
  for (long c0 = 0; c0 < FN; c0 += p->C) RUN(solve_chunk<T>(p, c0));
  return FL_OK;
}

template <typename T>
struct Tw {
  const cx<T>*x, *y, *z, *ktab;
};

template <typename T>
Tw<T> twiddles_of(fl_plan* p) {
  Tw<T> t;
  t.x = (const cx<T>*)(sizeof(T) == 4 ? (const void*)p->tw_x32 : (const void*)p->tw_x);
  t.y = (const cx<T>*)(sizeof(T) == 4 ? (const void*)p->tw_y32 : (const void*)p->tw_y);
  t.z = (const cx<T>*)(sizeof(T) == 4 ? (const void*)p->tw_z32 : (const void*)p->tw_z);
  t.ktab = (const cx<T>*)(sizeof(T) == 4 ? (const void*)p->ktab32 : (const void*)p->ktab);
  return t;
}

// Columns [F*nz][py][px] in w1 (rows 0..ny-1 significant, zero padded) ->
// FFT along y -> FFT along z, product with the kernel transform (conjugated
// for the adjoint), inverse along z -> inverse along y (rows 0..ny-1) ->
// inverse along x (columns 0..nx-1) + addend -> out [F][nz][ny][nx].
// in_rows: the padded x-transformed rows, [F*nz*ny][px], in w2.
template <typename T>
fl_status conv_tail(fl_plan* p, z64* out, const z64* add, int conj_mul) {
  hipStream_t st = p->st;
  const Tw<T> tw = twiddles_of<T>(p);
  const long N = p->N;
  const int F = p->F, nz = p->nz, nx = p->nx, ny = p->ny, px = p->px, py = p->py;
  FftArgs c = cols_args(p->w2, p->w1, tw.y, py, px, F * nz);
  c.lin = ny;
  c.in_sp = (long)ny * px;
  RUN(mark(p, FL_STAGE_CONV_COLS));
  RUN((run_fft<T, T, T, -1>(c, st)));
  FftArgs z{};
  z.in = p->w1;
  z.out = p->w1;
  z.tw = tw.z;
  z.L = 2 * nz;
  z.lin = nz;
  z.lout = nz;
  z.in_sk = N;
  z.in_sb = 1;
  z.in_sp = (long)nz * N;
  z.out_sk = N;
  z.out_sb = 1;
  z.out_sp = (long)nz * N;
  z.B = (int)N;
  z.planes = F;
  z.scale = 1.0;
  RUN(mark(p, FL_STAGE_CONV_Z));
  if (p2_supported(2 * nz)) {
#define CONVP2(LL)                                                                              \
  hipLaunchKernelGGL((k_fft_conv_p2<T, LL>), dim3(nblk(N, p2_cb<LL, T>()), F),                 \
                     dim3(p2_cb<LL, T>() * (LL / P2<LL>::E)), 0, st, z, tw.ktab, (long)N,       \
                     (long)2 * nz * N, conj_mul)
    switch (2 * nz) {
      case 32: CONVP2(32); break;
      case 64: CONVP2(64); break;
      case 128: CONVP2(128); break;
      case 256: CONVP2(256); break;
      case 512: CONVP2(512); break;
      default: CONVP2(1024); break;
    }
#undef CONVP2
  } else {
    int CBz = pick_cb(2 * nz, sizeof(cx<T>));
    size_t ldsz = fft_lds(2 * nz, CBz, sizeof(cx<T>));
    allow_lds(k_fft_conv<T>);
    hipLaunchKernelGGL(k_fft_conv<T>, dim3(nblk(N, CBz), F), dim3(256), ldsz, st, z, tw.ktab,
                       (long)N, (long)2 * nz * N, CBz, conj_mul);
  }
  LAUNCHCHK();
  FftArgs b = cols_args(p->w1, p->w2, tw.y, py, px, F * nz);
  b.lout = ny;
  b.out_sp = (long)ny * px;
  RUN(mark(p, FL_STAGE_CONV_ICOLS));
  RUN((run_fft<T, T, T, 1>(b, st)));
  FftArgs r = rows_args(p->w2, out, tw.x, px, (long)F * nz * ny);
  r.lout = nx;
  r.out_sb = nx;
  r.add = add;
  RUN(mark(p, FL_STAGE_CONV_IROWS));
  RUN((run_fft<T, T, double, 1>(r, st)));
  return FL_OK;
}

// Stage (c) of the forward map: v = crop(IFFT2(Vin)) / N -> vout, then
// uout = add + omega^2 K v.
template <typename T>
fl_status stage_c(fl_plan* p, const void* Vin, z64* vout, z64* uout, const z64* add) {
  hipStream_t st = p->st;
  const Tw<T> tw = twiddles_of<T>(p);
  const long N = p->N;
  const int F = p->F, nz = p->nz, nx = p->nx, ny = p->ny, px = p->px, py = p->py;
  RUN(mark(p, FL_STAGE_IFFT_COLS));
  FftArgs g = cols_args(Vin, p->w1, tw.y, py, px, F * nz);
  g.lout = ny;
  g.out_off = p->oy;
  g.out_sp = (long)ny * px;
  RUN((run_fft<T, T, T, 1>(g, st)));
  long rows = (long)F * nz * ny;
  RUN(mark(p, FL_STAGE_CROP_PAD));
  if (p2_supported(px)) {
#define CROPP2(LL)                                                                             \
  hipLaunchKernelGGL((k_rows_crop_pad_p2<T, LL>), dim3(nblk(rows, p2_cb<LL, T>())),            \
                     dim3(p2_cb<LL, T>() * (LL / P2<LL>::E)), 0, st, (const cx<T>*)p->w1, vout, \
                     (cx<T>*)p->w2, tw.x, nx, p->ox, (int)rows, 1.0 / (double)N)
    switch (px) {
      case 32: CROPP2(32); break;
      case 64: CROPP2(64); break;
      case 128: CROPP2(128); break;
      case 256: CROPP2(256); break;
      case 512: CROPP2(512); break;
      default: CROPP2(1024); break;
    }
#undef CROPP2
  } else {
    int CB = pick_cb(px, sizeof(cx<T>));
    size_t lds = fft_lds(px, CB, sizeof(cx<T>));
    allow_lds(k_rows_crop_pad<T>);
    hipLaunchKernelGGL(k_rows_crop_pad<T>, dim3(nblk(rows, CB)), dim3(256), lds, st,
                       (const cx<T>*)p->w1, vout, (cx<T>*)p->w2, tw.x, px, nx, p->ox, (int)rows,
                       1.0 / (double)N, CB);
  }
  LAUNCHCHK();
  return conv_tail<T>(p, uout, add, 0);
}

// The inversion launch sequence; T is the FFT / storage precision.
template <typename T>
fl_status invert_impl(fl_plan* p, const void* W, const void* u0, double delta, void* xi_out) {
  hipStream_t st = p->st;
  const long N = p->N;
  const int F = p->F, nd = p->nd, nz = p->nz, nx = p->nx, ny = p->ny, px = p->px, py = p->py;
  const long nvox = (long)nx * ny * nz;
  // noise thresholds thr2[f] = (tau delta ||W_f||)^2: from the sums of
  // squares that the power-of-two row transform of stage (a) leaves per row,
  // else from a pass over W of its own
  const double td = p->opts.tau * delta;
  const bool fused_norm = p2_supported(px);
  if (!fused_norm) {
    RUN(mark(p, FL_STAGE_NORM));
    dim3 g(256, F);
    if (p->opts.input_dtype == 0)
      hipLaunchKernelGGL(k_sumsq<double>, g, dim3(1024), 0, st, (const z64*)W, (long)nd * N, p->partial);
    else
      hipLaunchKernelGGL(k_sumsq<float>, g, dim3(1024), 0, st, (const z32*)W, (long)nd * N, p->partial);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_thresholds, dim3(F), dim3(1024), 0, st, p->partial, 256, F, td * td, p->thr2,
                       p->norm2);
    LAUNCHCHK();
  }
  const z64* u0d = (const z64*)u0;
  if (p->opts.input_dtype == 1) {
    hipLaunchKernelGGL(k_widen<float>, dim3(nblk(F * nvox, 256)), dim3(256), 0, st, (const z32*)u0,
                       p->u0w, (long)F * nvox);
    LAUNCHCHK();
    u0d = p->u0w;
  }
  // (a) FFT2 of W: rows, then columns -> W^ plane-major [F][nd][py][px]
  {
    RUN(mark(p, FL_STAGE_FFT_ROWS));
    // in FP64 in both precisions: the regularized solves amplify the
    // rounding of w^ by their conditioning
    FftArgs g = rows_args(W, p->w1, p->tw_x, px, (long)F * nd * py);
    if (fused_norm) g.rowsq = p->rowsq;
    if (p->opts.input_dtype == 0)
      RUN((run_fft<double, double, double, -1>(g, st)));
    else
      RUN((run_fft<float, double, double, -1>(g, st)));
    if (fused_norm) {
      RUN(mark(p, FL_STAGE_NORM));
      hipLaunchKernelGGL(k_thresholds, dim3(F), dim3(1024), 0, st, p->rowsq, nd * py, F, td * td,
                         p->thr2, p->norm2);
      LAUNCHCHK();
    }
    RUN(mark(p, FL_STAGE_FFT_COLS));
    RUN((run_fft<double, double, double, -1>(cols_args(p->w1, p->What, p->tw_y, py, px, F * nd), st)));
  }
  // (b) regularized solves of the active systems -> v^ plane-major
  RUN(solve_systems<T>(p));
  // (c) v = crop(IFFT2(v^)) / N, then u = u0 + omega^2 K v (zero-padded 3D FFT)
  RUN(stage_c<T>(p, p->Vh, p->vX, p->u, u0d));
  // (d) xi, in FP64
  RUN(mark(p, FL_STAGE_XI));
  hipLaunchKernelGGL(k_xi, dim3(nblk(nvox, 256)), dim3(256), 0, st, p->u, p->vX, nvox, F,
                     p->opts.combine, freq_weights(p), (z64*)xi_out);
  LAUNCHCHK();
  RUN(mark(p, -1));
  return FL_OK;
}

// ------------------------------------------------------------ derivatives

// Layout of the derivative workspaces in one block of bytes: fills b's
// pointers from base (when base is not NULL) and returns the block's size,
// each part aligned to 256 bytes.
size_t adj_layout(const fl_plan* p, char* base, AdjBufs* b) {
  const size_t F = p->F, N = p->N;
  const size_t nvox = (size_t)p->nx * p->ny * p->nz;
  const size_t big = F * std::max(p->nd, p->nz) * N * sizeof(z64);
  const size_t sizes[8] = {F * nvox * sizeof(z64), F * nvox * sizeof(z64), F * nvox * sizeof(z64),
                           F * nvox * sizeof(z64), big, big, F * N * sizeof(double),
                           F * sizeof(double)};
  void** ptrs[8] = {(void**)&b->xi_tmp, (void**)&b->vbar, (void**)&b->ubar, (void**)&b->vbar2,
                    &b->Xb, &b->Yb, (void**)&b->cm, (void**)&b->Tb};
  size_t off = 0;
  for (int i = 0; i < 8; ++i) {
    if (base) *ptrs[i] = base + off;
    off += (sizes[i] + 255) / 256 * 256;
  }
  return off;
}

fl_status ensure_adjoint_buffers(fl_plan* p) {
  if (p->has_adj) return FL_OK;
  void* base = nullptr;
  RUN(dalloc_bytes(p, &base, adj_layout(p, nullptr, &p->adj)));
  adj_layout(p, (char*)base, &p->adj);
  p->has_adj = true;
  return FL_OK;
}

// The derivative calls' own conditions (regularizer, alpha rule, layer).
fl_status adjoint_supported(fl_plan* p) {
  if (p->opts.combine != 0)
    return fail(FL_EUNSUPPORTED, "derivatives are implemented for the least-squares xi (combine 0)");
  if (p->opts.alpha_rule != 0)
    return fail(FL_EUNSUPPORTED, "derivatives are implemented for the per-system alpha (alpha_rule 0)");
  if (p->thin) return fail(FL_EUNSUPPORTED, "derivatives are not implemented for a thin data layer");
  if (p->general)
    return fail(FL_EUNSUPPORTED, "derivatives need data planes on X's lattice with nd = nz");
  if (p->tsvd_sq)
    return fail(FL_EUNSUPPORTED, "derivatives are implemented for Tikhonov (regularizer 0)");
  return FL_OK;
}

fl_status adjoint_preconditions(fl_plan* p) {
  RUN(adjoint_supported(p));
  return ensure_adjoint_buffers(p);
}

AdjArgs adj_args(fl_plan* p) {
  AdjArgs a{};
  a.gsys = p->gsys;
  a.tpitch = p->TP;
  a.list = p->list;
  a.count = p->count;
  a.C = p->C;
  a.n = p->n;
  a.N = p->N;
  a.alpha = p->alpha;
  a.branch = p->branch;
  a.bd_d = p->bd_d;
  a.bd_e = p->bd_e;
  a.bd_dr = p->bd_dr;
  a.refl = p->refl;
  a.gam = p->gam;
  a.What = p->What;
  a.Vh = p->Vh;
  a.single = p->prec;
  a.x_single = p->prec;
  return a;
}

// Per-system derivative pass over every solved system. With shared
// factorizations (the forward factorized one matrix per active orbit) one
// launch takes the orbit-grouped systems and their orbits' slots. Otherwise
// the forward left the factorization of the last chunk in the workspace;
// when the systems span several chunks, each chunk is factorized again
// (same kernels, same results) right before its derivative pass.
template <int MODE, typename T>
fl_status launch_sys_adjoint(fl_plan* p, AdjArgs& a) {
  const long FN = (long)p->F * p->N;
  if (p->last_shared) {
    a.list = p->olist_sys;
    a.count = p->count;
    a.C = (int)FN;
    a.chunk0 = 0;
    a.oslot = p->oslot;
    a.orep = p->orep;
    a.dg = p->dg;
    a.sp = p->sp;
    const unsigned gs = (unsigned)std::min<long>(FN, 16384);
    // with several orbit chunks the forward left the last active one in the
    // workspace: factorize each other chunk again (same kernel, same
    // results) right before its derivative pass
    const long nch = p->prefactored ? 1 : orbit_chunks(p);
    for (long o0 = 0, c = 0; c < nch; o0 += p->C, ++c) {
      if (nch > 1) RUN(run_bidiag_orbits<T>(p, o0, true));
      if (!p->prefactored) {
        a.osys0 = p->osys0;
        a.ocount = p->ocount;
        a.slot0 = (int)o0;
        a.OC = p->C;
      }
      if (p->n <= 64)
        hipLaunchKernelGGL((k_sys_adjoint<64, MODE>), dim3(gs), dim3(64), 0, p->st, a);
      else
        hipLaunchKernelGGL((k_sys_adjoint<128, MODE>), dim3(gs), dim3(64), 0, p->st, a);
      LAUNCHCHK();
    }
    return FL_OK;
  }
  const unsigned g = (unsigned)std::min<long>(p->C, 8192);
  const bool resident = (long)p->C >= FN;
  for (long c0 = 0; c0 < FN; c0 += p->C) {
    if (!resident) RUN(solve_chunk<T>(p, c0));
    a.chunk0 = (int)c0;
    if (p->n <= 64)
      hipLaunchKernelGGL((k_sys_adjoint<64, MODE>), dim3(g), dim3(64), 0, p->st, a);
    else
      hipLaunchKernelGGL((k_sys_adjoint<128, MODE>), dim3(g), dim3(64), 0, p->st, a);
    LAUNCHCHK();
  }
  return FL_OK;
}

template <typename T>
fl_status vjp_impl(fl_plan* p, const AdjBufs& b, const void* W, const void* u0, double delta,
                   const z64* gxi, z64* gW, z64* gu0) {
  hipStream_t st = p->st;
  const long N = p->N;
  const int F = p->F, nd = p->nd, nz = p->nz, nx = p->nx, ny = p->ny, px = p->px, py = p->py;
  const long nvox = (long)nx * ny * nz;
  RUN(invert_impl<T>(p, W, u0, delta, b.xi_tmp));
  const Tw<T> tw = twiddles_of<T>(p);
  // (d) reversed
  hipLaunchKernelGGL(k_xi_vjp, dim3(nblk(nvox, 256)), dim3(256), 0, st, gxi, b.xi_tmp, p->u, p->vX,
                     nvox, F, freq_weights(p), b.vbar, b.ubar);
  LAUNCHCHK();
  // (c) reversed: vbar2 = vbar + K^H ubar, then V^bar = FFT2(pad(vbar2)) / N
  {
    FftArgs r = rows_args(b.ubar, p->w2, tw.x, px, (long)F * nz * ny);
    r.lin = nx;
    r.in_sb = nx;
    RUN((run_fft<double, T, T, -1>(r, st)));
    RUN(conv_tail<T>(p, b.vbar2, b.vbar, 1));
    FftArgs a = rows_args(b.vbar2, p->w1, tw.x, px, (long)F * nz * ny);
    a.lin = nx;
    a.in_sb = nx;
    a.in_off = p->ox;
    RUN((run_fft<double, T, T, -1>(a, st)));
    FftArgs c = cols_args(p->w1, b.Xb, tw.y, py, px, F * nz);
    c.lin = ny;
    c.in_off = p->oy;
    c.in_sp = (long)ny * px;
    c.scale = 1.0 / (double)N;
    RUN((run_fft<T, T, T, -1>(c, st)));
  }
  // (b) reversed, per solved system
  const long FN = (long)F * N;
  hipLaunchKernelGGL(k_zero<double>, dim3(nblk(FN * nd, 256)), dim3(256), 0, st, (z64*)b.Yb, FN * nd);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_zero_real, dim3(nblk(FN, 256)), dim3(256), 0, st, b.cm, FN);
  LAUNCHCHK();
  AdjArgs a = adj_args(p);
  a.X = b.Xb;
  a.Y = b.Yb;
  a.cm = b.cm;
  RUN((launch_sys_adjoint<0, T>(p, a)));
  hipLaunchKernelGGL(k_sum_rows, dim3(F), dim3(1024), 0, st, b.cm, N, b.Tb);
  LAUNCHCHK();
  // (a) reversed: Wbar = N IFFT2(W^bar) + 2 tau^2 delta^2 Tbar_f W_f (FP64)
  {
    FftArgs c = cols_args(b.Yb, p->w1, p->tw_y, py, px, F * nd);
    RUN((run_fft<double, double, double, 1>(c, st)));
    FftArgs r = rows_args(p->w1, gW, p->tw_x, px, (long)F * nd * py);
    RUN((run_fft<double, double, double, 1>(r, st)));
    const double cc = 2.0 * p->opts.tau * p->opts.tau * delta * delta;
    const long per_f = (long)nd * N;
    if (p->opts.input_dtype == 0)
      hipLaunchKernelGGL(k_add_noise_term<double>, dim3(nblk(per_f * F, 256)), dim3(256), 0, st, gW,
                         (const z64*)W, b.Tb, cc, per_f, F);
    else
      hipLaunchKernelGGL(k_add_noise_term<float>, dim3(nblk(per_f * F, 256)), dim3(256), 0, st, gW,
                         (const z32*)W, b.Tb, cc, per_f, F);
    LAUNCHCHK();
  }
  if (gu0) HIPCHK(hipMemcpyAsync(gu0, b.ubar, (size_t)F * nvox * sizeof(z64), hipMemcpyDeviceToDevice, st));
  return FL_OK;
}

template <typename T>
fl_status jvp_impl(fl_plan* p, const void* W, const void* u0, double delta, const void* dW,
                   z64* dxi) {
  hipStream_t st = p->st;
  const long N = p->N;
  const int F = p->F, nd = p->nd, nz = p->nz, nx = p->nx, ny = p->ny, px = p->px, py = p->py;
  const long nvox = (long)nx * ny * nz;
  RUN(invert_impl<T>(p, W, u0, delta, p->adj.xi_tmp));
  // T'_f = 2 tau^2 delta^2 Re <W_f, W'_f>
  {
    dim3 g(256, F);
    if (p->opts.input_dtype == 0)
      hipLaunchKernelGGL(k_dotre<double>, g, dim3(256), 0, st, (const z64*)W, (const z64*)dW,
                         (long)nd * N, p->partial);
    else
      hipLaunchKernelGGL(k_dotre<float>, g, dim3(256), 0, st, (const z32*)W, (const z32*)dW,
                         (long)nd * N, p->partial);
    LAUNCHCHK();
    const double cc = 2.0 * p->opts.tau * p->opts.tau * delta * delta;
    hipLaunchKernelGGL(k_finish_dot, dim3(1), dim3(64), 0, st, p->partial, 256, F, cc, p->adj.Tb);
    LAUNCHCHK();
  }
  // W^' = FFT2(W')
  {
    // FP64 in both precisions, like W^ itself
    FftArgs g = rows_args(dW, p->w1, p->tw_x, px, (long)F * nd * py);
    if (p->opts.input_dtype == 0)
      RUN((run_fft<double, double, double, -1>(g, st)));
    else
      RUN((run_fft<float, double, double, -1>(g, st)));
    RUN((run_fft<double, double, double, -1>(cols_args(p->w1, p->adj.Xb, p->tw_y, py, px, F * nd), st)));
  }
  const long FN = (long)F * N;
  hipLaunchKernelGGL(k_zero<T>, dim3(nblk(FN * nz, 256)), dim3(256), 0, st, (cx<T>*)p->adj.Yb, FN * nz);
  LAUNCHCHK();
  AdjArgs a = adj_args(p);
  a.X = p->adj.Xb;
  a.x_single = 0;
  a.Y = p->adj.Yb;
  a.Tdot = p->adj.Tb;
  RUN((launch_sys_adjoint<1, T>(p, a)));
  // v' and u' = K v' (no incident term), then xi'
  RUN(stage_c<T>(p, p->adj.Yb, p->adj.vbar, p->adj.ubar, nullptr));
  hipLaunchKernelGGL(k_xi_jvp, dim3(nblk(nvox, 256)), dim3(256), 0, st, p->adj.xi_tmp, p->u, p->vX,
                     p->adj.vbar, p->adj.ubar, nvox, F, freq_weights(p), dxi);
  LAUNCHCHK();
  return FL_OK;
}

}  // namespace

namespace {
template <typename T>
fl_status tune_impl(fl_plan* p, int reps, fl_tuning* best) {
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreate(&e0));
  HIPCHK(hipEventCreate(&e1));
  const bool prof = p->prof;
  p->prof = false;
  auto time_it = [&](auto&& launch, float* ms) -> fl_status {
    RUN(launch());  // warm-up
    HIPCHK(hipEventRecord(e0, p->st));
    for (int r = 0; r < reps; ++r) RUN(launch());
    HIPCHK(hipEventRecord(e1, p->st));
    HIPCHK(hipEventSynchronize(e1));
    HIPCHK(hipEventElapsedTime(ms, e0, e1));
    return FL_OK;
  };
  fl_status st = FL_OK;
  float bt = 1e30f;
  const int nv = (int)bd_variants(p->n).size();
  best->bidiag_grid = 0;
  for (int v = 0; v < nv && st == FL_OK; ++v) {
    p->bd_var = v;
    float ms = 0.f;
    st = time_it([&] { return p->last_shared ? run_bidiag_orbits<T>(p) : run_bidiag<T>(p, 0); },
                 &ms);
    if (st != FL_OK) break;
    if (ms < bt) {
      bt = ms;
      best->bidiag_variant = v;
    }
  }
  p->bd_var = best->bidiag_variant;
  p->bd_grid = best->bidiag_grid;
  float dt = 1e30f;
  const int dgrids[] = {2048, 4096, 8192, 16384};
  const int spws[] = {1, 2, 4};
  for (int w : spws) {
    for (int g : dgrids) {
      if (st != FL_OK) break;
      p->dp_grid = g;
      p->dp_spw = w;
      float ms = 0.f;
      st = time_it([&] { return run_dp<T>(p, 0, false, p->last_shared); }, &ms);
      if (st == FL_OK && ms < dt) {
        dt = ms;
        best->dp_grid = g;
        best->dp_systems_per_wave = w;
      }
    }
  }
  p->dp_grid = best->dp_grid;
  p->dp_spw = best->dp_systems_per_wave;
  p->prof = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  return st;
}
// ------------------------------------------------------------ forward solve

// The data operator on X's lattice as a convolution along z: W^[j] =
// sum_l t[j - l + nz - 1] V^[l] is entry j + nz - 1 of the 2nz-point
// circular convolution of the table row t (2nz - 1 entries, zero padded)
// with the zero-extended V^ column, and no entry of that window wraps
// around. The transforms of the table rows, scaled by 1 / (2nz) for the
// unnormalized inverse, are formed by the first call that needs them.
fl_status ensure_toeplitz_transform(fl_plan* p) {
  if (p->ttab) return FL_OK;
  const long N = p->N;
  const int F = p->F, nz2 = 2 * p->nz;
  z64* tt = nullptr;
  ALLOC(tt, (long)F * nz2 * N);
  FftArgs g{};
  g.in = p->gtab;
  g.out = tt;
  g.tw = p->tw_z;
  g.L = nz2;
  g.lin = nz2 - 1;
  g.lout = nz2;
  g.in_sk = N;
  g.in_sb = 1;
  g.in_sp = (long)(nz2 - 1) * N;
  g.out_sk = N;
  g.out_sb = 1;
  g.out_sp = (long)nz2 * N;
  g.B = (int)N;
  g.planes = F;
  g.scale = 1.0 / nz2;
  RUN((run_fft<double, double, double, -1>(g, p->st)));
  p->ttab = tt;
  return FL_OK;
}

fl_status ensure_ls_buffers(fl_plan* p) {
  if (p->has_ls) return FL_OK;
  const long F = p->F, nvox = (long)p->nx * p->ny * p->nz;
  for (auto& b : p->bv) ALLOC(b, F * nvox);
  ALLOC(p->lsw, F * nvox);
  ALLOC(p->dpart, F * 256);
  ALLOC(p->dots, F * 8);
  ALLOC(p->b_rho, F);
  ALLOC(p->b_alpha, F);
  ALLOC(p->b_omega, F);
  ALLOC(p->b_beta, F);
  ALLOC(p->b_bn2, F);
  ALLOC(p->b_active, F);
  p->has_ls = true;
  return FL_OK;
}

// out = y - omega^2 K(xi y), every frequency (K: the zero-padded 3D FFT
// convolution of stage (c), in FP64)
fl_status ls_apply(fl_plan* p, const double* xi, const z64* y, z64* out) {
  const long nvox = (long)p->nx * p->ny * p->nz;
  hipLaunchKernelGGL(k_neg_xi, dim3(nblk(p->F * nvox, 256)), dim3(256), 0, p->st, xi, y, nvox, p->F,
                     p->lsw);
  LAUNCHCHK();
  FftArgs r = rows_args(p->lsw, p->w2, p->tw_x, p->px, (long)p->F * p->nz * p->ny);
  r.lin = p->nx;
  r.in_sb = p->nx;
  RUN((run_fft<double, double, double, -1>(r, p->st)));
  return conv_tail<double>(p, out, y, 0);
}

// dots[slot][f] = <a_f, b_f> = sum conj(a) b
fl_status cdot(fl_plan* p, const z64* a, const z64* b, int slot) {
  const long nvox = (long)p->nx * p->ny * p->nz;
  hipLaunchKernelGGL(k_cdot, dim3(256, p->F), dim3(256), 0, p->st, a, b, nvox, p->dpart);
  LAUNCHCHK();
  hipLaunchKernelGGL(k_cdot_finish, dim3(p->F), dim3(64), 0, p->st, p->dpart, 256, p->F,
                     p->dots + (long)slot * p->F);
  LAUNCHCHK();
  return FL_OK;
}

__global__ void k_bicg_init(BicgScalars S, const z64* __restrict__ bb, int F) {
  const int f = threadIdx.x;
  if (f < F) {
    S.bn2[f] = bb[f].x;
    S.rho[f] = bb[f];
    S.alpha[f] = mk(1.0, 0.0);
    S.omega[f] = mk(1.0, 0.0);
    S.active[f] = bb[f].x > 0.0;
  }
}

// BiCGSTAB from x0 = 0 on u - omega^2 K(xi u) = b; stops each frequency at
// ||s|| or ||r|| <= tol ||b||. Leaves u in bv[0].
// Algorithm 1's fixed point u_{n+1} = u0 + omega^2 K(xi u_n) from u_0 = u0
// (Section 3), every frequency at once; a frequency stops once its change
// ||u_{n+1} - u_n|| is within tol ||u0||. Converges when the spectral radius
// of omega^2 K(xi .) is below one (small omega or contrast).
fl_status ls_fixed_point(fl_plan* p, const double* xi, const z64* b, double tol, int maxit,
                         int* iters) {
  RUN(ensure_ls_buffers(p));
  hipStream_t st = p->st;
  const int F = p->F;
  const long nvox = (long)p->nx * p->ny * p->nz, n = F * nvox;
  z64 *X = p->bv[0], *T = p->bv[1], *Dl = p->bv[2];
  z64* D = p->dots;
  const dim3 g(nblk(n, 256)), blk(256);
  HIPCHK(hipMemcpyAsync(X, b, (size_t)n * sizeof(z64), hipMemcpyDeviceToDevice, st));
  RUN(cdot(p, b, b, 0));
  std::vector<z64> bn2(F), dn2(F);
  std::vector<int> act(F);
  HIPCHK(hipMemcpyAsync(bn2.data(), D, F * sizeof(z64), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  bool any = false;
  for (int f = 0; f < F; ++f) {
    act[f] = bn2[f].x > 0.0;
    any = any || act[f];
  }
  const double tol2 = tol * tol;
  int it = 0;
  while (any && it < maxit) {
    ++it;
    HIPCHK(hipMemcpyAsync(p->b_active, act.data(), F * sizeof(int), hipMemcpyHostToDevice, st));
    RUN(ls_apply(p, xi, X, T));
    hipLaunchKernelGGL(k_fp_step, g, blk, 0, st, b, T, nvox, F, p->b_active, X, Dl);
    LAUNCHCHK();
    RUN(cdot(p, Dl, Dl, 1));
    HIPCHK(hipMemcpyAsync(dn2.data(), D + F, F * sizeof(z64), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    any = false;
    for (int f = 0; f < F; ++f) {
      if (act[f] && dn2[f].x <= tol2 * bn2[f].x) act[f] = 0;
      any = any || act[f];
    }
  }
  *iters = it;
  if (any)
    return fail(FL_ENOCONV, "fixed point: change above %g after %d iterations", tol, maxit);
  return FL_OK;
}

fl_status ls_solve(fl_plan* p, const double* xi, const z64* b, double tol, int maxit, int* iters) {
  RUN(ensure_ls_buffers(p));
  hipStream_t st = p->st;
  const int F = p->F;
  const long nvox = (long)p->nx * p->ny * p->nz, n = F * nvox;
  const size_t bytes = (size_t)n * sizeof(z64);
  z64 *X = p->bv[0], *R = p->bv[1], *Rh = p->bv[2], *P = p->bv[3], *V = p->bv[4], *S = p->bv[5],
      *T = p->bv[6];
  BicgScalars sc{p->b_rho, p->b_alpha, p->b_omega, p->b_beta, p->b_bn2, p->b_active};
  z64* D = p->dots;  // slots: 0 <rh,v>, 1 <s,s>, 2 <t,s>, 3 <t,t>, 4 <r,r>, 5 <rh,r>
  const dim3 g(nblk(n, 256)), blk(256);
  hipLaunchKernelGGL(k_zero<double>, g, blk, 0, st, X, n);
  LAUNCHCHK();
  HIPCHK(hipMemcpyAsync(R, b, bytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(Rh, b, bytes, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(P, b, bytes, hipMemcpyDeviceToDevice, st));
  RUN(cdot(p, b, b, 0));
  hipLaunchKernelGGL(k_bicg_init, dim3(1), dim3(64), 0, st, sc, D, F);
  LAUNCHCHK();
  std::vector<double> bn2(F);
  std::vector<int> act(F);
  std::vector<z64> hd(2 * F);
  HIPCHK(hipMemcpyAsync(bn2.data(), p->b_bn2, F * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(act.data(), p->b_active, F * sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const double tol2 = tol * tol;
  int it = 0;
  bool any = false;
  for (int f = 0; f < F; ++f) any = any || act[f];
  while (any && it < maxit) {
    ++it;
    RUN(ls_apply(p, xi, P, V));
    RUN(cdot(p, Rh, V, 0));
    hipLaunchKernelGGL(k_bicg_alpha, dim3(1), dim3(64), 0, st, sc, D, F);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_bicg_s, g, blk, 0, st, sc, R, V, nvox, F, S);
    LAUNCHCHK();
    RUN(cdot(p, S, S, 1));
    RUN(ls_apply(p, xi, S, T));
    RUN(cdot(p, T, S, 2));
    RUN(cdot(p, T, T, 3));
    hipLaunchKernelGGL(k_bicg_omega, dim3(1), dim3(64), 0, st, sc, D + 2 * F, D + 3 * F, D + F, tol2,
                       F);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_bicg_xr, g, blk, 0, st, sc, P, S, T, nvox, F, X, R);
    LAUNCHCHK();
    RUN(cdot(p, R, R, 4));
    // convergence of each frequency: ||s|| (then x took only the alpha p
    // step) or ||r|| within tol ||b||
    HIPCHK(hipMemcpyAsync(hd.data(), D + F, F * sizeof(z64), hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(hd.data() + F, D + 4 * F, F * sizeof(z64), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    any = false;
    for (int f = 0; f < F; ++f) {
      if (act[f] && (hd[f].x <= tol2 * bn2[f] || hd[F + f].x <= tol2 * bn2[f])) act[f] = 0;
      any = any || act[f];
    }
    HIPCHK(hipMemcpyAsync(p->b_active, act.data(), F * sizeof(int), hipMemcpyHostToDevice, st));
    if (!any) break;
    RUN(cdot(p, Rh, R, 5));
    hipLaunchKernelGGL(k_bicg_beta, dim3(1), dim3(64), 0, st, sc, D + 5 * F, F);
    LAUNCHCHK();
    hipLaunchKernelGGL(k_bicg_p, g, blk, 0, st, sc, R, V, nvox, F, P);
    LAUNCHCHK();
  }
  HIPCHK(hipStreamSynchronize(st));
  *iters = it;
  if (any) return fail(FL_ENOCONV, "BiCGSTAB: no convergence to %g in %d iterations", tol, maxit);
  return FL_OK;
}

}  // namespace

extern "C" {

void fl_opts_default(fl_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof *o);
  o->tau = 1.5;
  o->eta = 1e-10;
}

const char* fl_last_error(void) { return g_err.c_str(); }

fl_status fl_plan_create(int nx, int ny, int nz, int nd, double h, const double* planes,
                         const double* omegas, double c0, int n_omega, const fl_opts* opts,
                         fl_plan** out) {
  g_err.clear();
  if (!out) return fail(FL_EINVAL, "out is NULL");
  *out = nullptr;
  if (nx < 1 || ny < 1 || nz < 1 || nd < 1 || n_omega < 1)
    return fail(FL_EINVAL, "sizes must be >= 1 (nx=%d ny=%d nz=%d nd=%d n_omega=%d)", nx, ny, nz, nd,
                n_omega);
  if (!(h > 0) || !std::isfinite(h)) return fail(FL_EINVAL, "h must be positive and finite");
  if (!(c0 > 0) || !std::isfinite(c0)) return fail(FL_EINVAL, "c0 must be positive and finite");
  if (!planes || !omegas) return fail(FL_EINVAL, "planes and omegas must be host arrays");
  for (int f = 0; f < n_omega; ++f)
    if (!(omegas[f] > 0) || !std::isfinite(omegas[f]))
      return fail(FL_EINVAL, "omegas[%d] = %g must be positive and finite", f, omegas[f]);
  fl_opts o;
  fl_opts_default(&o);
  if (opts) o = *opts;
  if (!(o.tau > 0)) o.tau = 1.5;
  if (!(o.eta > 0)) o.eta = 1e-10;
  const int px = o.px > 0 ? o.px : 2 * nx;
  const int py = o.py > 0 ? o.py : 2 * ny;
  if (px < 2 * nx - 1 || py < 2 * ny - 1)
    return fail(FL_EINVAL, "torus %dx%d too small for window %dx%d (need >= 2n-1)", px, py, nx, ny);
  if (!(o.hz >= 0.0) || !std::isfinite(o.hz)) return fail(FL_EINVAL, "hz must be >= 0 and finite");
  // vertical cell size (0: cubic cells)
  const double hz = o.hz > 0.0 ? o.hz : h;
  const double top = nz * hz;
  bool lattice = true, above = false, below = false;
  for (int j = 0; j < nd; ++j) {
    if (!std::isfinite(planes[j])) return fail(FL_EINVAL, "planes[%d] not finite", j);
    if (planes[j] >= 0.0 && planes[j] <= top)
      return fail(FL_EINVAL, "data plane %d at z=%g lies inside X = [0, %g]", j, planes[j], top);
    lattice = lattice && std::fabs(planes[j] - (planes[0] + j * hz)) <= 1e-9 * hz;
    above = above || planes[j] > top;
    below = below || planes[j] < 0.0;
  }
  if (above && below) return fail(FL_EINVAL, "data planes straddle X");
  // a thin data layer: a few planes at any heights (wide systems)
  // Plane sets: nd = nz planes on X's lattice (square Toeplitz systems, A
  // from one table row of 2 nz - 1 heights) when nz is one of the solver
  // sizes; a thin layer (nd <= THIN_ND <= ... planes at any heights, nd <=
  // nz: wide systems); otherwise a general set: A_m of nd x nz entries from
  // a table of nd nz heights, zero padded to the smallest solver size n >=
  // max(nd, nz).
  static const int kSizes[] = {16, 32, 48, 64, 80, 96, 128};
  auto solver_size = [&](int need) {
    for (int s : kSizes)
      if (s >= need) return s;
    return 0;
  };
  const bool toeplitz = lattice && nd == nz && solver_size(nz) == nz;
  const bool thin = !toeplitz && nd <= THIN_ND && nd <= nz;
  const bool general = !toeplitz && !thin;
  if (general && solver_size(std::max(nd, nz)) == 0)
    return fail(FL_EUNSUPPORTED, "systems of %d data planes x %d X planes: the solver takes at "
                                 "most 128 of each", nd, nz);
  if (!smooth235(px) || !smooth235(py) || !smooth235(2 * nz) || px > 1024 || py > 1024 ||
      2 * nz > 1024)
    return fail(FL_EUNSUPPORTED, "FFT sizes %d, %d, %d need factors 2, 3, 5 only and <= 1024", px,
                py, 2 * nz);
  if (thin && nz > 128) return fail(FL_EUNSUPPORTED, "thin layer: nz = %d > 128", nz);
  if (o.precision != 0 && o.precision != 1) return fail(FL_EUNSUPPORTED, "precision must be 0 or 1");
  if (o.kernel_mode != 0 && o.kernel_mode != 1) return fail(FL_EINVAL, "kernel_mode must be 0 or 1");
  if (!(o.damping >= 0) || !std::isfinite(o.damping)) return fail(FL_EINVAL, "damping must be >= 0");
  if (o.kernel_mode == 1 && o.damping == 0.0) {
    // the closed form is singular where |k_m| = k0 (gamma = 0)
    for (int f = 0; f < n_omega; ++f) {
      const double k0 = omegas[f] / c0;
      for (int my = 0; my < py; ++my)
        for (int mx = 0; mx < px; ++mx) {
          const double sx = mx <= px / 2 ? mx : mx - px, sy = my <= py / 2 ? my : my - py;
          const double kx = 2.0 * M_PI * sx / (px * h), ky = 2.0 * M_PI * sy / (py * h);
          if (std::fabs(k0 * k0 - kx * kx - ky * ky) <= 1e-12 * k0 * k0)
            return fail(FL_ENUMERIC,
                        "closed-form kernel: |k| = k0 at wavenumber (%d, %d) of frequency %d "
                        "(gamma = 0); use damping > 0",
                        mx, my, f);
        }
    }
  }
  if (o.input_dtype != 0 && o.input_dtype != 1) return fail(FL_EINVAL, "input_dtype must be 0 or 1");
  if (o.combine != 0 && o.combine != 1) return fail(FL_EINVAL, "combine must be 0 or 1");
  if (o.alpha_rule < 0 || o.alpha_rule > 2) return fail(FL_EINVAL, "alpha_rule must be 0, 1 or 2");
  if (o.alpha_rule == 2) {
    if (o.factor_per_system || o.prefactor || o.regularizer)
      return fail(FL_EUNSUPPORTED, "alpha_rule 2 needs factor_per_system 0, prefactor 0 and "
                                   "regularizer 0");
    if (n_omega > JOINT_FMAX)
      return fail(FL_EUNSUPPORTED, "alpha_rule 2 stacks at most %d frequencies", JOINT_FMAX);
  }
  if (o.factor_per_system != 0 && o.factor_per_system != 1)
    return fail(FL_EINVAL, "factor_per_system must be 0 or 1");
  if (o.forward_method != 0 && o.forward_method != 1)
    return fail(FL_EINVAL, "forward_method must be 0 or 1");
  if (o.prefactor != 0 && o.prefactor != 1) return fail(FL_EINVAL, "prefactor must be 0 or 1");
  if (o.prefactor && (o.factor_per_system || o.alpha_rule))
    return fail(FL_EUNSUPPORTED, "prefactor needs shared factorizations (factor_per_system 0, "
                                 "alpha_rule 0)");
  if (thin && (o.alpha_rule || o.prefactor))
    return fail(FL_EUNSUPPORTED, "thin layer: alpha_rule 1 or 2 and prefactor are not supported");
  if (o.regularizer != 0 && o.regularizer != 1) return fail(FL_EINVAL, "regularizer must be 0 or 1");
  if (o.regularizer == 1 && !thin) {
    if (o.factor_per_system || o.alpha_rule || o.prefactor)
      return fail(FL_EUNSUPPORTED, "TSVD (regularizer 1) of square systems needs shared "
                                   "factorizations per call (factor_per_system 0, alpha_rule 0, "
                                   "prefactor 0)");
  }

  fl_plan* p = new fl_plan();
  if (hipGetDevice(&p->dev) != hipSuccess) {
    delete p;
    return fail(FL_EDEVICE, "no HIP device");
  }
  p->nx = nx;
  p->ny = ny;
  p->nz = nz;
  p->nd = nd;
  p->px = px;
  p->py = py;
  p->F = n_omega;
  p->h = h;
  p->hz = hz;
  p->c0 = c0;
  p->planes.assign(planes, planes + nd);
  p->omegas.assign(omegas, omegas + n_omega);
  p->opts = o;
  p->opts.px = px;
  p->opts.py = py;
  p->st = (hipStream_t)o.stream;
  p->N = (long)px * py;
  p->thin = thin;
  p->general = general;
  p->nzeta = toeplitz ? nd + nz - 1 : nd * nz;
  p->TP = toeplitz ? 2 * nz : nd * nz;
  p->ox = (px - nx) / 2;
  p->oy = (py - ny) / 2;
  p->n = thin ? nd : general ? solver_size(std::max(nd, nz)) : nz;
  p->prec = o.precision;
  auto bail = [&](fl_status s) {
    fl_plan_destroy(p);
    return s;
  };
#define PALLOC(ptr, cnt)                              \
  do {                                                \
    fl_status s_ = dalloc(p, &(ptr), (size_t)(cnt));  \
    if (s_ != FL_OK) return bail(s_);                 \
  } while (0)
  const long N = p->N, F = p->F;
  const long FN = F * N;
  {
    fl_status s;
    if ((s = make_twiddles(p, &p->tw_x, px)) != FL_OK) return bail(s);
    if ((s = make_twiddles(p, &p->tw_y, py)) != FL_OK) return bail(s);
    if ((s = make_twiddles(p, &p->tw_z, 2 * nz)) != FL_OK) return bail(s);
    if (p->prec) {
      if ((s = make_twiddles(p, &p->tw_x32, px)) != FL_OK) return bail(s);
      if ((s = make_twiddles(p, &p->tw_y32, py)) != FL_OK) return bail(s);
      if ((s = make_twiddles(p, &p->tw_z32, 2 * nz)) != FL_OK) return bail(s);
    }
  }
  PALLOC(p->gtab, F * p->nzeta * N);
  if (!toeplitz) {
    // height differences z_j - z'_l, index j nz + l
    std::vector<double> zt((size_t)nd * nz);
    for (int j = 0; j < nd; ++j)
      for (int l = 0; l < nz; ++l) zt[(size_t)j * nz + l] = planes[j] - (l + 0.5) * hz;
    PALLOC(p->zt, nd * nz);
    hipError_t e = hipMemcpy(p->zt, zt.data(), zt.size() * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(fail(FL_EDEVICE, "heights: %s", hipGetErrorString(e)));
  }
  PALLOC(p->gsys, FN * p->TP);
  PALLOC(p->ktab, F * 2 * nz * N);
  const long big = F * std::max(nd, nz) * N;
  const size_t esz = p->prec ? sizeof(z32) : sizeof(z64);
  {
    fl_status s;
    if ((s = dalloc_bytes(p, &p->What, (size_t)(F * nd * N) * sizeof(z64))) != FL_OK) return bail(s);
    if ((s = dalloc_bytes(p, &p->Vh, (size_t)(F * nz * N) * esz)) != FL_OK) return bail(s);
    // the work arrays also serve fl_forward, which runs in FP64
    if ((s = dalloc_bytes(p, &p->w1, (size_t)big * sizeof(z64))) != FL_OK) return bail(s);
    if ((s = dalloc_bytes(p, &p->w2, (size_t)big * sizeof(z64))) != FL_OK) return bail(s);
  }
  if (p->prec) PALLOC(p->ktab32, F * 2 * nz * N);
  const long nvox = (long)nx * ny * nz;
  PALLOC(p->vX, F * nvox);
  PALLOC(p->u, F * nvox);
  PALLOC(p->u0w, F * nvox);
  PALLOC(p->wn2, FN);
  PALLOC(p->flag, FN);
  {
    // v^ is zero for every system without a solve and stays so between
    // calls: k_classify zeroes only the systems that were solved last time
    // and are not now
    hipError_t e = hipMemset(p->flag, 0, (size_t)FN * sizeof(int));
    if (e == hipSuccess) e = hipMemset(p->Vh, 0, (size_t)(F * nz * N) * esz);
    if (e != hipSuccess) return bail(fail(FL_EDEVICE, "plan memset: %s", hipGetErrorString(e)));
  }
  p->nb_scan = (int)nblk(FN, 1024);
  PALLOC(p->cnt, p->nb_scan);
  PALLOC(p->list, FN);
  PALLOC(p->count, 1);
  PALLOC(p->partial, F * 256);
  PALLOC(p->fw, F);
  PALLOC(p->rowsq, (long)F * nd * py);
  PALLOC(p->thr2, F);
  PALLOC(p->norm2, F);
  std::vector<int> reps;  // orbit representatives, increasing
  std::vector<int> orep_h(N), omem_h(N * 8, -1);
  {
    // symmetry orbits of the wavenumber lattice: mx -> -mx, my -> -my, and
    // mx <-> my on a square torus; the sampled kernel is radial, so Ghat and
    // every A_m are invariant under them
    int n_orb = 0;
    for (int my = 0; my < py; ++my)
      for (int mx = 0; mx < px; ++mx) {
        const int m = my * px + mx;
        int img[8], ni = 0;
        auto add = [&](int x, int y) {
          const int v = y * px + x;
          for (int j = 0; j < ni; ++j)
            if (img[j] == v) return;
          img[ni++] = v;
        };
        const int xs[2] = {mx, (px - mx) % px}, ys[2] = {my, (py - my) % py};
        for (int x : xs)
          for (int y : ys) {
            add(x, y);
            if (px == py) add(y, x);
          }
        int r = m;
        for (int j = 0; j < ni; ++j) r = std::min(r, img[j]);
        orep_h[m] = r;
        if (r == m) {
          ++n_orb;
          reps.push_back(m);
          for (int j = 0; j < ni; ++j) omem_h[(long)m * 8 + j] = img[j];
        }
      }
    p->n_orb = n_orb;
  }
  const long FO = F * p->n_orb;
  // Reflector workspace of C systems (per-system factorizations: the packed
  // right reflectors) or C orbit slots (shared factorizations, which also
  // keep the left reflectors: n^2 complex per slot): up to 80 GiB and 40 %
  // of the free device memory, so that every orbit of the 256^2 x 128 grid
  // with seven frequencies (61 GB) has a slot and one launch factorizes them.
  const bool shared = o.factor_per_system == 0 && o.alpha_rule != 1 && !thin;
  const int ns = p->n;  // solver system size (nz, or the padded size of a general set)
  {
    size_t fr = 0, tot = 0;
    long budget = 80L << 30;
    if (hipMemGetInfo(&fr, &tot) == hipSuccess) budget = std::min<long>(budget, (long)(fr / 5 * 2));
    long slot = (long)sizeof(z64) * (tri_size(ns, 1) + (shared ? tri_size(ns, 0) : 0));
    // the orbit-batched solve keeps q' and then D_R y of up to eight members
    if (shared) slot += (long)sizeof(z64) * DPO_MEMBERS * ns;
    // the truncated SVD keeps both singular vector sets of every slot
    if (o.regularizer == 1 && !thin) slot += 2L * ns * ns * (long)sizeof(double);
    long cap = std::max<long>(1024, budget / slot);
    if (o.max_chunk > 0) cap = std::min<long>(cap, o.max_chunk);
    // the thin solver needs no workspace
    p->C = thin ? 1 : (int)std::min<long>(shared ? FO : FN, cap);
  }
  const long C = p->C;
  PALLOC(p->dg, C * ns);
  PALLOC(p->sp, C * ns);
  PALLOC(p->q, C * ns);
  PALLOC(p->fro, C);
  PALLOC(p->wnc, C);
  PALLOC(p->refl, C * tri_size(ns, 1));
  PALLOC(p->gam, C * ns);
  PALLOC(p->bd_d, C * ns);
  PALLOC(p->bd_e, C * ns);
  PALLOC(p->bd_dr, C * ns);
  PALLOC(p->alpha, FN);
  PALLOC(p->branch, FN);
  if (o.alpha_rule == 1) {
    p->gB = (int)std::min<long>(2048, N);
    PALLOC(p->gd, FN * ns);
    PALLOC(p->ge, FN * ns);
    PALLOC(p->gq, FN * ns);
    PALLOC(p->gfro, FN);
    PALLOC(p->gf, FN);
    PALLOC(p->gstart, F + 1);
    PALLOC(p->gst, F);
    PALLOC(p->galpha, F);
    PALLOC(p->gbranch, F);
    PALLOC(p->gpart, (long)F * p->gB * 64);
  }
  {
    p->orbits = shared;
    if (o.prefactor && FO > C)
      return bail(fail(FL_EUNSUPPORTED,
                       "prefactor needs a workspace of all %ld orbits (max_chunk)", FO));
    if (o.alpha_rule == 2 && FO > C)
      return bail(fail(FL_EUNSUPPORTED,
                       "alpha_rule 2 needs a workspace of all %ld orbits (max_chunk)", FO));
    if (o.alpha_rule == 2) {
      PALLOC(p->mflag, N);
      PALLOC(p->mlist, N);
      PALLOC(p->mcount, 1);
    }
    if (p->orbits) {
      PALLOC(p->orep, N);
      PALLOC(p->omem, N * 8);
      PALLOC(p->oflag, FN);
      PALLOC(p->olist, FO);
      PALLOC(p->ocount, 1);
      PALLOC(p->oslot, FN);
      PALLOC(p->ocnt, p->nb_scan);
      PALLOC(p->olist_sys, FN);
      PALLOC(p->osys0, FO + 1);
      PALLOC(p->oresident, 1);
      PALLOC(p->refl_l, C * tri_size(ns, 0));
      PALLOC(p->gam_l, C * ns);
      PALLOC(p->qy, std::min<long>(DPO_MEMBERS * C, FN) * ns);
      if (o.prefactor) PALLOC(p->opos, FN + 1);
      hipError_t e = hipMemcpy(p->orep, orep_h.data(), N * sizeof(int), hipMemcpyHostToDevice);
      if (e == hipSuccess)
        e = hipMemcpy(p->omem, omem_h.data(), N * 8 * sizeof(int), hipMemcpyHostToDevice);
      if (e != hipSuccess) return bail(fail(FL_EDEVICE, "orbit tables: %s", hipGetErrorString(e)));
    }
    if (o.regularizer == 1 && !thin) {
      p->tsvd_sq = true;
      PALLOC(p->tsv.sig, C * ns);
      PALLOC(p->tsv.P, C * ns * ns);
      PALLOC(p->tsv.Qc, C * ns * ns);
      PALLOC(p->tsv.cdl, C * ns);
      PALLOC(p->tsv.dr, C * ns);
    }
  }
#undef PALLOC
  fl_status s = build_tables(p);
  if (s != FL_OK) return bail(s);
  if (p->prec) {
    const long nk = F * 2 * nz * N;
    hipLaunchKernelGGL(k_narrow, dim3(nblk(nk, 256)), dim3(256), 0, p->st, p->ktab, p->ktab32, nk);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = hipStreamSynchronize(p->st);
    if (e != hipSuccess) return bail(fail(FL_EDEVICE, "table narrowing: %s", hipGetErrorString(e)));
  }
  if (o.prefactor) {
    s = prefactor(p, reps);
    if (s != FL_OK) return bail(s);
  }
  p->fw_host.assign(F, 1.0);
  {
    hipError_t e = hipMemcpy(p->fw, p->fw_host.data(), F * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(fail(FL_EDEVICE, "weights: %s", hipGetErrorString(e)));
  }
  *out = p;
  return FL_OK;
}

fl_status fl_profile_enable(fl_plan* p, int on) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  p->prof = on != 0;
  return FL_OK;
}

fl_status fl_profile_read(fl_plan* p, double* ms, int* launches) {
  if (!p || !ms || !launches) return fail(FL_EINVAL, "NULL argument");
  HIPCHK(hipStreamSynchronize(p->st));
  for (int i = 0; i < FL_N_STAGES; ++i) {
    ms[i] = 0.0;
    launches[i] = 0;
  }
  for (size_t i = 0; i + 1 < p->marks.size(); ++i) {
    int s = p->marks[i].first;
    if (s < 0) continue;
    float t = 0.f;
    HIPCHK(hipEventElapsedTime(&t, p->marks[i].second, p->marks[i + 1].second));
    ms[s] += t;
    launches[s] += 1;
  }
  p->marks.clear();
  p->ev_used = 0;
  return FL_OK;
}

struct fl_graph {
  fl_plan* plan;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

fl_status fl_graph_create(fl_plan* p, const void* W, const void* u0, double delta, void* xi_out,
                          fl_graph** out) {
  if (!p || !out) return fail(FL_EINVAL, "NULL argument");
  *out = nullptr;
  if (p->prof) return fail(FL_EINVAL, "disable stage timing before capturing a graph");
  hipStream_t cap;
  HIPCHK(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
  hipStream_t keep = p->st;
  // order the capture after everything already queued on the plan's stream
  HIPCHK(hipStreamSynchronize(keep));
  p->st = cap;
  hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  fl_status s = FL_OK;
  if (e == hipSuccess) {
    s = fl_invert(p, W, u0, delta, xi_out);
  }
  hipGraph_t graph = nullptr;
  hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(cap, &graph) : e;
  p->st = keep;
  (void)hipStreamDestroy(cap);
  if (s != FL_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess || e2 != hipSuccess)
    return fail(FL_EDEVICE, "stream capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
  fl_graph* g = new fl_graph();
  g->plan = p;
  g->graph = graph;
  e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    fl_graph_destroy(g);
    return fail(FL_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = g;
  return FL_OK;
}

fl_status fl_graph_launch(fl_graph* g) {
  if (!g) return fail(FL_EINVAL, "NULL graph");
  HIPCHK(hipGraphLaunch(g->exec, g->plan->st));
  return FL_OK;
}

void fl_graph_destroy(fl_graph* g) {
  if (!g) return;
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  delete g;
}

struct fl_batch {
  std::vector<fl_plan*> plans;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> done;
  hipEvent_t fork = nullptr;
  hipStream_t st = nullptr;
};

fl_status fl_batch_create(fl_plan* const* plans, int n, void* stream, fl_batch** out) {
  if (!plans || n < 1 || !out) return fail(FL_EINVAL, "need at least one plan");
  *out = nullptr;
  for (int i = 0; i < n; ++i)
    if (!plans[i]) return fail(FL_EINVAL, "plan %d is NULL", i);
  fl_batch* b = new fl_batch();
  b->st = (hipStream_t)stream;
  b->plans.assign(plans, plans + n);
  hipError_t e = hipEventCreateWithFlags(&b->fork, hipEventDisableTiming);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    hipStream_t s;
    hipEvent_t ev;
    e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    b->streams.push_back(s);
    e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e != hipSuccess) break;
    b->done.push_back(ev);
  }
  if (e != hipSuccess) {
    fl_batch_destroy(b);
    return fail(FL_EDEVICE, "batch streams: %s", hipGetErrorString(e));
  }
  *out = b;
  return FL_OK;
}

fl_status fl_batch_invert(fl_batch* b, const void* const* W, const void* const* u0,
                          const double* delta, void* const* xi) {
  if (!b || !W || !u0 || !delta || !xi) return fail(FL_EINVAL, "NULL argument");
  const int n = (int)b->plans.size();
  HIPCHK(hipEventRecord(b->fork, b->st));
  fl_status s = FL_OK;
  for (int i = 0; i < n && s == FL_OK; ++i) {
    fl_plan* p = b->plans[i];
    HIPCHK(hipStreamWaitEvent(b->streams[i], b->fork, 0));
    hipStream_t keep = p->st;
    p->st = b->streams[i];
    s = fl_invert(p, W[i], u0[i], delta[i], xi[i]);
    p->st = keep;
    HIPCHK(hipEventRecord(b->done[i], b->streams[i]));
  }
  for (int i = 0; i < (int)b->done.size(); ++i) HIPCHK(hipStreamWaitEvent(b->st, b->done[i], 0));
  return s;
}

void fl_batch_destroy(fl_batch* b) {
  if (!b) return;
  for (hipStream_t s : b->streams) {
    (void)hipStreamSynchronize(s);
    (void)hipStreamDestroy(s);
  }
  for (hipEvent_t e : b->done) (void)hipEventDestroy(e);
  if (b->fork) (void)hipEventDestroy(b->fork);
  delete b;
}

void fl_plan_destroy(fl_plan* p) {
  if (!p) return;
  (void)hipStreamSynchronize(p->st);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  for (void* v : p->allocs) (void)hipFree(v);
  delete p;
}

fl_status fl_plan_info(const fl_plan* p, fl_plan_info_t* info) {
  if (!p || !info) return fail(FL_EINVAL, "NULL argument");
  info->nx = p->nx;
  info->ny = p->ny;
  info->nz = p->nz;
  info->nd = p->nd;
  info->px = p->px;
  info->py = p->py;
  info->n_omega = p->F;
  info->precision = p->opts.precision;
  info->device_bytes = p->bytes;
  info->last_active = p->last_active;
  info->last_factorized = p->last_factorized;
  return FL_OK;
}

fl_status fl_set_frequency_weights(fl_plan* p, const double* w) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  std::vector<double> v(p->F, 1.0);
  if (w) {
    bool any = false;
    for (int f = 0; f < p->F; ++f) {
      if (!(w[f] >= 0.0) || !std::isfinite(w[f]))
        return fail(FL_EINVAL, "weight %d must be finite and >= 0", f);
      any = any || w[f] > 0.0;
      v[f] = w[f];
    }
    if (!any) return fail(FL_EINVAL, "at least one frequency weight must be positive");
  }
  // the previous inversion may still read the weights: wait for it
  HIPCHK(hipStreamSynchronize(p->st));
  p->fw_host = v;
  HIPCHK(hipMemcpy(p->fw, p->fw_host.data(), p->F * sizeof(double), hipMemcpyHostToDevice));
  return FL_OK;
}

fl_status fl_plan_refresh_info(fl_plan* p) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  int c = 0;
  int o = 0;
  HIPCHK(hipMemcpyAsync(&c, p->count, sizeof(int), hipMemcpyDeviceToHost, p->st));
  if (p->last_shared)
    HIPCHK(hipMemcpyAsync(&o, p->ocount, sizeof(int), hipMemcpyDeviceToHost, p->st));
  HIPCHK(hipStreamSynchronize(p->st));
  p->last_active = c;
  p->last_factorized = p->last_shared ? (p->prefactored ? 0 : o) : c;
  return FL_OK;
}

fl_status fl_tuning_get(const fl_plan* p, fl_tuning* t) {
  if (!p || !t) return fail(FL_EINVAL, "NULL argument");
  t->bidiag_variant = p->bd_var;
  t->bidiag_grid = p->bd_grid;
  t->dp_grid = p->dp_grid;
  t->dp_systems_per_wave = p->dp_spw;
  return FL_OK;
}

fl_status fl_tuning_set(fl_plan* p, const fl_tuning* t) {
  if (!p || !t) return fail(FL_EINVAL, "NULL argument");
  const int nv = (int)bd_variants(p->n).size();
  if (t->bidiag_variant < 0 || t->bidiag_variant >= nv)
    return fail(FL_EINVAL, "bidiag_variant %d out of range [0, %d)", t->bidiag_variant, nv);
  if (t->bidiag_grid < 0 || t->dp_grid < 0) return fail(FL_EINVAL, "grid sizes must be >= 0");
  const int w = t->dp_systems_per_wave;
  if (!(w == 0 || w == 1 || w == 2 || w == 4))
    return fail(FL_EINVAL, "dp_systems_per_wave %d: 0, 1, 2 or 4", w);
  p->bd_var = t->bidiag_variant;
  p->bd_grid = t->bidiag_grid;
  p->dp_grid = t->dp_grid;
  p->dp_spw = w;
  return FL_OK;
}

int fl_tuning_variants(const fl_plan* p) { return p ? (int)bd_variants(p->n).size() : 0; }

fl_status fl_tuning_describe(const fl_plan* p, int variant, int* tr, int* tc, int* wps) {
  if (!p || !tr || !tc || !wps) return fail(FL_EINVAL, "NULL argument");
  const auto& vs = bd_variants(p->n);
  if (variant < 0 || variant >= (int)vs.size()) return fail(FL_EINVAL, "variant out of range");
  *tr = vs[variant].tr;
  *tc = vs[variant].tc;
  *wps = vs[variant].wpe;
  return FL_OK;
}


fl_status fl_plan_tune(fl_plan* p, const void* W, const void* u0, double delta, int reps,
                       void* xi_scratch, fl_tuning* chosen) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  if (!W || !u0 || !xi_scratch) return fail(FL_EINVAL, "NULL array argument");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(FL_EINVAL, "delta must be >= 0 and finite");
  if (p->thin) return fail(FL_EUNSUPPORTED, "a thin data layer has no solver schedule to tune");
  if (p->tsvd_sq) return fail(FL_EUNSUPPORTED, "the TSVD solver has no schedule to tune");
  if (p->opts.alpha_rule == 2)
    return fail(FL_EUNSUPPORTED, "the one-alpha-per-wavenumber solver has no schedule to tune");
  if (reps < 1) reps = 1;
  fl_tuning keep{p->bd_var, p->bd_grid, p->dp_grid, p->dp_spw};
  RUN(fl_invert(p, W, u0, delta, xi_scratch));
  fl_tuning best = keep;
  fl_status s = p->prec ? tune_impl<float>(p, reps, &best) : tune_impl<double>(p, reps, &best);
  if (s != FL_OK) {
    p->bd_var = keep.bidiag_variant;
    p->bd_grid = keep.bidiag_grid;
    p->dp_grid = keep.dp_grid;
    p->dp_spw = keep.dp_systems_per_wave;
  }
  // the timing runs overwrote a plan-time factorization: redo it with the
  // schedule kept
  if (p->prefactored) {
    RUN(run_bidiag_orbits<double>(p));
    HIPCHK(hipStreamSynchronize(p->st));
  }
  if (s != FL_OK) return s;
  if (chosen) *chosen = best;
  return FL_OK;
}

fl_status fl_invert(fl_plan* p, const void* W, const void* u0, double delta, void* xi_out) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  if (!W || !u0 || !xi_out) return fail(FL_EINVAL, "NULL array argument");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(FL_EINVAL, "delta must be >= 0 and finite");
  return p->prec ? invert_impl<float>(p, W, u0, delta, xi_out)
                 : invert_impl<double>(p, W, u0, delta, xi_out);
}

}  // extern "C"

namespace {

// Device memory of fl_invert_vjp_noalloc: one array per GPU, which holds it
// until the process ends. In host code `scratch` names a host-side stand-in,
// not device memory: kernels get the device address from
// hipGetSymbolAddress, taken once per device with that device current.
constexpr size_t kScratchBytes = size_t(FL_NOALLOC_SCRATCH_MB) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 256;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of `scratch` on the current device.
fl_status scratch_of_current_device(void** out) {
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FL_EDEVICE, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FL_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FL_OK;
}

}  // namespace

extern "C" {

fl_status fl_invert_vjp_noalloc(fl_plan* p, const void* W, const void* u0, double delta,
                                const void* grad_xi, void* grad_W, void* grad_u0) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  if (!W || !u0 || !grad_xi || !grad_W) return fail(FL_EINVAL, "NULL array argument");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(FL_EINVAL, "delta must be >= 0 and finite");
  RUN(adjoint_supported(p));
  // stage timing would create events
  if (p->prof) return fail(FL_EINVAL, "stage timing is on (fl_profile_enable): it creates events");
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  if (dev != p->dev)
    return fail(FL_EINVAL, "the plan lives on device %d; make it current (device %d is)", p->dev,
                dev);
  AdjBufs b;
  const size_t need = adj_layout(p, nullptr, &b);
  if (need > kScratchBytes)
    return fail(FL_EINVAL,
                "the plan's derivative workspace needs %zu bytes; the allocation-free call has "
                "%zu (FL_NOALLOC_SCRATCH_MB)", need, kScratchBytes);
  void* base = nullptr;
  RUN(scratch_of_current_device(&base));
  adj_layout(p, (char*)base, &b);
  return p->prec ? vjp_impl<float>(p, b, W, u0, delta, (const z64*)grad_xi, (z64*)grad_W,
                                   (z64*)grad_u0)
                 : vjp_impl<double>(p, b, W, u0, delta, (const z64*)grad_xi, (z64*)grad_W,
                                    (z64*)grad_u0);
}

fl_status fl_invert_vjp(fl_plan* p, const void* W, const void* u0, double delta,
                        const void* grad_xi, void* grad_W, void* grad_u0) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  if (!W || !u0 || !grad_xi || !grad_W) return fail(FL_EINVAL, "NULL array argument");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(FL_EINVAL, "delta must be >= 0 and finite");
  RUN(adjoint_preconditions(p));
  return p->prec ? vjp_impl<float>(p, p->adj, W, u0, delta, (const z64*)grad_xi, (z64*)grad_W,
                                   (z64*)grad_u0)
                 : vjp_impl<double>(p, p->adj, W, u0, delta, (const z64*)grad_xi, (z64*)grad_W,
                                    (z64*)grad_u0);
}

fl_status fl_invert_jvp(fl_plan* p, const void* W, const void* u0, double delta, const void* dW,
                        void* dxi) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  if (!W || !u0 || !dW || !dxi) return fail(FL_EINVAL, "NULL array argument");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(FL_EINVAL, "delta must be >= 0 and finite");
  RUN(adjoint_preconditions(p));
  return p->prec ? jvp_impl<float>(p, W, u0, delta, dW, (z64*)dxi)
                 : jvp_impl<double>(p, W, u0, delta, dW, (z64*)dxi);
}

fl_status fl_forward(fl_plan* p, const double* xi, const void* u0, double tol, int maxit,
                     void* W_out) {
  if (!p) return fail(FL_EINVAL, "NULL plan");
  if (!xi || !u0 || !W_out) return fail(FL_EINVAL, "NULL array argument");
  if (maxit < 0) return fail(FL_EINVAL, "maxit must be >= 0");
  if (!(tol >= 0) || !std::isfinite(tol)) return fail(FL_EINVAL, "tol must be >= 0 and finite");
  if (tol == 0) tol = 1e-12;
  hipStream_t st = p->st;
  const long N = p->N;
  const int F = p->F, nd = p->nd, nz = p->nz, px = p->px, py = p->py;
  const long nvox = (long)p->nx * p->ny * nz;
  const z64* u = (const z64*)u0;
  if (p->opts.input_dtype == 1) {
    hipLaunchKernelGGL(k_widen<float>, dim3(nblk(F * nvox, 256)), dim3(256), 0, st, (const z32*)u0,
                       p->u0w, (long)F * nvox);
    LAUNCHCHK();
    u = p->u0w;
  }
  if (maxit > 0) {
    // total field: u - omega^2 K(xi u) = u0 in X (system (2), first line)
    int it = 0;
    if (p->opts.forward_method == 1)
      RUN(ls_fixed_point(p, xi, u, tol, maxit, &it));
    else
      RUN(ls_solve(p, xi, u, tol, maxit, &it));
    u = p->bv[0];
  }
  // W = omega^2 G * (xi u) on the data planes (eq. 3; eq. 7, second line)
  z64* w1 = (z64*)p->w1;
  z64* w2 = (z64*)p->w2;
  hipLaunchKernelGGL(k_zero<double>, dim3(nblk((long)F * nz * N, 256)), dim3(256), 0, st, w1,
                     (long)F * nz * N);
  LAUNCHCHK();
  hipLaunchKernelGGL((k_current<double, double>), dim3(nblk(F * nvox, 256)), dim3(256), 0, st, xi, u,
                     p->nx, p->ny, nz, F, px, py, p->ox, p->oy, w1);
  LAUNCHCHK();
  RUN((run_fft<double, double, double, -1>(rows_args(w1, w1, p->tw_x, px, (long)F * nz * py), st)));
  RUN((run_fft<double, double, double, -1>(cols_args(w1, w1, p->tw_y, py, px, F * nz), st)));
  if (!p->thin && !p->general && p2_supported(2 * nz)) {
    RUN(ensure_toeplitz_transform(p));
    FftArgs z{};
    z.in = w1;
    z.out = w2;
    z.tw = p->tw_z;
    z.L = 2 * nz;
    z.lin = nz;
    z.lout = nz;
    z.out_off = nz - 1;
    z.in_sk = N;
    z.in_sb = 1;
    z.in_sp = (long)nz * N;
    z.out_sk = N;
    z.out_sb = 1;
    z.out_sp = (long)nz * N;
    z.B = (int)N;
    z.planes = F;
    z.scale = 1.0;
#define APPLYP2(LL)                                                                             \
  hipLaunchKernelGGL((k_fft_conv_p2<double, LL, false>), dim3(nblk(N, p2_cb<LL, double>()), F), \
                     dim3(p2_cb<LL, double>() * (LL / P2<LL>::E)), 0, st, z, p->ttab, (long)N,  \
                     (long)2 * nz * N, 0)
    switch (2 * nz) {
      case 32: APPLYP2(32); break;
      case 64: APPLYP2(64); break;
      case 128: APPLYP2(128); break;
      case 256: APPLYP2(256); break;
      case 512: APPLYP2(512); break;
      default: APPLYP2(1024); break;
    }
#undef APPLYP2
  } else if (!p->thin && !p->general && nz % 16 == 0)
    hipLaunchKernelGGL(k_apply_toeplitz<16>, dim3(nblk((long)F * N, 256)), dim3(256), 0, st, p->gtab,
                       w1, nz, N, F, w2);
  else
    hipLaunchKernelGGL(k_apply_systems<double>, dim3(nblk((long)F * N, 256)), dim3(256), 0, st,
                       p->gtab, w1, nd, nz, N, F, (int)(p->thin || p->general), w2);
  LAUNCHCHK();
  FftArgs c = cols_args(w2, w2, p->tw_y, py, px, F * nd);
  RUN((run_fft<double, double, double, 1>(c, st)));
  FftArgs r = rows_args(w2, W_out, p->tw_x, px, (long)F * nd * py);
  r.scale = 1.0 / (double)N;
  RUN((run_fft<double, double, double, 1>(r, st)));
  return FL_OK;
}

fl_status fl_debug_read(fl_plan* p, int tap, void* dst, size_t bytes) {
  if (!p || !dst) return fail(FL_EINVAL, "NULL argument");
  const long N = p->N, F = p->F;
  const long nvox = (long)p->nx * p->ny * p->nz;
  const void* src = nullptr;
  size_t need = 0;
  switch (tap) {
    case FL_TAP_WHAT: src = p->What; need = F * p->nd * N * sizeof(z64); break;
    case FL_TAP_VHAT: src = p->Vh; need = F * p->nz * N * (p->prec ? sizeof(z32) : sizeof(z64)); break;
    case FL_TAP_V: src = p->vX; need = F * nvox * sizeof(z64); break;
    case FL_TAP_U: src = p->u; need = F * nvox * sizeof(z64); break;
    case FL_TAP_ALPHA: src = p->alpha; need = F * N * sizeof(double); break;
    case FL_TAP_BRANCH: src = p->branch; need = F * N; break;
    case FL_TAP_GTAB: src = p->gtab; need = F * p->nzeta * N * sizeof(z64); break;
    case FL_TAP_KTAB: src = p->ktab; need = F * 2 * p->nz * N * sizeof(z64); break;
    default: return fail(FL_EINVAL, "unknown tap %d", tap);
  }
  if (bytes != need) return fail(FL_EINVAL, "tap %d needs %zu bytes, got %zu", tap, need, bytes);
  HIPCHK(hipStreamSynchronize(p->st));
  if (tap == FL_TAP_ALPHA || tap == FL_TAP_BRANCH) {
    // entries of systems that were not solved keep their zero-branch values
    int c = 0;
    HIPCHK(hipMemcpy(&c, p->count, sizeof(int), hipMemcpyDeviceToHost));
    std::vector<int> flag(F * N);
    HIPCHK(hipMemcpy(flag.data(), p->flag, F * N * sizeof(int), hipMemcpyDeviceToHost));
    if (tap == FL_TAP_ALPHA) {
      std::vector<double> a(F * N);
      HIPCHK(hipMemcpy(a.data(), p->alpha, need, hipMemcpyDeviceToHost));
      for (long i = 0; i < F * N; ++i)
        if (!flag[i]) a[i] = INFINITY;
      std::memcpy(dst, a.data(), need);
    } else {
      std::vector<signed char> b(F * N);
      HIPCHK(hipMemcpy(b.data(), p->branch, need, hipMemcpyDeviceToHost));
      for (long i = 0; i < F * N; ++i)
        if (!flag[i]) b[i] = 0;
      std::memcpy(dst, b.data(), need);
    }
    return FL_OK;
  }
  HIPCHK(hipMemcpy(dst, src, need, hipMemcpyDeviceToHost));
  return FL_OK;
}

}  // extern "C"
