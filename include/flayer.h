/*
 * flayer: flat-layer inversion of the 3D multi-frequency scalar Helmholtz
 * coefficient problem on one AMD MI355X (gfx950).
 *
 * The method is Algorithm 2 of Bakushinsky & Leonov, "To the numerical
 * solution of the inverse multi-frequency scalar acoustics problem"
 * (Section 4, eq. 8 and 9, with the discretization of Section 5.2):
 *
 *   (a) 2D FFT of the scattered field W on every data plane z_j of Y;
 *   (b) for every frequency omega and horizontal wavenumber m, the first-kind
 *       system A_m v_m = w_m with A_m[j][l] = omega^2 h G^(z_j - z'_l, m)
 *       solved by Tikhonov regularization, the parameter chosen per system by
 *       the discrepancy principle (the paper leaves the regularizing
 *       algorithm's parameter rule open; see fl_opts);
 *   (c) inverse FFT of v^ to v on X, then u = u0 + omega^2 G * v in X as a
 *       zero-padded 3D FFT convolution (eq. 4 / 9);
 *   (d) xi = v / u, combined over frequencies by least squares (Section 4,
 *       item 3; Section 5.2).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Geometry: X is the box [0, nx h] x [0, ny h] x [0, nz h] sampled at cell
 *   centres ((i + 1/2) h). The data planes z_j (j < nd) lie outside
 *   [0, nz h], all on one side. Either nd = nz and they are spaced exactly h
 *   apart (z_j = z_0 + j h: z_j - z'_l depends on j - l only and every A_m
 *   is Toeplitz), or nd <= 4 planes at any heights form a thin data
 *   layer (Section 5, second experiment; nd <= nz, every A_m is wide,
 *   nz <= 128). The horizontal plane is a px x py torus (default
 *   2 nx x 2 ny); X's window sits at offset ((px - nx) / 2, (py - ny) / 2).
 * Arrays: complex values are interleaved (re, im), C order, contiguous.
 *   W       [n_omega][nd][py][px]   data on the torus of every data plane
 *   u0      [n_omega][nz][ny][nx]   incident field in X
 *   xi      [nz][ny][nx]            complex128; the physical contrast
 *                                   c0^-2 - c^-2 is its real part
 *   Element type of W and u0: complex128 (input_dtype 0) or complex64 (1).
 * Memory: array arguments of fl_invert / fl_forward / fl_invert_* are DEVICE
 *   pointers owned by the caller; planes and omegas are HOST pointers read
 *   during fl_plan_create only. The plan owns every table and workspace it
 *   allocates and frees them in fl_plan_destroy.
 * Execution: calls are enqueued on opts.stream (a hipStream_t; NULL = the
 *   null stream) and return before the device work ends; outputs are valid
 *   after the stream is synchronized. A plan is not safe for concurrent use.
 * Errors: every call returns an fl_status; nothing throws across the ABI. On
 *   a non-OK status the outputs are untouched unless the status is
 *   FL_EDEVICE, and fl_last_error() (thread-local) explains.
 */
#ifndef FLAYER_H
#define FLAYER_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fl_plan fl_plan;

typedef enum {
  FL_OK = 0,
  FL_EINVAL = 1,       /* an argument is out of range or inconsistent */
  FL_ENOMEM = 2,       /* a device allocation failed */
  FL_EDEVICE = 3,      /* a HIP runtime call or kernel launch failed */
  FL_ENOCONV = 4,      /* an iterative solve did not reach its tolerance */
  FL_ENUMERIC = 5,     /* non-finite value met where a finite one is needed */
  FL_EUNSUPPORTED = 6  /* a valid request the library does not implement */
} fl_status;

/* Options. Zero-initialize and call fl_opts_default, then override. */
typedef struct {
  int px, py;          /* horizontal torus; 0 => 2 nx, 2 ny; need px >= 2 nx - 1,
                          py >= 2 ny - 1, and px, py of the form 2^a 3^b 5^c */
  int precision;       /* 0 = FP64 throughout; 1 = mixed: FP32 FFTs and
                          convolution of stage (c), FP64 data transform (a),
                          regularized solve and division */
  double tau;          /* discrepancy factor: ||A v - w|| = tau delta_m; default 1.5 */
  double eta;          /* alpha >= eta ||A_m||_F^2; default 1e-10; also the
                          parameter used for noise-free data (delta = 0) */
  int combine;         /* 0 = least squares over frequencies (default);
                          1 = one xi per frequency: xi_out is [n_omega][nz][ny][nx] */
  int input_dtype;     /* 0 = complex128 W and u0 (default); 1 = complex64 */
  void *stream;        /* hipStream_t for every call on this plan */
  int max_chunk;       /* 0 = library default; otherwise an upper bound on the
                          systems factorized per solver launch (the workspace
                          holds one chunk of n x n reflectors; derivative calls
                          re-factorize chunk by chunk when there are several) */
  int kernel_mode;     /* table of A: 0 = FFT of G sampled on the torus
                          (Section 5, default); 1 = the continuous transform
                          -i exp(i gamma |zeta|) / (2 gamma) at the torus
                          wavenumbers, gamma = sqrt(k0^2 - |k|^2), Im >= 0 */
  double damping;      /* kernel_mode 1 only: k0 -> k0 (1 + i damping), >= 0;
                          with damping = 0 a wavenumber on |k| = k0 gives
                          FL_ENUMERIC (gamma = 0) */
  int alpha_rule;      /* Tikhonov parameter of item 1 (Section 4; Section 5.1
                          gives one noise level for the whole data set):
                          0 = per system: ||A_m v_m - w_m|| = tau delta_m
                          (default); 1 = one alpha per frequency:
                          sum_m ||A_m v_m - w_m||^2 = tau^2 N delta_m^2 over
                          its N systems, alpha >= eta max_m ||A_m||_F^2, v = 0
                          when sum_m ||w_m||^2 <= tau^2 N delta_m^2. Rule 1
                          keeps every phase-scaled bidiagonal (32 nz bytes per
                          system) and has no derivatives (FL_EUNSUPPORTED);
                          2 = item 1 over all frequencies at once (Section 4,
                          comment c): per wavenumber m the frequencies'
                          systems are one block-diagonal system with one
                          alpha_m, sum_f ||A_fm v_f - w_fm||^2 =
                          tau^2 sum_f delta_fm^2, alpha_m >= eta sum_f
                          ||A_fm||_F^2, v = 0 at every frequency when
                          sum_f ||w_fm||^2 <= tau^2 sum_f delta_fm^2; needs
                          n_omega <= 8, shared factorizations with every
                          active orbit in the workspace, regularizer 0; no
                          derivatives */
  int factor_per_system; /* 0 (default): the kernel G is radial, so A_m is the
                          same for wavenumbers related by the torus symmetries
                          (kx -> -kx, ky -> -ky, and kx <-> ky when px = py):
                          fl_invert factorizes each such orbit once (about N/8
                          systems on a square torus) and applies the orbit's
                          left reflectors to every member's data (the
                          derivative calls use the orbit factorizations too);
                          1 = one factorization per system (always so for
                          alpha_rule 1) */
  int forward_method;  /* fl_forward with maxit > 0: 0 = BiCGSTAB (default);
                          1 = Algorithm 1's fixed point u <- u0 + omega^2 K(xi u)
                          from u0, stopped per frequency when the change is
                          within tol ||u0|| (converges for small omega xi only;
                          FL_ENOCONV otherwise) */
  int prefactor;       /* 1: A_m does not depend on the data, so fl_plan_create
                          factorizes every orbit representative of every
                          frequency once (F x about N/8 matrices kept in the
                          plan) and fl_invert only classifies and solves;
                          needs factor_per_system 0 and alpha_rule 0
                          (FL_EUNSUPPORTED otherwise). 0 (default): each
                          fl_invert factorizes the orbits it needs */
  int regularizer;     /* item 1's regularizing algorithm: 0 = Tikhonov with the
                          discrepancy-chosen alpha (default); 1 = truncated
                          SVD (Section 5.2 reports it best): the fewest
                          leading singular triplets with s_i^2 > eta ||A||_F^2
                          whose residual is within tau delta_m; the ALPHA tap
                          then holds that count. For a thin data layer, and
                          for the square (or padded) systems on the per-call
                          orbit factorizations (factor_per_system 0,
                          alpha_rule 0, prefactor 0; FL_EUNSUPPORTED
                          otherwise). No derivatives (fl_invert_vjp / _jvp
                          return FL_EUNSUPPORTED) */
  double hz;           /* vertical cell size of X (Section 5's grids have
                          different horizontal and vertical steps): X's cells
                          are h x h x hz, X = [0, nx h] x [0, ny h] x
                          [0, nz hz], the quadrature weight of eq. (8) is hz
                          and the volume kernel's h^2 hz; data planes hz apart
                          with nd = nz give Toeplitz systems. 0 (default) =
                          h */
} fl_opts;

void fl_opts_default(fl_opts *opts);

/*
 * Build a plan: validate the geometry, build the per-frequency tables
 * (the FFT of G sampled on the torus at every height difference: Section 5
 * obtains the discrete transform of G from its sampled values by the FFT;
 * and the 3D FFT of the in-X volume kernel with the self-cell integral of G
 * over the ball of volume h^3), and allocate workspaces.
 *   nx, ny, nz   X grid (>= 1); nd data planes (nd = nz on X's lattice, or
 *                a thin layer of nd <= min(4, nz) planes at any heights)
 *   h            cell size (> 0); planes: nd heights (host); omegas: n_omega
 *                angular frequencies (host, > 0); c0 > 0 background speed
 *   opts         NULL => defaults
 *   out          receives the plan (library-owned; free with fl_plan_destroy)
 * Errors: FL_EINVAL (sizes, planes inside X, straddling X, or more than 4
 * planes off the h lattice, torus too small, omega or c0 or h not positive),
 * FL_EUNSUPPORTED (nd != nz beyond a thin layer, torus sizes with prime
 * factors other than 2, 3, 5, or above 1024; a thin layer with alpha_rule 1,
 * prefactor, derivatives or fl_plan_tune), FL_ENOMEM, FL_EDEVICE.
 */
fl_status fl_plan_create(int nx, int ny, int nz, int nd, double h,
                         const double *planes, const double *omegas, double c0,
                         int n_omega, const fl_opts *opts, fl_plan **out);

/*
 * W -> xi (Algorithm 2). delta >= 0 is the relative data error of every
 * frequency, ||W^delta - W|| <= delta ||W|| (Section 5.1); the per-system
 * noise level is delta_m = delta ||W^delta_f||_2 (Parseval). Systems with
 * ||w_m|| <= tau delta_m get v_m = 0; delta = 0 uses alpha = eta ||A_m||_F^2.
 * W, u0, xi_out: device pointers (layouts above). Asynchronous on the plan's
 * stream. Errors: FL_EINVAL (NULL pointers, delta < 0 or not finite),
 * FL_EDEVICE.
 */
fl_status fl_invert(fl_plan *plan, const void *W, const void *u0, double delta,
                    void *xi_out);

/*
 * Reverse derivative (vector-Jacobian product) of xi = invert(W, u0):
 * given the xi cotangent grad_xi ([nz][ny][nx] complex128, the gradient of a
 * real loss as dL/dRe + i dL/dIm), write grad_W ([n_omega][nd][py][px]
 * complex128) and, if grad_u0 is not NULL, grad_u0 ([n_omega][nz][ny][nx]
 * complex128), with <grad_W, dW> = Re sum conj(grad_W) dW the directional
 * derivative. Hand-written adjoint of every stage: the transposed FFTs, the
 * adjoint of the volume convolution, the adjoint Tikhonov solve reusing the
 * forward factorization, the implicit derivative of the discrepancy-chosen
 * alpha (including the dependence of delta_m on ||W||). Runs the forward
 * first (same inputs as fl_invert). Errors: FL_EINVAL, FL_EUNSUPPORTED
 * (combine = 1, alpha_rule = 1), FL_EDEVICE.
 */
fl_status fl_invert_vjp(fl_plan *plan, const void *W, const void *u0, double delta,
                        const void *grad_xi, void *grad_W, void *grad_u0);

/*
 * fl_invert_vjp for callers that cannot allocate device memory at call time
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and results, but the derivative
 * workspaces come from a static device array of the library
 * (FL_NOALLOC_SCRATCH_MB MiB on every GPU the library runs on, held until the
 * process ends) instead of buffers the plan allocates at its first derivative
 * call. Nothing is allocated or freed. The plan's workspace must fit:
 * (4 F nx ny nz + 2 F max(nd, nz) px py) complex128 + F px py doubles, else
 * FL_EINVAL (e.g. 32x32x16 with one frequency needs 3 MiB). The plan's device
 * must be current, and stage timing off (FL_EINVAL otherwise). Every call on
 * one GPU shares that GPU's array and leaves its contents behind (they are
 * rewritten before use): calls that overlap on one GPU, from any plan or
 * stream, race. Other errors as fl_invert_vjp.
 */
#define FL_NOALLOC_SCRATCH_MB 64
fl_status fl_invert_vjp_noalloc(fl_plan *plan, const void *W, const void *u0, double delta,
                                const void *grad_xi, void *grad_W, void *grad_u0);

/*
 * Tangent (Jacobian-vector product): dxi ([nz][ny][nx] complex128) for the
 * data tangent dW (same layout and element type as W), u0 held fixed.
 * Same errors as fl_invert_vjp.
 */
fl_status fl_invert_jvp(fl_plan *plan, const void *W, const void *u0, double delta,
                        const void *dW, void *dxi);

/*
 * Synthetic data (the role of Algorithm 1, Section 3): v = xi u in X, then
 * W = omega^2 G * v on the data planes (eq. 7, second line) over the torus.
 * maxit = 0 takes u = u0 (Born data). maxit > 0 solves the second-kind
 * equation u - omega^2 K(xi u) = u0 in X (system (2), first line; K the
 * zero-padded 3D convolution of stage (c), FP64) by BiCGSTAB from u = 0,
 * every frequency at once, stopping a frequency when its residual is within
 * tol ||u0|| (tol = 0 means 1e-12); FL_ENOCONV if one has not converged
 * after maxit iterations (W_out is then untouched). The Krylov vectors
 * (eight arrays shaped like u0, complex128) are allocated by the first such
 * call and kept by the plan. With the data planes on X's z-lattice and 2 nz
 * a power of two, the first call also forms and keeps the z-transforms of
 * the system table ([n_omega][2 nz][py][px] complex128), with which the
 * data operator runs as a convolution along z.
 *   xi     [nz][ny][nx] real float64, device; u0 as in fl_invert (device)
 *   W_out  [n_omega][nd][py][px] complex128, device
 */
fl_status fl_forward(fl_plan *plan, const double *xi, const void *u0, double tol,
                     int maxit, void *W_out);

/* Read-only facts about a plan. */
typedef struct {
  int nx, ny, nz, nd, px, py, n_omega, precision;
  size_t device_bytes;     /* tables + workspaces held by the plan */
  int last_active;         /* systems solved by the last fl_invert (all
                              frequencies); valid after the stream syncs and
                              a call to fl_plan_refresh_info */
  int last_factorized;     /* matrices A_m it factorized: the active orbits
                              with shared factorizations, else last_active */
} fl_plan_info_t;

fl_status fl_plan_info(const fl_plan *plan, fl_plan_info_t *info);

/*
 * Weights of the frequencies in the least-squares xi of item 3 (Section 5
 * notes that the single-frequency reconstructions differ in accuracy):
 * xi = sum_f w_f conj(u_f) v_f / sum_f w_f |u_f|^2; a frequency of weight 0
 * is not solved at all (frequency selection). w: HOST array of n_omega
 * finite weights >= 0, not all 0, copied; NULL restores all ones. Applies
 * to combine = 0 and to fl_invert_vjp / fl_invert_jvp; synchronizes the
 * plan's stream. The kernels read the weights from device memory at run
 * time, so a graph captured earlier (fl_graph_create) replays with the
 * weights set last. Errors: FL_EINVAL, FL_EDEVICE.
 */
fl_status fl_set_frequency_weights(fl_plan *plan, const double *w);

/* Copy the active-system and factorization counts of the last fl_invert into
 * the info block (synchronizes the plan's stream). */
fl_status fl_plan_refresh_info(fl_plan *plan);

/*
 * Diagnostics: copy an internal array of the last fl_invert (or of the plan's
 * tables) into a HOST buffer of `bytes` bytes; synchronizes the stream.
 *   FL_TAP_WHAT    [n_omega][nd][py][px] complex (FFT of W, unnormalized)
 *   FL_TAP_VHAT    [n_omega][nz][py][px] complex (regularized v^)
 *   FL_TAP_V       [n_omega][nz][ny][nx] complex (v in X)
 *   FL_TAP_U       [n_omega][nz][ny][nx] complex (u in X)
 *   FL_TAP_ALPHA   [n_omega][py][px] float64 (inf where v^ = 0)
 *   FL_TAP_BRANCH  [n_omega][py][px] int8 (0 zero, 1 floor, 2 root)
 *   FL_TAP_GTAB    [n_omega][nd+nz-1][py][px] complex: omega^2 h^3 DFT(G
 *                  sampled at height difference zeta_d), d = j - l + nz - 1
 *   FL_TAP_KTAB    [n_omega][2nz][py][px] complex: omega^2 / (2 nz px py)
 *                  times the 3D DFT of the volume kernel
 * VHAT holds complex64 when precision = 1; every other tap is complex128
 * (the tables are built in FP64; the mixed path keeps an FP32 copy of KTAB).
 * Errors: FL_EINVAL for an unknown tap or a size mismatch.
 */
enum {
  FL_TAP_WHAT = 1, FL_TAP_VHAT = 2, FL_TAP_V = 3, FL_TAP_U = 4,
  FL_TAP_ALPHA = 5, FL_TAP_BRANCH = 6, FL_TAP_GTAB = 7, FL_TAP_KTAB = 8
};
fl_status fl_debug_read(fl_plan *plan, int tap, void *dst_host, size_t bytes);

/*
 * Stage timing (tracing): while enabled, every fl_invert records a HIP event
 * on the plan's stream at the start of each stage and at its end.
 * fl_profile_read synchronizes the stream, returns per-stage sums (ms) and
 * launch counts over all calls since the previous read, and clears them.
 * Stages: */
enum {
  FL_STAGE_NORM = 0,      /* ||W_f||^2 and the per-frequency thresholds */
  FL_STAGE_FFT_ROWS,      /* (a) FFT of W along x */
  FL_STAGE_FFT_COLS,      /* (a) FFT along y */
  FL_STAGE_CLASSIFY,      /* (b) ||w_m||, zero test, compaction, v^ := 0 */
  FL_STAGE_BIDIAG,        /* (b) Householder bidiagonalization */
  FL_STAGE_DP,            /* (b) discrepancy root, bidiagonal Tikhonov solve, v^ = V y */
  FL_STAGE_BACK,          /* (b) reserved (the back-transform is part of FL_STAGE_DP) */
  FL_STAGE_IFFT_COLS,     /* (c) inverse FFT along y, rows of X's window */
  FL_STAGE_CROP_PAD,      /* (c) inverse FFT along x, crop, pad, FFT along x */
  FL_STAGE_CONV_COLS,     /* (c) FFT along y of the padded v */
  FL_STAGE_CONV_Z,        /* (c) FFT along z, kernel product, inverse along z */
  FL_STAGE_CONV_ICOLS,    /* (c) inverse FFT along y */
  FL_STAGE_CONV_IROWS,    /* (c) inverse FFT along x, + u0 */
  FL_STAGE_XI,            /* (d) xi */
  FL_N_STAGES
};
fl_status fl_profile_enable(fl_plan *plan, int on);
fl_status fl_profile_read(fl_plan *plan, double *ms /*[FL_N_STAGES]*/,
                          int *launches /*[FL_N_STAGES]*/);

/*
 * Graph replay: capture the whole launch sequence of
 * fl_invert(plan, W, u0, delta, xi_out) into a HIP graph (no host work and no
 * memset nodes inside), then replay it with fl_graph_launch on the plan's
 * stream. The graph keeps the pointers and delta it was captured with; the
 * caller may change the contents of W and u0 between replays. The plan must
 * outlive the graph. Errors: as fl_invert, plus FL_EDEVICE for capture
 * failures.
 */
typedef struct fl_graph fl_graph;
fl_status fl_graph_create(fl_plan *plan, const void *W, const void *u0, double delta,
                          void *xi_out, fl_graph **out);
fl_status fl_graph_launch(fl_graph *graph);
void fl_graph_destroy(fl_graph *graph);

/*
 * Uneven batch: several independent inversions with different grids (one
 * plan each) issued together. fl_batch_invert forks one stream per plan from
 * `stream` (event waits, so it can itself be graph-captured), runs each
 * instance's fl_invert on its own stream so that their kernels overlap, and
 * joins them back into `stream`. Array i of W, u0, xi and delta[i] belong to
 * plans[i]. The batch borrows the plans; destroy it before them.
 */
typedef struct fl_batch fl_batch;
fl_status fl_batch_create(fl_plan *const *plans, int n, void *stream, fl_batch **out);
fl_status fl_batch_invert(fl_batch *batch, const void *const *W, const void *const *u0,
                          const double *delta, void *const *xi_out);
void fl_batch_destroy(fl_batch *batch);

/*
 * Launch schedule of the per-system solver, and its autotuner (a project-
 * written search over schedules timed on the caller's own data).
 *   bidiag_variant  bidiagonalization schedule, 0 .. fl_tuning_variants() - 1:
 *                   a TR x TC thread grid per system (each thread holds an
 *                   (n/TR) x (n/TC) block of the matrix in registers) and a
 *                   waves-per-SIMD register budget (fl_tuning_describe)
 *   bidiag_grid     unused (kept for the layout): the bidiagonalization
 *                   launches one workgroup per factorization
 *   dp_grid         one-wave workgroups of the discrepancy launch (0 = 16384)
 *   dp_systems_per_wave  systems w one discrepancy wave takes, each in a
 *                   group of 64 / w lanes for the alpha search (64 / w
 *                   points per round) and the Elden solve; 1, 2 or 4. With
 *                   shared orbit factorizations (the default) the
 *                   reflector passes run orbit by orbit and 0 = 4; with
 *                   one factorization per system the groups also apply the
 *                   reflectors, 0 = 4 for nz <= 64, else 2, and 4 counts
 *                   as 2 above nz = 64
 * Schedules sum in different orders, so their results agree to rounding, not
 * bitwise; a plan starts with schedule {0, 0, 0, 0}.
 */
typedef struct {
  int bidiag_variant, bidiag_grid, dp_grid, dp_systems_per_wave;
} fl_tuning;
fl_status fl_tuning_get(const fl_plan *plan, fl_tuning *t);
fl_status fl_tuning_set(fl_plan *plan, const fl_tuning *t); /* FL_EINVAL if out of range */
int fl_tuning_variants(const fl_plan *plan);                 /* 0 for a NULL plan */
fl_status fl_tuning_describe(const fl_plan *plan, int variant, int *tr, int *tc,
                             int *waves_per_simd);
/* Autotune: one fl_invert(plan, W, u0, delta, xi_scratch) to classify the
 * systems, then every schedule candidate timed with HIP events over `reps`
 * solver launches on the first chunk; the fastest is kept in the plan and
 * copied to *chosen (nullable). xi_scratch: device buffer shaped like
 * fl_invert's xi_out (its contents are an inversion result afterwards).
 * Synchronizes the plan's stream. */
fl_status fl_plan_tune(fl_plan *plan, const void *W, const void *u0, double delta, int reps,
                       void *xi_scratch, fl_tuning *chosen);

/* Free a plan and everything it owns (NULL is a no-op). */
void fl_plan_destroy(fl_plan *plan);

/* Message of the last non-OK status on this thread ("" if none). */
const char *fl_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FLAYER_H */
