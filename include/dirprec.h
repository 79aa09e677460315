/*
 * dirprec: directional-preconditioned CFIE solves for 2-D high-frequency
 * obstacle scattering on AMD MI355X (gfx950).
 *
 * Method: L. Ying, "Directional preconditioner for high frequency obstacle
 * scattering".  The problem statement (Sec. 1) is a smooth closed boundary,
 * sampled at n quadrature points with outward normals and weights, a
 * frequency omega, a coupling parameter eta = O(omega), a boundary condition
 * (sound-soft or sound-hard) and incident data; the unknown is the density q
 * of the combined-field integral equation
 *     soft (eq. (1)/(3)):  (1/2 I + D - i eta S) q = -u_I
 *     hard (eq. (2)):      (1/2 I - D' + (1/(i eta)) N) q = -du_I/dn
 * solved by right-preconditioned restarted GMRES (Sec. 3) with the
 * directional preconditioner of Sec. 2.
 *
 * Conventions for every call below
 *   - all sizes are int64_t; complex numbers are interleaved (re, im) pairs
 *     of double; an n x nrhs complex array is column-major (column c starts
 *     at complex offset c*n);
 *   - pointers documented as "device" must point to device memory of the
 *     context's GPU, with the whole array inside one allocation; the library
 *     checks this (hipPointerGetAttributes, hipMemGetAddressRange) before any
 *     kernel runs and returns DP_EINVAL otherwise (also when an operation's
 *     input and output overlap); it reads/writes them on the context stream
 *     and returns after that work has completed (every call is synchronous);
 *   - "host" pointers are read/written before the call returns;
 *   - the caller owns every buffer it passes; the library copies what it
 *     keeps and frees its own allocations in the matching destroy call.  Its
 *     device memory is stream-ordered (hipMallocAsync / hipFreeAsync on the
 *     context stream, kept in the device's memory pool), so destroying a
 *     problem does not wait for the device; destroy every problem before its
 *     context;
 *   - return value: DP_OK (0) on success, DP_ENOCONV (> 0, a warning) when a
 *     solve stopped before reaching the tolerance, a negative DP_E* code on
 *     error; dp_last_error() then describes it (thread-local string);
 *   - one dp_problem must not be used from two threads at once.
 */
#ifndef DIRPREC_H
#define DIRPREC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dp_ctx dp_ctx;
typedef struct dp_problem dp_problem;

enum {
  DP_OK = 0,
  DP_ENOCONV = 1,     /* solve stopped at max_iters; q holds the last iterate */
  DP_EINVAL = -1,     /* invalid argument (see dp_last_error) */
  DP_ENOMEM = -2,     /* device allocation failed */
  DP_EDEVICE = -3,    /* HIP runtime error */
  DP_ESINGULAR = -4,  /* zero pivot in the LU of floor(W) */
  DP_ESTATE = -5      /* call order violated (e.g. apply before build) */
};

enum { DP_SOFT = 0, DP_HARD = 1 };

/* Single operators for tests (Sec. 1 definitions, Kress-corrected Nystrom
 * matrices): S, D, D', and the arclength derivative D_s of the trigonometric
 * interpolant (used in Maue's form of N). */
enum { DP_OP_S = 2, DP_OP_D = 3, DP_OP_DP = 4, DP_OP_DS = 5 };

/* ------------------------------------------------------------------ context */
/* device: HIP device ordinal.  stream: a hipStream_t to run on (e.g. the
 * caller's current stream) or NULL for a library-owned stream.  Device
 * blocks of 256 MB or more that the context's problems release (Krylov
 * bases, sweep partial sums) stay with the context, up to 16 GB, and are
 * reused by later problems on it; dp_ctx_destroy returns them to the pool.
 * (The contexts of a dp_server keep none: its admission budget counts every
 * request's memory.)  Errors: DP_EINVAL (bad ordinal, out == NULL),
 * DP_EDEVICE. */
int dp_ctx_create(int device, void* stream, dp_ctx** out);
void dp_ctx_destroy(dp_ctx* ctx);
const char* dp_last_error(void);

/* ------------------------------------------------------------------ problem */
/* Boundary samples of Sec. 1 / Sec. 2 (host pointers, copied):
 *   xy    n x 2 row-major node positions, counter-clockwise, equispaced in a
 *         2*pi-periodic parameter t_j = 2*pi*j/n;
 *   nrm   n x 2 row-major outward unit normals;
 *   w     n quadrature weights w_j = (2*pi/n)|x'(t_j)| (trapezoid weights);
 *   kappa n signed curvatures (positive where convex); needed by the
 *         diagonal of D and D'.  May be NULL: the library then computes
 *         kappa = (x' y'' - y' x'') / |x'|^3 from the t-derivatives of the
 *         trigonometric interpolant of the node positions (the same
 *         interpolation as D_s), exact for band-limited curves up to
 *         rounding that grows like n^2 * 1e-16 relative to max|x''|.
 * omega > 0 frequency, eta > 0 coupling (typically omega), kind DP_SOFT or
 * DP_HARD.  The spectral derivative (DP_HARD, kappa == NULL) uses radix-2/4
 * FFTs of length n when n is a power of two, else Bluestein's chirp-z DFT
 * with FFTs of the next power of two >= 2n - 1.  Errors (DP_EINVAL): n odd
 * or n < 16, n > 2^26, or (DP_HARD or kappa == NULL) with n > 2^24 (a power
 * of two) or n > 2^23 (other n), a non-finite entry,
 * |nrm_j| differing from 1 by more than 1e-10, w_j <= 0, omega <= 0,
 * eta <= 0.  The problem keeps device copies of the geometry and the Kress
 * correction table C_k (k = 0..n-1). */
int dp_problem_create(dp_ctx* ctx, int64_t n, const double* xy, const double* nrm,
                      const double* w, const double* kappa, double omega, double eta,
                      int kind, dp_problem** out);
void dp_problem_destroy(dp_problem* p);

/* The curvatures the problem uses (the caller's, or those computed when
 * kappa was NULL).  kappa: host, n doubles, written.  Errors: DP_EINVAL. */
int dp_problem_kappa(const dp_problem* p, double* kappa);

/* Incident plane waves u_I = exp(i omega d_k . x), d_k = (cos a_k, sin a_k)
 * (Sec. 3 uses a_0 = 0).  angles: host, nrhs doubles.  f: device n x nrhs
 * complex output, f = -u_I (soft) or -du_I/dn (hard). */
int dp_rhs_plane_wave(dp_problem* p, int64_t nrhs, const double* angles, double* f);

/* y = A q for the problem's CFIE matrix A (Sec. 1; hard via Maue's identity
 * N = D_s S D_s + omega^2 (nu_1 S nu_1 + nu_2 S nu_2)).  q, y: device n x nrhs
 * complex, must not overlap.  nrhs >= 1. */
int dp_matvec(dp_problem* p, int64_t nrhs, const double* q, double* y);

/* y = A_32 q: the single-precision operator used by the correction solves of
 * DP_PREC_MIXED (FP32 kernel values and matrix-core products, FP64 geometry,
 * phase reduction, small-argument Hankel values, diagonal terms and output).
 * Same arguments as dp_matvec; relative error ~1e-6. */
int dp_matvec_mixed(dp_problem* p, int64_t nrhs, const double* q, double* y);

/* y = OP q for one operator (DP_OP_S, DP_OP_D, DP_OP_DP, DP_OP_DS); device
 * n x nrhs complex arrays.  Exposed for parity tests of the single layers.
 * DP_OP_DS of a sound-soft problem created with given curvatures needs a
 * power-of-two n (the Bluestein tables are built only when a problem needs
 * the derivative); DP_EINVAL otherwise. */
int dp_layer_apply(dp_problem* p, int op, int64_t nrhs, const double* q, double* y);

/* ------------------------------------------------------------------ preconditioner */
typedef struct {
  double m_ell;    /* non-planar leaf length in wavelengths (Sec. 2.1: 2 or 4); default 4 */
  int min_pts;     /* never split a segment below this many points; default 8 */
  int m_c;         /* Chebyshev grid size for e_ij (Sec. 3: 10); default 10 */
  double t_keep;   /* floor(T_i) keeps ~t_keep*|K_i| entries (Sec. 2.2); 0 = all; default 3 */
  int w_solver;    /* factorisation of floor(W): 0 = automatic (dense LU on the device when
                      m (m - 1) > 2 NW or the fill-reducing ordering predicts more than
                      32 NW factor entries, else host sparse LU), 1 = sparse, 2 = dense;
                      default 0 */
  int graphs;      /* 1: after the first dp_precond_apply with a given column count,
                      capture the apply's kernels into a HIP graph and replay it;
                      0: launch them one by one; default 1 */
  int gj_steps;    /* Gauss-Jordan steps per launch in the inversions of the size-class
                      blocks B_s and S_s: 0 = automatic (up to 8, as the panel fits in
                      LDS), k > 0 = at most k (1 = one launch per step); default 0 */
} dp_precond_opts;

typedef struct {
  int64_t m;          /* number of segments */
  int64_t n_classes;  /* distinct segment sizes */
  int64_t NW;         /* dimension of floor(W) = sum_i |K_i| */
  int64_t nnzE;       /* m (m - 1) */
  int64_t nnzW;       /* non-zeros of floor(W) */
  int64_t nnzLU;      /* non-zeros of its sparse LU factors */
  int64_t levels;     /* dependency levels of the two triangular solves (sparse) */
  double t_setup;     /* seconds spent in dp_precond_build */
  int64_t dense_w;    /* 1 when floor(W) was factored densely on the device (nnzLU = NW^2) */
} dp_precond_info;

/* Build the directional preconditioner of Sec. 2 (segments, flat blocks B_j,
 * partial Fourier factors U_i, S_i = U_i^t B_i^{-1} U_i, T_i = S_i^{-1},
 * floor(T_i), rank-1 entries e_ij of eq. (14), floor(W) = E + antidiag(T) and
 * its LU: sparse with minimum-degree ordering on the host, or dense with
 * partial pivoting on the device when the sparse factors would fill in).  opts may be NULL (defaults).  Requires arclength-
 * equispaced nodes (all w_j equal within 1e-12 relative), else DP_EINVAL;
 * DP_ESINGULAR on a zero pivot. */
int dp_precond_build(dp_problem* p, const dp_precond_opts* opts);

/* z = P v: the first block of eq. (19) applied to (v, 0, 0).  Device n x nrhs
 * complex arrays (must not overlap).  DP_ESTATE before dp_precond_build. */
int dp_precond_apply(dp_problem* p, int64_t nrhs, const double* v, double* z);

/* The same apply with single-precision copies of the size-class tables
 * (B^{-1}, U, U^t, floor(T)) and of the sparse factors of floor(W), and
 * single-precision vectors (FP64 in and out; a dense floor(W) is solved in
 * FP64 between conversions): the preconditioner of the correction solves of
 * DP_PREC_MIXED.  Relative difference from dp_precond_apply ~1e-6. */
int dp_precond_apply_mixed(dp_problem* p, int64_t nrhs, const double* v, double* z);

/* dp_precond_apply for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * FP64 apply and the same kernels, with every workspace taken from a device
 * array of 128 MiB that the library holds on each GPU it runs on (set up by
 * dp_ctx_create, resident until the process ends); no allocation, no graph.
 * The workspaces need 16 bytes x nrhs x (2 n + 4 NW), and 2 NW more when
 * floor(W) was factored densely (each rounded up to 256 bytes); beyond
 * 128 MiB the call returns DP_EINVAL and names the size.  v, z: device
 * n x nrhs complex, must not overlap.  All calls on one GPU share that array:
 * calls that overlap in time on one GPU (several threads, contexts or
 * problems) race and must be serialised by the caller.  DP_ESTATE before
 * dp_precond_build. */
int dp_precond_apply_noalloc(dp_problem* p, int64_t nrhs, const double* v, double* z);

int dp_precond_get_info(dp_problem* p, dp_precond_info* info);

/* Structure export for tests (host arrays, caller-allocated):
 * seg_off, seg_len: m entries; e_idx: 4*m*(m-1) entries (i, j, k^i_ij,
 * k^j_ij for each ordered pair, row-major in (i, j)); e_val: 2*m*(m-1)
 * doubles (e_ij).  Any pointer may be NULL. */
int dp_precond_export(dp_problem* p, int64_t* seg_off, int64_t* seg_len, int64_t* e_idx,
                      double* e_val);

/* ------------------------------------------------------------------ solve */
enum { DP_PREC_FP64 = 0, DP_PREC_MIXED = 1 };

typedef struct {
  double tol;       /* relative residual ||f - A q|| / ||f|| per column; default 1e-8 */
  int restart;      /* GMRES restart length; default 80 (Sec. 3) */
  int max_iters;    /* total Arnoldi steps per column; default 2000 */
  int use_precond;  /* 1: right-precondition with the built preconditioner */
  int precision;    /* DP_PREC_FP64, or DP_PREC_MIXED: iterative refinement whose
                       corrections come from GMRES with the single-precision
                       operator (FP32 kernel values and matrix-core products;
                       FP64 geometry, phase reduction, small-argument Hankel
                       values, diagonal terms, Krylov vectors and Givens
                       rotations) preconditioned by dp_precond_apply_mixed,
                       and whose residuals f - A q are FP64 */
  double inner_tol; /* mixed: relative tolerance of the correction solves, at least the one
                       that takes every column from its current FP64 residual r to
                       0.3 tol (0.3 tol/r for the worst column); <= 0: sqrt(tol)
                       within [1e-5, 1e-2] (two corrections share the reduction) */
  int eager;        /* 1: launch the kernels of each Arnoldi step's orthogonalisation
                       and rotation update one by one instead of replaying their
                       captured HIP graph (the same kernels and results); default 0 */
} dp_solve_opts;

typedef struct {
  int64_t iters_max;   /* largest iteration count over the columns */
  int64_t matvecs;     /* operator applications (including true-residual checks) */
  int64_t applies;     /* preconditioner applications */
  double relres_max;   /* largest true relative residual at exit */
  double t_total, t_matvec, t_apply, t_krylov;  /* seconds */
  int64_t sweep_launches;  /* launches of the pair-sweep kernel during the solve */
  double t_sweep;          /* their summed duration (HIP events on the context stream), s */
  int64_t refinements;     /* mixed: outer refinement steps (FP64 residuals) */
  int64_t matvecs_fp32;    /* mixed: operator applications in single precision */
  int64_t sweep_launches_fp32;  /* mixed: launches of the single-precision sweep */
  double t_sweep_fp32;          /* their summed duration, s */
} dp_solve_info;

/* Solve A q = f for nrhs right-hand sides by restarted GMRES (x0 = 0, CGS2
 * Arnoldi, Givens rotations; Sec. 3), right-preconditioned when requested; the
 * preconditioned vectors are stored (flexible form) so q = Z y needs no extra
 * apply.  Each Arnoldi step, its least-squares update and the per-column
 * stopping test run on the device; the host queues step k + 1 while step k
 * runs and reads the column states back one step late, so it does not wait
 * for the device inside a restart cycle except where the residual estimates
 * predict that a step may stop the last columns.  With DP_PREC_MIXED the solve is q_{k+1} = q_k + GMRES_32(f - A q_k)
 * until the FP64 residual meets tol.  f, q: device n x nrhs complex.
 * opts/info may be NULL.  iters, relres: optional host arrays of nrhs entries
 * (per-column iteration counts and true FP64 relative residuals).  The
 * solve's device workspaces (the Krylov basis and its preconditioned copy,
 * (restart + 1) and restart n x nrhs complex arrays, and the refinement
 * vectors) stay allocated with the problem, grown as needed, until
 * dp_problem_destroy, so that repeated solves do not allocate; calls on one
 * problem must not overlap.  Returns DP_OK or DP_ENOCONV. */
int dp_solve(dp_problem* p, int64_t nrhs, const double* f, double* q, const dp_solve_opts* opts,
             dp_solve_info* info, int64_t* iters, double* relres);

/* ------------------------------------------------------------------ autotuning */
typedef struct {
  double t_default_ms;   /* one sweep of nrhs columns with the default launch configuration */
  double t_best_ms;      /* with the chosen configuration */
  int64_t target_blocks; /* grid size the source chunking aims at (1024..8192) */
  int64_t matrix_cores;  /* 1 if the chosen sweep runs on the matrix cores */
  int64_t candidates;    /* configurations timed */
} dp_tune_info;

/* Time the problem's operator sweep (nrhs columns, up to 64, in the given
 * precision: DP_PREC_FP64 or DP_PREC_MIXED) over its candidate launch
 * configurations (grid sizes; for FP64 with 5-16 columns also the VALU kernel
 * against the 16-column matrix-core kernel) and keep the fastest
 * for later calls on this problem with the same column count.  A
 * configuration fixes the order of the partial sums, so results are
 * reproducible once it is chosen; they may differ in the last bits from
 * another configuration's.  info may be NULL. */
int dp_autotune(dp_problem* p, int64_t nrhs, int precision, dp_tune_info* info);

/* ------------------------------------------------------------------ serving */
/* A request server for streams of independent solves (different n, omega,
 * geometries, boundary conditions and right-hand-side counts).  Each request
 * is the whole path of Sec. 1-3: problem set-up, the directional
 * preconditioner of Sec. 2 (optional), plane-wave or given data, and the
 * GMRES solve.  The server owns `slots` worker threads, each with its own
 * context and HIP stream; a free worker admits the oldest queued request once
 * its estimated device-memory footprint fits in the budget next to the
 * requests already running, so requests that arrive while others are on the
 * GPU start as soon as a slot and memory free up and their kernels overlap
 * on the device.  A request's result does not depend on what else runs: it
 * executes the same kernels on its own buffers and stream as it would alone. */
typedef struct dp_server dp_server;

typedef struct {
  int slots;           /* concurrent requests (worker threads); default 4, 1..64 */
  int64_t mem_budget;  /* bytes of device memory the admitted requests may hold by
                          estimate; 0 = 80% of the free memory at creation */
} dp_server_opts;

typedef struct {
  int64_t n;                   /* as dp_problem_create; the host arrays are copied by submit */
  const double *xy, *nrm, *w, *kappa;
  double omega, eta;
  int kind;                    /* DP_SOFT or DP_HARD */
  int64_t nrhs;                /* >= 1 */
  const double* angles;        /* host, nrhs plane-wave angles (dp_rhs_plane_wave), or NULL */
  const double* f;             /* host n x nrhs complex data, used when angles == NULL */
  dp_solve_opts solve;         /* use_precond = 1 builds the preconditioner (default options) */
} dp_request;

typedef struct {
  double t_submit, t_admit, t_done;  /* seconds since dp_server_create */
  int64_t mem_estimate;              /* bytes charged against the budget while running */
  int slot;                          /* worker that ran it */
} dp_request_times;

typedef struct {
  int64_t submitted, completed, failed, running, queued;
  int64_t mem_in_use, mem_budget, mem_peak;  /* bytes, by estimate */
} dp_server_stats;

/* opts may be NULL.  Errors: DP_EINVAL (bad device or options), DP_EDEVICE. */
int dp_server_create(int device, const dp_server_opts* opts, dp_server** out);
/* Queue a request (returns at once) and give its id.  The request is
 * validated as dp_problem_create would; DP_ENOMEM if its estimated footprint
 * exceeds the whole budget (it could never be admitted). */
int dp_server_submit(dp_server* s, const dp_request* r, int64_t* id);
/* Block until request id has finished; copy its solution (host n x nrhs
 * complex, may be NULL), solve info and times (may be NULL), and forget the
 * request.  Returns the request's own status (DP_OK, DP_ENOCONV, or the
 * negative error of the step that failed, described by dp_last_error in the
 * calling thread); DP_EINVAL for an unknown id. */
int dp_server_wait(dp_server* s, int64_t id, double* q, dp_solve_info* info, dp_request_times* times);
int dp_server_get_stats(dp_server* s, dp_server_stats* st);
/* Finish every queued and running request, then stop the workers. */
void dp_server_destroy(dp_server* s);

/* ------------------------------------------------------------------ test hooks */
/* H_0^(1)(z), H_1^(1)(z) for m real z > 0: out[4k..4k+3] = Re H0, Im H0,
 * Re H1, Im H1.  _dev: device arrays evaluated by the GPU kernel code;
 * _host: host arrays evaluated by the same source compiled for the CPU. */
int dp_hankel_dev(dp_ctx* ctx, int64_t m, const double* z, double* out);
int dp_hankel_host(int64_t m, const double* z, double* out);

/* The dense device LU with partial pivoting that factors floor(W) when its
 * sparse factors would fill in (Sec. 2.2), on a given matrix: a is a host
 * n x n complex matrix (column-major, interleaved re/im, 1 <= n <= 8192).
 * On DP_OK, lu (host, n x n, same layout) holds the unit lower L below the
 * diagonal and U on and above, and perm (host, n) the row order: row i of
 * L U is row perm[i] of a.  Pivots: the largest modulus in the column, ties
 * to the lower row index.  DP_ESINGULAR when a pivot column is zero or not
 * finite (lu and perm then untouched).  Synchronous. */
int dp_dense_lu_test(dp_ctx* ctx, int64_t n, const double* a, double* lu, int64_t* perm);

#ifdef __cplusplus
}
#endif

#endif /* DIRPREC_H */
