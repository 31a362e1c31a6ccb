/*
 * libppcg -- C ABI of the PPCG eigensolver hot path on MI355X (gfx950).
 *
 * Method: Vecharynski, Yang, Pask, "A Projected Preconditioned Conjugate
 * Gradient Algorithm for Computing Many Extreme Eigenpairs of a Hermitian
 * Matrix".  The problem statement (section 1; Algorithm 3 in the appendix):
 * given a Hermitian A (only products A x are needed), a Hermitian positive
 * definite preconditioner T, a start block X0 with k + nbuf columns, the
 * Rayleigh-Ritz period rr_period and the sub-block width sbsize, return
 * approximate eigenvectors X (n x k) and eigenvalues Lambda of the k
 * algebraically smallest eigenvalues.
 *
 * Here A is the finite-difference Kohn-Sham operator
 *     H = -1/2 Lap_h + diag(V)
 * on a periodic N x N x N grid with spacing h (7-point or 13-point
 * Laplacian), applied matrix-free, and T = diag(H)^{-1} (Jacobi).  With a
 * nonzero Bloch vector kappa the operator is complex Hermitian: the coupling
 * from grid point r to r + a h e_d carries the phase exp(i kappa_d a h) and
 * the one from r to r - a h e_d its conjugate (a = 1, 2), which is the gauge
 * form of -1/2 (grad + i kappa)^2 on a periodic cell; diag(H) is unchanged.
 *
 * Conventions
 *   - grid index of point (i, j, l) is i + N*(j + N*l) (x fastest); n = N^3.
 *   - blocks are column-major n x ncols with leading dimension n, float64
 *     for a real operator (kappa = 0) and interleaved complex float64
 *     (re, im pairs, 16 bytes per element, numpy complex128) for a complex
 *     one; V, eigenvalues and every other vector are real float64.
 *   - every pointer marked "device" is a device pointer on the handle's
 *     device; the caller owns it and keeps it alive until the call returns.
 *     The library owns its workspace (allocated lazily per shape inside the
 *     handle, released by ppcg_destroy).
 *   - all work is ordered on the stream given to ppcg_create; calls return
 *     after the stream work they enqueue has finished (synchronous).
 *   - a handle is not thread-safe; use one handle per host thread.
 *   - errors are return codes; ppcg_last_error() gives a message.
 */
#ifndef PPCG_H
#define PPCG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PPCG_OK = 0,
  PPCG_EINVAL = 1,    /* bad argument: sizes, null pointers, NaN in V */
  PPCG_ENOTHPD = 2,   /* Jacobi preconditioner not positive definite (diag(H) <= 0);
                         Theorem 2 assumes an HPD T */
  PPCG_ERANK = 3,     /* Cholesky breakdown of X^H X (Cholesky-QR) or of the
                         Rayleigh-Ritz Gram, or a sub-block pencil of rank < sbsize */
  PPCG_ENOCONV = 4,   /* max_iter reached; outputs hold the last Rayleigh-Ritz
                         result, info->resid_final its residual */
  PPCG_ENOSTATE = 5,  /* ppcg_grad called without a successful real solve */
  PPCG_EHIP = 6,      /* HIP runtime failure */
  PPCG_ENOMEM = 7     /* device allocation failed */
} ppcg_status;

typedef enum { PPCG_FP64 = 0, PPCG_MIXED = 1 } ppcg_precision;
/* Orthonormalisation of the updated block in iterations without a
 * Rayleigh-Ritz step (steps 17-19 of Algorithm 3; section 5.5), decided from
 * e = |Xbar^H Xbar - I|_F over the active columns. */
typedef enum {
  PPCG_ORTH_CHOLQR = 0, /* Cholesky-QR every such iteration */
  PPCG_ORTH_SKIP = 1,   /* omit steps 18-19 while e <= orth_skip, else Cholesky-QR */
  PPCG_ORTH_TAYLOR = 2, /* omit while e <= orth_skip; X <- X (I - Y/2 + 3Y^2/8 - 5Y^3/16),
                           Y = Xbar^H Xbar - I (four Taylor terms of the polar factor)
                           while e <= orth_taylor; else Cholesky-QR */
  PPCG_ORTH_NONE = 3    /* always omit steps 18-19 (the SCF use of section 6) */
} ppcg_orth;
/* Stopping test (section 5.2). */
typedef enum {
  PPCG_STOP_RESIDUAL = 0, /* relative subspace residual <= tol, then the final
                             Rayleigh-Ritz must pass a fresh residual check */
  PPCG_STOP_TRACE = 1     /* |trace(X^H H X) - previous| <= tol |trace(X^H H X)| between
                             consecutive iterations (all K columns), then the final
                             Rayleigh-Ritz (its residual is reported, not required) */
} ppcg_stop;
typedef enum { PPCG_PRECOND_NONE = 0, PPCG_PRECOND_JACOBI = 1 } ppcg_precond;

/* One record per PPCG iteration, passed to options.log_cb at the loop head
 * (convergence test of section 5.2) on the host thread of the call. */
typedef struct {
  int32_t iter;         /* iterations completed so far (0 = after the start block) */
  int32_t n_locked;     /* locked columns (soft locking, section 5.7) */
  int32_t n_active;     /* active columns K - n_locked */
  int32_t kind;         /* what the last iteration ended with: 0 start, 1 Cholesky-QR
                           (steps 18-20), 2 Rayleigh-Ritz (steps 21-31), 3 final
                           Rayleigh-Ritz that failed the fresh residual check */
  double rho;           /* relative subspace residual of the k wanted columns */
  double time_s;        /* wall time since the call started */
  double orth_err;      /* |Xbar^H Xbar - I|_F of the active block before the last
                           iteration's orthonormalisation (section 5.5); -1 when
                           not measured (Rayleigh-Ritz iterations, PPCG_ORTH_NONE) */
  double trace;         /* trace(X^H H X) over all K columns (locked ones from the
                           last Rayleigh-Ritz): the quantity PPCG minimises */
} ppcg_iter_log;
typedef void (*ppcg_log_fn)(const ppcg_iter_log* rec, void* user);

typedef struct {
  int32_t precision;  /* ppcg_precision.  PPCG_MIXED keeps W, P, HW, HP and the
                         projections X^H W, X^H P in float32 (MFMA, float32
                         accumulation), and forms the column coupling
                         X (G - diag G) of the residual from a float32 shadow
                         of X; X, H X, the Cholesky-QR, every Gram of the
                         sub-block pencils, the pencils themselves, the
                         Rayleigh-Ritz, H X - X diag(G) and the final residual
                         check stay float64 */
  int32_t nbuf;       /* buffer vectors (section 5.3); -1 = sbsize*ceil((k +
                         max(2, ceil(0.02 k)))/sbsize) - k, so k + nbuf is a
                         multiple of sbsize */
  int32_t max_iter;   /* iteration cap (default 20000 when <= 0) */
  int32_t profile;    /* nonzero: time every kernel launch with HIP events on
                         the handle's stream (see ppcg_kernel_times) */
  int32_t flags;      /* bit set of ppcg_flags */
  double singular_tol;/* Theorem 1 test of a sub-block step taken with P: C_X counts
                         as singular when a Cholesky pivot of C_X^H C_X is below this
                         floor (C^H B C = I and X orthonormal give C_X^H C_X <= I), and
                         the block is solved again without P (Theorem 2).  <= 0: 1e-12 */
  uint64_t seed;      /* X0 == NULL in ppcg_solve: the start block is drawn on the
                         device, N(0,1) entries (complex: real and imaginary parts
                         N(0,1/2)) from the Philox-4x32-10 counter generator keyed
                         by this seed, counter (row, column) */
  const char* tune_table; /* PPCG_AUTOTUNE: text file of autotuner decisions, read by
                         ppcg_create when it exists (an unreadable or malformed file
                         is PPCG_EINVAL) and rewritten after a solve that timed a
                         new shape class; NULL = decisions live in the handle only */
  ppcg_log_fn log_cb; /* per-iteration record (ppcg_iter_log); NULL = none */
  void* log_user;     /* passed back to log_cb */
  int32_t orth;       /* ppcg_orth (default PPCG_ORTH_CHOLQR) */
  int32_t stop;       /* ppcg_stop (default PPCG_STOP_RESIDUAL) */
  int32_t rr_max;     /* dynamic Rayleigh-Ritz period (section 5.6): the first
                         Rayleigh-Ritz after rr_max iterations, each following
                         interval one iteration shorter, down to rr_period;
                         <= rr_period: fixed period rr_period */
  double orth_skip;   /* PPCG_ORTH_SKIP / _TAYLOR threshold on e; <= 0: 0.1 */
  double orth_taylor; /* PPCG_ORTH_TAYLOR threshold on e (< 1); <= 0: 0.3 */
} ppcg_options;

typedef enum {
  PPCG_NO_GRAPHS = 1, /* issue the block-Jacobi sweeps of the Rayleigh-Ritz
                         eigensolve launch by launch instead of replaying the
                         captured HIP graph of one sweep (same results) */
  PPCG_AUTOTUNE = 2   /* time the candidate Gram / update kernels and row
                         splits of each new shape class once on the handle and
                         keep the fastest (see ppcg_tune_report); results stay
                         within rounding of the untuned choice, and after the
                         first solve of a shape class repeat exactly */,
  PPCG_RETURN_BUFFERS = 4 /* X_out receives all K = k + nbuf columns (n x K) and
                         lambda_out all K Ritz values of the final
                         Rayleigh-Ritz, buffer vectors included: the start
                         block of a warm-started next solve (a sequence of
                         slowly changing operators, as in the SCF use of
                         section 6) */
} ppcg_flags;

typedef struct {
  int32_t nx;           /* grid points per dimension N (n = N^3) */
  double h;             /* grid spacing */
  int32_t order;        /* 2 = 7-point Laplacian, 4 = 13-point (fourth order) */
  double kpt[3];        /* Bloch vector kappa (1/length); all zero = real
                           operator, otherwise complex Hermitian blocks */
  const double* V;      /* device, n potential values */
  int32_t precond;      /* ppcg_precond: PPCG_PRECOND_JACOBI, T = diag(H)^-1
                           (PPCG_ENOTHPD when diag(H) <= 0 anywhere), or
                           PPCG_PRECOND_NONE, T = I (step 8 of Algorithm 3
                           leaves W as it is); other values PPCG_EINVAL */
  const double* B;      /* device, n positive values, or NULL: the generalized
                           problem H x = lambda B x with B = diag(B) (section 1:
                           solved without factoring B, every inner product of
                           the method a B inner product, X^H B X = I on return).
                           Single FP64 solves only (PPCG_EINVAL with PPCG_MIXED,
                           in ppcg_solve_batched, and in ppcg_grad after such a
                           solve); B <= 0 anywhere is PPCG_ENOTHPD */
} ppcg_operator;

typedef struct {
  int32_t iters;        /* PPCG iterations (loop bodies executed) */
  int32_t n_rr;         /* Rayleigh-Ritz steps, the final one included */
  int32_t n_locked;     /* columns locked when the solve ended */
  int32_t n_backtrack;  /* sub-block solves redone without P (Theorem 2) */
  double resid_final;   /* |H X - X Lambda|_F / |Lambda|_F of the returned pairs,
                           from a fresh float64 H X */
  double orth_err;      /* |X^H X - I|_F of the returned X */
  double time_s;        /* wall time of the call */
  double stage_ms[6];   /* device time (HIP events, options.profile set; zeros
                           otherwise) in the categories of the paper's time
                           breakdown (section 6, Tables 4-5):
                           [0] GEMM: projection Grams and updates (steps 9-10),
                               per-block Grams (step 13 input), block update
                               (steps 14-15), residual X^H H X and H X - X G;
                           [1] AX: stencil products;
                           [2] RR: Rayleigh-Ritz Grams, Cholesky, eigensolve,
                               rotation and Ritz residuals (steps 21-31, final);
                           [3] CholQR: X^H X, Cholesky + inverse, X R^{-1}
                               (steps 18-19), and the start block's;
                           [4] small eig: the sub-block pencils (step 13);
                           [5] other: reductions of split partials outside the
                               above, column norms, copies */
  int32_t n_dropped;    /* W/P columns left out of sub-block pencils as zero or
                           dependent (summed over iterations and blocks) */
  int32_t n_unlock;     /* Rayleigh-Ritz steps at which the locked prefix shrank
                           (P is then reset: P(J_act) is undefined) */
  int32_t n_cholqr;     /* iterations without Rayleigh-Ritz that ran Cholesky-QR, */
  int32_t n_taylor;     /* ... the Taylor polar step, */
  int32_t n_orth_skip;  /* ... and neither (steps 18-19 omitted) */
  double roofline_ms;   /* options.profile set: sum over the modelled launches of
                           max(bytes / 8 TB/s, flops / dense MFMA peak of the
                           launch's dtype: 78.6 TFLOP/s float64, 157.3 float32),
                           i.e. the time of this solve with every modelled kernel
                           at the MI355X roofline */
} ppcg_info;

typedef struct ppcg_handle ppcg_handle;

/* Create a handle bound to the current HIP device and to `stream`
 * (hipStream_t passed as void*; NULL = the default stream).  opt may be NULL
 * (defaults: FP64, nbuf -1, max_iter 20000, no profiling). */
ppcg_status ppcg_create(ppcg_handle** out, const ppcg_options* opt, void* stream);

/* Solve for the k lowest eigenpairs (Algorithm 3).
 *   k         wanted pairs, 0 < k; K = k + nbuf must satisfy K <= n/4
 *   sbsize    sub-block width q of the block update (section 5.1), 1 <= q <= 32;
 *             K must be a multiple of q
 *   tol       relative subspace residual |HX - X(X^H H X)|_F / |X^H H X|_F
 *             over the k wanted columns (section 5.2); > 0
 *   rr_period Rayleigh-Ritz every rr_period iterations (section 5.6); >= 1
 *   X0        device, n x K start block (ld n), need not be orthonormal
 *             (complex when op->kpt != 0); NULL draws a seeded N(0,1) block on
 *             the device (options.seed)
 *   X_out     device, n x k (ld n): eigenvectors, orthonormal (complex when
 *             op->kpt != 0); n x K with PPCG_RETURN_BUFFERS
 *   lambda_out device, k: eigenvalues ascending (K with PPCG_RETURN_BUFFERS)
 *   info      may be NULL
 * On PPCG_ENOCONV the outputs hold the last Rayleigh-Ritz pairs. */
ppcg_status ppcg_solve(ppcg_handle* h, const ppcg_operator* op, int32_t k, int32_t sbsize, double tol,
                       int32_t rr_period, const double* X0, double* X_out, double* lambda_out, ppcg_info* info);

/* Backward pass (derivative of the eigen-decomposition).  For the pairs saved
 * by the last successful ppcg_solve on this handle (X n x k, Lambda), and the
 * loss L = sum_i g_lambda[i] lambda_i + sum_r w[r] rho[r] with the density
 * rho = sum_{i<k} |x_i|^2 (x_i Euclidean-normalised), writes
 *   dL_dV[r] = sum_i g_lambda[i] |x_i(r)|^2 - 2 Re sum_i conj(z_i(r)) x_i(r),
 * where z_i (orthogonal to X) solves the projected Sternheimer system
 *   Q (H - lambda_i) Q z_i = Q (w .* x_i),  Q = I - X X^H,
 * by block preconditioned CG (Jacobi 1/(diag(H) - lambda_i) when positive)
 * to relative residual `tol` per column (first-order perturbation of the
 * occupied invariant subspace; d lambda_i / dV = x_i^2 is Hellmann-Feynman).
 *   g_lambda  device, k
 *   w         device, n; NULL means w = 0 (eigenvalue terms only)
 *   dL_dV     device, n (output)
 *   max_iter  CG iteration cap (<= 0: 10000); iters (may be NULL) receives
 *             the iterations used, resid (may be NULL) the largest relative
 *             residual |r_i| / |b_i| over the columns at exit.
 * Real and complex Hermitian (Bloch) operators; V, w, g_lambda and dL_dV are
 * real in both cases.
 * PPCG_ENOCONV when the cap is reached with a column above tol (dL_dV then
 * holds the gradient of the last CG iterate); PPCG_ENOSTATE without a
 * successful solve.  Requires a gap between lambda_k and lambda_{k+1} (the
 * density is not differentiable otherwise). */
ppcg_status ppcg_grad(ppcg_handle* h, const double* g_lambda, const double* w, double* dL_dV, double tol,
                      int32_t max_iter, int32_t* iters, double* resid);

/* rho[r] = sum_{i<k} |x_i(r)|^2 for the pairs of the last successful solve
 * (device, n, real).  PPCG_ENOSTATE without a successful solve. */
ppcg_status ppcg_density(ppcg_handle* h, double* rho);

/* Columns K = k + nbuf of the start block ppcg_solve expects for this handle's
 * options (nbuf = -1 resolved by the default rule); -1 on bad arguments. */
int32_t ppcg_columns(const ppcg_handle* h, int32_t k, int32_t sbsize);

/* Batched form: nprob independent problems of uneven sizes (own operator,
 * k[b], start block X0[b] of n_b x K_b, outputs X_out[b] n_b x k[b] and
 * lambda_out[b]), sharing sbsize, tol and rr_period.  All problems advance
 * in lockstep: each stage of an iteration (projection Grams, stencils,
 * per-block Grams, every 3q x 3q block pencil of every problem, block
 * updates, Cholesky-QR, Rayleigh-Ritz) is one grouped launch over all
 * unconverged problems, instead of one launch per problem.  Each problem
 * follows exactly the arithmetic of ppcg_solve, so results equal those of
 * nprob separate ppcg_solve calls.
 *   ops, k, X0, X_out, lambda_out: host arrays of nprob entries (the
 *                 pointers they hold are device pointers); X0 may be NULL,
 *                 or hold NULL entries: problem b then draws its start block
 *                 on the device with seed options.seed + b
 *   infos, statuses: host arrays of nprob entries, may be NULL
 * A batch holds either only real or only complex operators; a problem whose
 * kind differs from the first valid one gets PPCG_EINVAL.
 * Returns PPCG_OK when every problem converged, else the first failing
 * problem's status (statuses[] holds each one).  The handle keeps one
 * workspace per problem index. */
ppcg_status ppcg_solve_batched(ppcg_handle* h, int32_t nprob, const ppcg_operator* ops, const int32_t* k,
                               int32_t sbsize, double tol, int32_t rr_period, const double* const* X0,
                               double* const* X_out, double* const* lambda_out, ppcg_info* infos,
                               int32_t* statuses);

/* Y = H X for ncols columns (device, ld n): the operator product alone.
 * X and Y are complex (interleaved) when op->kpt != 0.  PPCG_EINVAL for
 * nx < 4, h <= 0 or an order other than 2 and 4. */
ppcg_status ppcg_apply_h(ppcg_handle* h, const ppcg_operator* op, int32_t ncols, const double* X, double* Y);

/* The start block ppcg_solve draws on the device when X0 == NULL (the random
 * initial X of Algorithm 3), alone, so that the generator can be checked:
 * X[i + j n] for row i < n, column j < ncols is N(0,1) (cplx: real and
 * imaginary parts N(0,1/2), interleaved), from Philox-4x32-10 with counter
 * (i mod 2^32, j, i >> 32, 0) and key (seed mod 2^32, seed >> 32); the four
 * output words give two 53-bit uniforms u1, u2 in (0,1) and the Box-Muller
 * pair sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2).  Real blocks take the
 * first, complex blocks both, times sqrt(1/2).
 *   X   device out, n x ncols column-major (ld n), caller-owned
 * 0 <= n <= 2^31, 0 <= ncols <= 65535 (either zero: nothing drawn);
 * PPCG_EINVAL otherwise. */
ppcg_status ppcg_start_block(ppcg_handle* h, int64_t n, int32_t ncols, int32_t cplx, uint64_t seed, double* X);

/* The sub-block projected problems of one PPCG iteration alone (step 13 of
 * Algorithm 3; section 5.1; Theorems 1-2), for tests of that step: for each
 * of nblocks pencils (A_j, B_j) of order nS = 3q (has_p) or 2q, columns
 * ordered [X_j, W_j, P_j], returns the q lowest eigenvectors C_j of
 * herm(A_j) c = theta herm(B_j) c with C_j^H B_j C_j = I, exactly as
 * ppcg_solve computes them: diagonal scaling, zero W/P columns dropped,
 * greedy Cholesky in the order X, W, P, cyclic Jacobi, and when P took part
 * the Theorem 1 test on C_X (options.singular_tol) with the re-solve without
 * P of Theorem 2.
 *   A, B     device, nblocks matrices of nS x nS (column-major, ld nS,
 *            stride nS*nS; complex interleaved when cplx)
 *   tol      the solve tolerance the Jacobi skip threshold is tied to
 *            (rotations below max(2.2e-16, min(1e-10, 1e-4 tol)) |M|_F are
 *            skipped, as in ppcg_solve)
 *   C        device out, nblocks x (3q x q), ld 3q, stride 3q*q; rows of
 *            dropped columns (and the P rows without P) are zero
 *   flags    device out, nblocks ints: bit 0 P used, bit 1 backtracked
 *            (Theorem 1 test failed), bit 2 rank below q (C then holds
 *            [I; 0; 0]), bits 8.. number of W/P columns left out
 * 1 <= q <= 32; PPCG_EINVAL otherwise. */
ppcg_status ppcg_block_pencils(ppcg_handle* h, int32_t nblocks, int32_t q, int32_t has_p, int32_t cplx,
                               const double* A, const double* B, double tol, double* C, int32_t* flags);

/* ppcg_block_pencils for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): same arguments, results bit-identical to ppcg_block_pencils,
 * but the packed pencils and the work matrices live in a static device
 * array of 32 MiB that each GPU the library runs on holds until the process
 * ends (no hipMalloc, hipFree or other allocating call).  The work is only
 * enqueued on the handle's stream: C and flags are valid once that stream's
 * work has completed.  Every call on one GPU shares that array and its
 * contents: calls that overlap on one GPU (other streams or handles) race.
 * PPCG_EINVAL when the nblocks pencils need more than 32 MiB (per block:
 * nS (2 nS - q) + q (q + 1) scalars, plus 4 * 96 * 97 for nS > 48, scalars of
 * 8 bytes, 16 when complex, each area rounded up to 256 bytes). */
ppcg_status ppcg_block_pencils_noalloc(ppcg_handle* h, int32_t nblocks, int32_t q, int32_t has_p, int32_t cplx,
                                       const double* A, const double* B, double tol, double* C, int32_t* flags);

/* Per-kernel accumulated device time (ms) and launch counts since the last
 * reset, for kernels launched while options.profile was set.  names,
 * ms and counts are host arrays of capacity `cap`; returns the number of
 * kernel kinds written. */
int32_t ppcg_kernel_times(ppcg_handle* h, const char** names, double* ms, int64_t* counts, int32_t cap);
/* As ppcg_kernel_times, plus the algorithmic work of the same launches:
 * flops (floating-point operations the method needs, not the padded work
 * the kernels do) and bytes (compulsory HBM traffic: every input block read
 * once, every output block written once).  Any array may be NULL. */
int32_t ppcg_kernel_stats(ppcg_handle* h, const char** names, double* ms, int64_t* counts, double* flops,
                          double* bytes, int32_t cap);
void ppcg_reset_kernel_times(ppcg_handle* h);

/* The autotuner's decisions on this handle (PPCG_AUTOTUNE), one text line per
 * shape class: the kernel variant, workgroup target and minimum rows per
 * split chosen, its time and every candidate tried.  Writes at most cap - 1
 * characters and a terminating 0 into buf (may be NULL); returns the full
 * length, or -1 for a NULL handle. */
int32_t ppcg_tune_report(const ppcg_handle* h, char* buf, int32_t cap);

void ppcg_destroy(ppcg_handle* h);
const char* ppcg_last_error(const ppcg_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* PPCG_H */
