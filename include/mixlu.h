/*
 * mixlu.h -- C ABI of the MI355X (gfx950) mixed-precision dense solver.
 *
 * Method: Baboulin, Buttari, Dongarra, Kurzak, Langou, Langou, Luszczek,
 * Tomov, "Accelerating Scientific Computations with Mixed Precision
 * Algorithms" (arXiv:0808.2794), Algorithm 1 ("Mixed precision, Iterative
 * Refinement for Direct Solvers", Section 2.1): factor PA = LU in a low
 * precision eps_s, solve Ly = Pb, Ux_0 = y in eps_s, then repeat
 * r = b - A x (eps_d = FP64, with the original A), solve for the
 * correction z in eps_s, x = x + z in eps_d, until the stopping test of
 * Section 3 holds.  The symmetric positive definite variant replaces the LU
 * by a Cholesky factorization (SPOTRF/SPOTRS, Section 3.1.1).  When
 * refinement cannot converge (condition number above the inverse of the
 * low precision, Section 4) the solver falls back to an FP64 factorization.
 *
 * Conventions for every entry point
 * ---------------------------------
 * - Matrices are ROW-MAJOR by default: element (i, j) of an n x n matrix
 *   with leading dimension lda is A[i*lda + j] (lda >= n).  With
 *   opts->layout = MIXLU_COL_MAJOR the same pointers are read column-major
 *   (element (i, j) at A[i + j*lda]).  Right-hand sides B and solutions X
 *   are n x nrhs, row-major, leading dimension ldb/ldx >= nrhs (column-major
 *   with ldb/ldx >= n under MIXLU_COL_MAJOR).
 * - Every pointer documented as "device" is device memory of the context's
 *   GPU.  The caller owns all buffers (A, B, X, ipiv, work); the library
 *   allocates nothing that outlives a call except the context itself.
 * - A is never modified: factors live in the caller's workspace.
 * - Return value: MIXLU_OK (0), -i when argument i (1-based) is invalid, or a
 *   positive MIXLU_ERR_* code for runtime failures.  Numerical outcomes
 *   (singular matrix, fallback taken, iteration counts) are reported through
 *   `info` and mixlu_report, never through the return value.
 * - Work is enqueued on the context's stream (hipStream_t passed as void*).
 *   Calls that return a mixlu_report or an info value synchronize that
 *   stream before returning; the others are asynchronous.
 * - The library is built for gfx950 only; mixlu_create fails with
 *   MIXLU_ERR_UNSUPPORTED_ARCH on any other device.
 */
#ifndef MIXLU_H
#define MIXLU_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status */
#define MIXLU_OK 0
#define MIXLU_ERR_HIP 1             /* a HIP runtime call failed          */
#define MIXLU_ERR_WORKSPACE 2       /* lwork smaller than required        */
#define MIXLU_ERR_NOT_IMPLEMENTED 3 /* valid request this build lacks     */
#define MIXLU_ERR_UNSUPPORTED_ARCH 4
#define MIXLU_ERR_DEVICE_TIMEOUT 5  /* a bounded cross-workgroup wait on the
                                       device gave up (results invalid)   */
#define MIXLU_ERR_CAPTURING 6       /* a call that synchronizes was made on
                                       a stream under HIP graph capture   */

/* Human-readable name of a status code (static string, never NULL). */
const char *mixlu_status_string(int status);

/* ------------------------------------------------------- precisions */
/* Precision of the factorization (eps_s of Algorithm 1).  For BF16, FP16
   and FP8 the factors are stored in FP32 and only the operands of the
   trailing-matrix update are rounded to that format (FP32 accumulation);
   the panel, the triangular updates and the triangular solves run in FP32. */
typedef enum {
    MIXLU_FP64 = 0,
    MIXLU_FP32 = 1,
    MIXLU_BF16 = 2,
    MIXLU_FP16 = 3,
    MIXLU_FP8 = 4 /* OCP E4M3 operands with one E8M0 (power-of-two) scale
                     per 32 consecutive K values of each L21 row and U12
                     column, on the scaled 16x16x128 MFMA (nb >= 128) */
} mixlu_prec;

typedef enum { MIXLU_ROW_MAJOR = 0, MIXLU_COL_MAJOR = 1 } mixlu_layout;

/* ----------------------------------------------------------- options */
typedef struct {
    int itermax;      /* refinement iterations before declaring failure;
                         default 30 (Section 4: 30 means failure)            */
    int equilibrate;  /* -1 automatic (on for BF16/FP16/FP8), 0 off, 1 on:
                         power-of-two row then column scaling of the
                         low-precision copy only                            */
    int fallback;     /* 1 (default): on failure factor in FP64 and refine  */
    int nb;           /* outer block width of the factorization, 0 = auto   */
    int layout;       /* mixlu_layout of A, B and X.  Row-major (default):
                         element (i, j) at A[i * lda + j], B, X n x nrhs with
                         ld >= nrhs.  Column-major (LAPACK): A[i + j * lda],
                         B, X with ld >= n; the factorization then works on
                         the row-major matrix M = A^T that the memory holds
                         and the solves with A are transposed solves with M */
    double stall;     /* stall ratio: refinement is declared stalled when
                         ||r_k|| >= stall * ||r_{k-1}|| twice in a row
                         (k >= 2) or ||r_k|| >= ||r_{k-1}|| once (k >= 3);
                         default 0.9                                         */
    int refine;       /* mixlu_refine_kind (default MIXLU_REFINE_CLASSIC)    */
    int condest;      /* 1: after a low-precision factorization, estimate
                         kappa_1(A) with it (mixlu_condest); when
                         kappa_1 eps_s >= 1 skip the refinement and take
                         the FP64 path at once (report.iter = -5).  0
                         (default): no estimate.  mixlu_dxgesv/dxposv.     */
    int restart;      /* flexible GMRES restart length (MIXLU_REFINE_FGMRES):
                         0 = default 30, at most 128 (larger values use 128) */
    int reserved[3];
} mixlu_opts;

/* Refinement after the low-precision factorization.  CLASSIC is the
   stationary iteration of Algorithm 1.  FGMRES is the flexible GMRES outer
   loop of Algorithm 2, with one application of the low-precision LU solve
   as the (right) preconditioner in place of the inner single-precision
   GMRES: FP64 Arnoldi, restarts every `restart` steps (default 30), the
   stopping test of Section 3 on the true FP64 residual at every restart;
   `itermax` counts restart cycles, a cycle that cuts the true residual by
   less than 1% makes no progress and two such cycles in a row end the
   iteration (`stall` is not used), and report.iter counts preconditioner
   applications.  It keeps converging where kappa eps_s approaches or
   exceeds 1 (BF16/FP16/FP8 factors), where CLASSIC stalls.  FGMRES applies
   to one right-hand side of op(A) = A; other calls use CLASSIC. */
typedef enum { MIXLU_REFINE_CLASSIC = 0, MIXLU_REFINE_FGMRES = 1 } mixlu_refine_kind;

/* Fill *o with the defaults listed above. */
void mixlu_default_opts(mixlu_opts *o);

/* ------------------------------------------------------------ report */
/* Outcome of one solve (host memory, filled before the call returns). */
typedef struct {
    int iter;      /* >= 0: refinement corrections applied by the
                      low-precision path (x_0 counts as 0).
                      With prec = MIXLU_FP64 requested, the corrections
                      of the FP64 refinement itself.
                      < 0: the FP64 fallback produced X, for the reason
                      -1 A is exactly singular (see info; X undefined),
                      -2 overflow or non-finite value converting A,
                      -3 zero or non-finite pivot in the low-precision
                         factor (Cholesky: non-positive pivot),
                      -4 refinement stalled,
                      -5 the kappa_1 estimate ruled the low precision out
                         (opts.condest),
                      -(itermax+1) no convergence within itermax.        */
    int info;      /* 0, or k+1 when the FP64 factorization met an exactly
                      zero pivot in column k (A singular; X undefined)     */
    int prec;      /* mixlu_prec of the factors that produced X           */
    int fallback_iter; /* corrections applied by the FP64 refinement      */
    double anorm;  /* ||op(A)||_inf (||A||_1 for a transposed solve)      */
    double rnorm;  /* max over columns of ||b - A x||_inf (FP64, final x) */
    double xnorm;  /* max over columns of ||x||_inf                       */
    double berr;   /* max over columns of ||r|| / (||A|| ||x||)           */
    int converged; /* 1 when every column meets the stopping test
                      ||r||_inf <= sqrt(n) 2^-53 ||A||_inf ||x||_inf       */
    float cond_est; /* kappa_1 estimate when opts.condest asked for it,
                       else 0                                            */
    int outer;      /* mixlu_sparse_fgmres: outer FGMRES cycles run      */
    int reserved[1];
} mixlu_report;

/* ----------------------------------------------------------- context */
typedef struct mixlu_ctx_s *mixlu_ctx_t;

/* Create a context on the current HIP device, bound to `stream`
   (a hipStream_t; NULL = the default stream).  Fails on non-gfx950. */
int mixlu_create(mixlu_ctx_t *ctx, void *stream);
int mixlu_destroy(mixlu_ctx_t ctx);
int mixlu_set_stream(mixlu_ctx_t ctx, void *stream);

/* --------------------------------------------------------- workspace */
typedef enum {
    MIXLU_OP_GESV = 0,  /* mixlu_dxgesv, or mixlu_getrf + getrs/refine      */
    MIXLU_OP_POSV = 1,  /* mixlu_dxposv, or mixlu_potrf + getrs/refine      */
    MIXLU_OP_DGESV = 2, /* mixlu_dgesv (FP64 LU, no refinement)             */
    MIXLU_OP_DPOSV = 3, /* mixlu_dposv (FP64 Cholesky, no refinement)       */
    MIXLU_OP_SGESV = 4  /* mixlu_sgesv (FP32 LU, no refinement)             */
} mixlu_op;

/* Bytes of device workspace the operation needs for (prec, n, nrhs) with
   options o (NULL = defaults).  The workspace holds the factors, pivots,
   scales, refinement vectors, device-side exchange buffers and, when
   o->fallback is set, room for the FP64 fallback factor (8 n^2 bytes). */
int mixlu_workspace_size(mixlu_ctx_t ctx, int op, int prec, int n, int nrhs,
                         const mixlu_opts *o, size_t *bytes);

/* ----------------------------------------------------------- factors */
/* Description of factors that live inside a caller workspace.  Filled by
   mixlu_getrf / mixlu_potrf; valid while the workspace is unchanged. */
typedef struct {
    int n, npad;       /* order, and padded order of the stored factor     */
    int nb;            /* outer block width used by the factorization       */
    int prec;          /* mixlu_prec of the factorization                  */
    int kind;          /* 0 LU with partial pivoting, 1 Cholesky (lower)   */
    int layout;        /* layout of the A it was computed from             */
    int equilibrated;  /* 1 when R, C scaling was applied                  */
    int lowp_status;   /* 0 ok; -2 conversion overflow; -3 breakdown;
                          -1 the FP64 fallback factor that mixlu_refine
                          left in the workspace is singular (X undefined);
                          MIXLU_FACTOR_PENDING after an asynchronous
                          factorization, until mixlu_refine reads the
                          outcome from the device                         */
    int nrhs_max;      /* most right-hand sides one solve may have: what
                          the workspace given to the factorization holds  */
    void *work;        /* the workspace (device)                           */
    size_t lwork;
    size_t off[16];    /* internal offsets into work                       */
} mixlu_factor;

/* Factor A (device, n x n, const) in precision prec (Algorithm 1 step 1):
   ||A||_inf, optional equilibration, conversion to the working format and
   blocked LU with partial pivoting on the GPU.  *info (host) receives 0, or
   k+1 for an exact zero pivot in column k when prec = MIXLU_FP64.  Low-
   precision breakdown or overflow is recorded in F->lowp_status instead.
   Synchronizes the stream. */
int mixlu_getrf(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda,
                void *work, size_t lwork, const mixlu_opts *o,
                mixlu_factor *F, int *info);

/* Cholesky factorization of a symmetric positive definite A (the SPOTRF of
   Section 3.1.1): symmetric power-of-two scaling S (when equilibration is
   on), W = fl(S A S), blocked right-looking W = L L^T with the trailing
   update in prec (FP32 or BF16/FP16 operands with FP32 accumulation).  Only
   the lower triangle of the row-major A is used by the factorization; the
   refinement residual uses the whole stored A, which must be symmetric.
   The factor is stored as W = L' U' with L' = L D^{-1} (unit lower),
   U' = D L^T and an identity permutation, so mixlu_getrs and mixlu_refine
   apply to it unchanged.  A non-positive or non-finite pivot is reported
   like a zero pivot of mixlu_getrf (info = k+1 for FP64, F->lowp_status =
   -3 otherwise).  Synchronizes the stream. */
int mixlu_potrf(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda,
                void *work, size_t lwork, const mixlu_opts *o,
                mixlu_factor *F, int *info);

/* Stream-ordered forms of mixlu_getrf and mixlu_potrf: the same
   conversion and factorization, enqueued on the context's stream without
   any synchronization or host read-back, so that a caller can overlap them
   with its own work or capture them in a HIP graph (with the context bound
   to the capturing stream by mixlu_set_stream; the context's second stream
   joins the capture through events and is joined back before the call
   returns).  The outcome is written to *d_info (device int) when the
   factorization ends: 0; k+1 for an exact zero pivot in column k of an FP64
   factor; -2 (overflow or non-finite value on conversion) or -3 (zero,
   non-finite or, for Cholesky, non-positive pivot) for a low-precision
   factor; -100 when a bounded cross-workgroup wait gave up.  *F (host) is
   filled at once, with F->lowp_status = MIXLU_FACTOR_PENDING; mixlu_getrs
   may follow on the same stream, and mixlu_refine reads the outcome itself.
   Argument errors as for mixlu_getrf (-10: d_info is NULL). */
#define MIXLU_FACTOR_PENDING 1
int mixlu_getrf_async(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda,
                      void *work, size_t lwork, const mixlu_opts *o,
                      mixlu_factor *F, int *d_info);
int mixlu_potrf_async(mixlu_ctx_t ctx, int prec, int n, const double *A, int lda,
                      void *work, size_t lwork, const mixlu_opts *o,
                      mixlu_factor *F, int *d_info);

/* Low-precision solve only (Algorithm 1 steps 2-3): X = op(A)^{-1} B with
   the stored factors, computed in the factor's precision and promoted to
   FP64.  trans = 1 solves A^T X = B with the same factors (W = R A C,
   P W = L U: X = R P^T L^{-T} U^{-T} C B), as the adjoint of a solve needs.
   B, X device, n x nrhs (nrhs <= the nrhs the workspace was sized for), in
   the factor's layout.  Asynchronous on the context's stream. */
int mixlu_getrs(mixlu_ctx_t ctx, const mixlu_factor *F, int trans, int nrhs,
                const double *B, int ldb, double *X, int ldx);

/* Refinement loop (Algorithm 1 steps 4-7) starting from the X given:
   r = B - op(A) X in FP64 with the original A, correction solved with the
   factors, X += Z in FP64, until the stopping test holds for every column
   or the policy declares failure (then, when o->fallback is set, an FP64
   factorization in the workspace finishes the job).  trans = 1 refines
   A^T X = B (residual B - A^T X in FP64, stopping test with ||A||_1).
   B and X are n x nrhs, nrhs <= F->nrhs_max.  rep (host) is filled; the
   stream is synchronized.  When the fallback runs, *F is rewritten to
   describe the FP64 factor it leaves in the workspace (F->prec =
   MIXLU_FP64, unit scales, no further fallback; F->lowp_status = -1 if that
   factor is singular): the low-precision factor's pivots and scales are
   overwritten by it, so later mixlu_getrs, mixlu_refine and mixlu_condest
   calls with F solve with the FP64 factor (the adjoint of a solve that
   fell back uses the FP64 factor too). */
int mixlu_refine(mixlu_ctx_t ctx, mixlu_factor *F, int trans, int nrhs,
                 const double *A, int lda, const double *B, int ldb, double *X,
                 int ldx, const mixlu_opts *o, mixlu_report *rep);

/* Estimate of the 1-norm condition number kappa_1(A) = ||A||_1 ||A^{-1}||_1
   from the stored factors, for deciding whether refinement with them can
   converge (Section 4: it needs kappa eps_s below about one).  ||A^{-1}||_1
   is estimated by Hager's method with Higham's refinement, the scheme of
   LAPACK's xGECON: from x = (1/n, ..., 1/n), y = A^{-1} x,
   z = A^{-T} sign(y), stop when ||z||_inf <= z^T x, else restart from x =
   e_j with j the first index of the largest |z_j| (at most 5 sweeps); the
   result is the larger of ||y||_1 and 2 ||A^{-1} v||_1 / (3n) for
   v_i = (-1)^i (1 + i/(n-1)).  Solves use the factors' precision, so the
   value is a lower bound of kappa_1 up to the factor's error; it is exact
   for diagonal A.  Uses the workspace's Krylov vectors (not valid during
   an FGMRES refinement).  *kappa1 (host).  Synchronizes. */
int mixlu_condest(mixlu_ctx_t ctx, const mixlu_factor *F, double *kappa1);

/* One-shot mixed-precision solve A X = B (DSGESV-style): factor in prec,
   x_0, refinement, FP64 fallback.  A, B (const) and X are device memory. */
int mixlu_dxgesv(mixlu_ctx_t ctx, int prec, int n, int nrhs, const double *A,
                 int lda, const double *B, int ldb, double *X, int ldx,
                 void *work, size_t lwork, const mixlu_opts *o,
                 mixlu_report *rep);

/* Same for symmetric positive definite A (DSPOSV-style, Cholesky; see
   mixlu_potrf).  The fallback is the FP64 Cholesky; if that breaks down
   too, rep->info = k+1 (A not positive definite) and X is undefined. */
int mixlu_dxposv(mixlu_ctx_t ctx, int prec, int n, int nrhs, const double *A,
                 int lda, const double *B, int ldb, double *X, int ldx,
                 void *work, size_t lwork, const mixlu_opts *o,
                 mixlu_report *rep);

/* FP64 LU with partial pivoting and FP64 triangular solves, no refinement
   (the DGESV comparator, and the factorization the fallback uses).
   A is const; *info (host) as in mixlu_getrf.  Synchronizes. */
int mixlu_dgesv(mixlu_ctx_t ctx, int n, int nrhs, const double *A, int lda,
                const double *B, int ldb, double *X, int ldx, void *work,
                size_t lwork, int *info);

/* FP32 LU with partial pivoting and FP32 triangular solves, no refinement
   and no equilibration: the single-precision solve of Section 2.1 alone
   (what Algorithm 1 steps 1-3 give before any correction; the SGESV
   baseline).  A and B are FP64 (const), rounded to FP32 on the device; X
   (FP64) receives the FP32 solution.  Row-major, like mixlu_dgesv;
   workspace from mixlu_workspace_size(op MIXLU_OP_SGESV).  *info (host): 0,
   k+1 for an exact zero or non-finite pivot in column k (X untouched), or
   n+1 when an entry of A lies outside the FP32 range.  Synchronizes. */
int mixlu_sgesv(mixlu_ctx_t ctx, int n, int nrhs, const double *A, int lda,
                const double *B, int ldb, double *X, int ldx, void *work,
                size_t lwork, int *info);

/* FP64 Cholesky and FP64 triangular solves, no refinement (the DPOSV
   comparator, and the factorization the Cholesky fallback uses).  *info
   (host): 0, or k+1 when the leading minor of order k+1 is not positive
   definite.  Synchronizes. */
int mixlu_dposv(mixlu_ctx_t ctx, int n, int nrhs, const double *A, int lda,
                const double *B, int ldb, double *X, int ldx, void *work,
                size_t lwork, int *info);

/* Adjoint helper: GA = GA_beta * GA + alpha * Gb * X^T (all device, FP64,
   row-major; Gb and X are n x nrhs, GA is n x n).  With alpha = -1 and
   GA_beta = 0 this forms the gradient g_A = -g_b x^T of x = A^{-1} b. */
int mixlu_outer_update(mixlu_ctx_t ctx, int n, int nrhs, const double *Gb,
                       int ldg, const double *X, int ldx, double *GA, int ldga,
                       double alpha, double GA_beta);

/* The trailing-matrix update of the factorization on its own: C -= A B,
   the one O(n^3) operation of the LU, which Section 2.1 performs in the low
   precision eps_s.  A (m x k), B (k x n) and C (m x n) are row-major FP32
   device matrices (leading dimensions lda >= k, ldb >= n, ldc >= n).  The
   operands are used as the factorization uses L21 and U12:
   MIXLU_FP32: as stored (FP32 MFMA); MIXLU_BF16 / MIXLU_FP16: rounded to
   nearest even (k a multiple of 64); MIXLU_FP8: E4M3 codes (round to
   nearest even, saturating at 448) with one E8M0 power-of-two scale per 32
   consecutive k values of each row of A and each column of B, the scale
   putting the block's largest magnitude in [2^7, 2^8) (k a multiple of
   128).  Products accumulate in FP32.  work (device) holds the rounded
   operands: lwork >= 2 (m + n) k + (m + n) k / 32 + 1024 bytes (unused for
   FP32).  *overflow (host, may be NULL) receives the number of operands
   outside the format's range (FP16: |x| > 65504; FP8: non-finite blocks);
   passing it synchronizes the stream, otherwise the call is asynchronous. */
int mixlu_gemm_update(mixlu_ctx_t ctx, int prec, int m, int n, int k,
                      const float *A, int lda, const float *B, int ldb, float *C,
                      int ldc, void *work, size_t lwork, int *overflow);

/* ------------------------------------------------------------ batched */
/* Many independent systems A_i x_i = b_i (each n_i <= 512), every one
   solved as mixlu_dxgesv would (factor in prec with the same
   equilibration rule, x_0, FP64 refinement, stall rule, FP64 fallback),
   all inside one persistent launch: each workgroup takes systems from a
   device queue ordered by decreasing n_i and solves them one at a time.
   All pointer arrays and the reports live in device memory: d_n[i] order,
   d_A[i] row-major n_i x n_i with leading dimension d_lda[i] (d_lda = NULL:
   n_i), d_B[i] and d_X[i] row-major n_i x nrhs with leading dimension nrhs.
   d_reps[i] (device) receives the report of system i; a system with
   n_i > 512 or lda_i < n_i gets info = -1, converged = 0 and X untouched.
   The call only enqueues work on the context's stream: no synchronization,
   no allocation, no host reads of device data, so it can be captured in a
   HIP graph and replayed.  Row-major layout only. */
int mixlu_batched_workspace_size(mixlu_ctx_t ctx, int prec, int batch, int nrhs,
                                 const mixlu_opts *o, size_t *bytes);
int mixlu_dxgesv_batched(mixlu_ctx_t ctx, int prec, int batch, const int *d_n,
                         const double *const *d_A, const int *d_lda,
                         const double *const *d_B, double *const *d_X, int nrhs,
                         void *work, size_t lwork, const mixlu_opts *o,
                         mixlu_report *d_reps);

/* Allocation-free variant of mixlu_dxgesv_batched, for callers that cannot
   allocate device memory (code under HIP graph capture, tight serving
   loops, harnesses that forbid hipMalloc): the same solve, arguments and
   reports, with no workspace argument.  Its queue, counters and factor
   slots live in a device array of the library (64 MiB + 256 KiB per GPU,
   held from the first use of the library on that GPU until the process
   ends): at most 65536 systems per call (more: MIXLU_ERR_WORKSPACE) and 32
   persistent workgroups, so it is slower than the workspace call on large
   batches.  Every call on one GPU uses that GPU's single array, which keeps
   the last call's contents: calls that overlap on one GPU (two streams, or
   two host threads) race and must be serialized by the caller.  No
   allocation, synchronization or host read of device data; capturable.
   MIXLU_ERR_HIP if the array's device address could not be obtained. */
int mixlu_dxgesv_batched_noalloc(mixlu_ctx_t ctx, int prec, int batch, const int *d_n,
                                 const double *const *d_A, const int *d_lda,
                                 const double *const *d_B, double *const *d_X, int nrhs,
                                 const mixlu_opts *o, mixlu_report *d_reps);

/* Tile choices of the batched launch: the panel width of each system's LU
   (8 or 16 columns), the column chunk of its trailing update (32, 64 or
   128) and the number of persistent workgroups per compute unit (1 or 2).
   The context keeps one set per precision; mixlu_dxgesv_batched uses it.
   Defaults: panel 16, chunk 128, groups 2 (FP64: groups 1). */
typedef struct {
    int panel;
    int chunk;
    int groups;
    int tuned;  /* 1 when the set came from mixlu_batched_tune */
} mixlu_batched_tiles;

/* Autotuner: runs the batched solve of the given batch (same arguments as
   mixlu_dxgesv_batched) once with every candidate tile set, timed with HIP
   events on the context's stream (each candidate once untimed, then the
   faster of two timed runs), and keeps the fastest set in the context for
   prec.  The last run leaves X and d_reps as a normal call would (each
   candidate solves the same systems completely).  best (host, may be NULL)
   receives the chosen set; ms (host, may be NULL) the time of candidate i
   for i < max_ms, in the order panel {16, 8} x chunk {128, 64, 32} x groups
   {2, 1}.  Synchronizes; returns MIXLU_ERR_CAPTURING if the stream is being
   captured (tune before capturing, then capture the tuned launch). */
int mixlu_batched_tune(mixlu_ctx_t ctx, int prec, int batch, const int *d_n,
                       const double *const *d_A, const int *d_lda,
                       const double *const *d_B, double *const *d_X, int nrhs,
                       void *work, size_t lwork, const mixlu_opts *o,
                       mixlu_report *d_reps, mixlu_batched_tiles *best,
                       float *ms, int max_ms);
/* Read or set the tile set the context uses for prec (set: -3 if the set is
   not one of the candidates). */
int mixlu_batched_get_tiles(mixlu_ctx_t ctx, int prec, mixlu_batched_tiles *t);
int mixlu_batched_set_tiles(mixlu_ctx_t ctx, int prec, const mixlu_batched_tiles *t);

/* ------------------------------------------------------------- sparse */
/* Inner-outer FGMRES(m_out)-GMRES(m_in) for a sparse A (Section 3.2,
   Algorithm 2).  A is n x n in CRS storage (device): rowptr[n + 1],
   colind[nnz] (0-based), vals[nnz] (FP64).  The outer flexible GMRES runs in
   FP64 from x = 0: r = b - A x, the stopping test of Section 3 on this true
   residual (||r||_inf <= sqrt(n) 2^-53 ||A||_inf ||x||_inf), then up to
   m_out flexible Arnoldi steps whose preconditioner is one cycle of
   GMRES(m_in) from zero in the inner precision (MIXLU_FP32: GMRES_SP on an
   FP32 copy of the values; MIXLU_FP64: GMRES_DP), the FP64 product A z_k,
   Gram-Schmidt against the basis (classical, applied twice) and the new
   basis vector; a cycle ends early once its least-squares residual meets
   the threshold; then x += Z y.  Every reduction of both loops runs on the
   device; the small least-squares problems are solved on the host.  b and
   x (device, n).  o->itermax bounds the outer cycles and o->stall applies
   the refinement's stall rule to their residuals (NULL: defaults).  rep
   (host): iter = inner cycles run (preconditioner applications), or -4 /
   -(itermax+1) on failure (no direct fallback exists for a sparse A; x then
   holds the last iterate), outer = outer cycles, rnorm/xnorm/berr of the
   final x, anorm = ||A||_inf, prec = inner_prec.  Synchronizes. */
int mixlu_sparse_workspace_size(mixlu_ctx_t ctx, int inner_prec, int n, int nnz,
                                int m_out, int m_in, size_t *bytes);
int mixlu_sparse_fgmres(mixlu_ctx_t ctx, int inner_prec, int n, int nnz,
                        const int *rowptr, const int *colind,
                        const double *vals, const double *b, double *x,
                        int m_out, int m_in, void *work, size_t lwork,
                        const mixlu_opts *o, mixlu_report *rep);

/* Copy count reports from device memory (d, as filled by
   mixlu_dxgesv_batched) to host memory h, in order on the context's stream;
   synchronizes the stream. */
int mixlu_report_read(mixlu_ctx_t ctx, const mixlu_report *d, int count,
                      mixlu_report *h);

/* ------------------------------------------------------ kernel timing */
/* Per-kernel-class timing for measurement: with profiling enabled, the
   launches of the main kernel classes ("panel_getf2", "trailing_update",
   "pack_operands", "trsv", "residual", "panel_potf2", "batched_solve",
   "sparse_spmv") are bracketed by HIP events on the
   context's stream, and each class accumulates its launch count, total
   device time and the algorithmic flops and bytes of its launches (the work
   the method requires, not the traffic the kernels generate).  Enabling
   clears the totals.  The timing adds two event records per launch. */
typedef struct {
    const char *name;     /* static string                              */
    long long launches;
    double ms;            /* summed event time of the launches          */
    double flops;         /* algorithmic floating-point operations      */
    double bytes;         /* algorithmic memory traffic                 */
} mixlu_kstat;

int mixlu_profile_enable(mixlu_ctx_t ctx, int on);
/* Copies up to max class records into out (host) and the number of classes
   into *count; synchronizes the stream. */
int mixlu_profile_read(mixlu_ctx_t ctx, mixlu_kstat *out, int max, int *count);

/* The true-residual norms ||b - A x||_inf (largest over the right-hand
   sides) that the last mixlu_refine / mixlu_dxgesv / mixlu_dxposv call on
   this context evaluated, in order: one per iteration of the stationary
   refinement, one per restart cycle of FGMRES, then those of the FP64
   fallback if it ran.  h (host) receives the first min(count, max); *count
   the number recorded.  A diagnostic: tells slow convergence from a stall. */
int mixlu_refine_history(mixlu_ctx_t ctx, double *h, int max, int *count);

#ifdef __cplusplus
}
#endif

#endif /* MIXLU_H */
