/*
 * rpca.h -- C ABI of an MI355X (gfx950) implementation of the randomized
 * principal component analysis of Szlam, Kluger and Tygert, "An
 * implementation of a randomized algorithm for principal component analysis"
 * (ACM TOMS 2014, arXiv:1412.3510).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All matrix pointers (A, U, V, S, lambda, workspace-free outputs) are
 *    DEVICE pointers owned by the caller.  The library never frees them.
 *    Host pointers appear only where a name says so (``*_host``).
 *  - Dense matrices are row-major with an explicit leading dimension (in
 *    elements).  A leading dimension that is a multiple of 4 and a 16-byte
 *    aligned base give the vectorized load path; other layouts are accepted
 *    and take a scalar path.
 *  - Every call is ordered on the context's HIP stream and returns before the
 *    device has finished, unless RPCA_SYNC is passed (or the call returns a
 *    host value, which implies a synchronization).
 *  - On error nothing is launched (argument errors) or the outputs are left
 *    unspecified (device-side failures: RPCA_ERR_NOT_PSD, RPCA_ERR_NUMERICAL,
 *    reported by the next synchronizing call); the status says which, and
 *    rpca_last_error() gives a message.
 *  - l <= 0 means l = k + 2 (the paper's default oversampling, Section 7).
 *    Supported range: 1 <= k <= l <= min(m, n) and l <= 128.
 *  - A context is not thread-safe; calls that overlap on one context race.
 */
#ifndef RPCA_H
#define RPCA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rpca_ctx_s* rpca_ctx;

typedef enum {
  RPCA_OK = 0,
  RPCA_ERR_INVALID_ARG = 1, /* bad sizes, null pointers, k > l, ...        */
  RPCA_ERR_UNSUPPORTED = 2, /* a format/dtype/size the library lacks        */
  RPCA_ERR_NO_MEMORY = 3,   /* workspace allocation failed or over the limit */
  RPCA_ERR_HIP = 4,         /* a HIP runtime call failed                     */
  RPCA_ERR_NOT_PSD = 5,     /* Nystrom: shifted B2 never positive definite   */
  RPCA_ERR_NUMERICAL = 6,   /* non-finite values met on the device           */
  RPCA_ERR_TIMEOUT = 7      /* a bounded device wait gave up: the workgroups
                               sharing one batched problem were not on the
                               device together (see rpca_set_batch_split)   */
} rpca_status;

typedef enum { RPCA_F32 = 0, RPCA_BF16 = 1, RPCA_FP8_E4M3 = 2 } rpca_dtype;
typedef enum { RPCA_DENSE_ROWMAJOR = 0, RPCA_SPARSE_CSR = 1 } rpca_format;

/* A matrix operand.  For RPCA_DENSE_ROWMAJOR, ``data`` holds m rows of n
 * elements of ``dtype`` with leading dimension ``ld`` (elements), in device
 * memory owned by the caller.  ``col_scale`` (E4M3 only, device, length n)
 * gives the per-column scale: A = data * diag(col_scale).
 *
 * Precision form: with dtype RPCA_BF16 or RPCA_FP8_E4M3 every pass of the
 * range finder reads the low-precision copy (products in bfloat16 on the
 * matrix cores, float32 accumulation), and the Rayleigh-Ritz product B = Q* A
 * (Section 2, (i3)), the Nystrom product B1 = A Q (Section 3, (start)) and
 * rpca_spectral_err read ``data_f32``/``ld_f32``, the float32 A, when it is
 * given; NULL means the low-precision copy is used there too (spectral_err
 * then returns RPCA_ERR_UNSUPPORTED).  Low-precision copies need n and ld to
 * be multiples of 8 (bfloat16) or 16 (E4M3) and 16-byte-aligned data, else
 * RPCA_ERR_UNSUPPORTED.  rpca_quantize prepares both copies.
 * The sparse fields are reserved for the CSR format. */
typedef struct {
  int32_t format; /* rpca_format */
  int32_t dtype;  /* rpca_dtype  */
  int64_t m, n;
  const void* data;
  int64_t ld;
  const float* col_scale;
  const float* data_f32;
  int64_t ld_f32;
  int64_t nnz;
  const int32_t* row_ptr;
  const int32_t* col_idx;
  const void* val;
  const int32_t* col_ptr;
  const int32_t* row_idx;
  const void* val_t;
} rpca_matrix;

/* flags */
enum {
  RPCA_CENTER = 1u, /* PCA of the column-centered matrix (Sections 2 and 5)     */
  RPCA_SYNC = 2u,   /* synchronize the stream before returning, and report the
                       device-side failures of every solve issued on the
                       context since the last synchronizing call (see
                       rpca_sync)                                              */
  RPCA_DETERMINISTIC = 4u, /* use the built-in tile configurations even where
                       the autotuner has stored others: every summation order
                       and pivot tournament is then fixed by the shapes and the
                       device's compute-unit count, so repeated calls (and
                       calls on other contexts of the same device model) give
                       bit-identical results.  Without it the results are still
                       bit-identical run to run on one context whose autotune
                       table does not change.                                  */
  RPCA_RENORM_ORTH = 8u, /* renormalize by the two-pass orthonormalization
                           (Cholesky QR twice) after every application of A
                           or A*                                               */
  RPCA_RENORM_LU = 16u, /* renormalize by pivoted LU (Q = P L, tournament
                           pivoting) after every application but the last --
                           the paper's choice (Section 5)                     */
  RPCA_OMEGA_UNIFORM = 32u, /* draw the test matrix Omega uniformly on (-1, 1)
                           (rpca_uniform) instead of from N(0, 1): Section 5
                           notes the method does not depend on the law, and
                           each 32-bit word then gives one entry (no
                           transcendental functions)                          */
  RPCA_NYSTROM_SQRT = 64u, /* rpca_eig_psd: stabilize by the self-adjoint square
                           root of B2 and a regularized pseudoinverse (Section
                           3's first remedy) instead of the shifted Cholesky
                           factor: B2 = W diag(w) W^T, F = B1 W diag(w)^-1/2
                           over the w above sqrt(n) u ||B1||_F (the shift's
                           scale), lambda = the squared singular values of F.
                           Never reports RPCA_ERR_NOT_PSD.                    */
  RPCA_FUSED_ATA = 128u /* rpca_svd: renormalize only after every second
                           application (the acceleration Section 5 describes
                           and the paper does not adopt): starting from Omega,
                           its times Z = A_c^T (A_c Z) with no renormalization
                           between the two products, then Z renormalized;
                           then Y = A_c Z orthonormalized and Rayleigh-Ritz
                           as usual.  The sketched range is the same in exact
                           arithmetic; the squared spectrum of A^T A costs
                           accuracy where sigma_j^2 / sigma_1^2 falls below
                           the products' resolution (2^-16 for float32 A,
                           2^-8 for a bfloat16 copy).  Where the shape allows,
                           A^T A Z is formed in one read of A (row panels:
                           Y_p = A_p Z, then Z += A_p^T Y_p).  Not for the
                           self-adjoint entry points (RPCA_ERR_INVALID_ARG). */
};
/* Renormalization between applications of A and A* (Sections 2 and 5).
 * Each is right-multiplication by an invertible l x l matrix, so the span and
 * the result in exact arithmetic do not depend on it; only its cost and the
 * conditioning of the basis it returns do.  By default one pass of Cholesky
 * QR with a float64 Gram matrix (Q = Y R^-1, R^T R = Y^T Y): on this device
 * it costs a third of the pivot tournament, whose l dependent elimination
 * steps bound it by latency, where Section 5 chose LU because it costs less
 * than QR on a CPU.  When that Cholesky factorization needs a shift (Y
 * numerically rank deficient) the repair passes of the orthonormalizing form
 * follow.  The last renormalization before B = Q* A is always the two-pass
 * orthonormalization.  RPCA_RENORM_LU and RPCA_RENORM_ORTH select the
 * others. */

/* Create a context on the current HIP device, ordered on ``hip_stream``
 * (a hipStream_t; NULL = the null stream).  Owns its workspace. */
rpca_status rpca_create(rpca_ctx* out, void* hip_stream);
rpca_status rpca_destroy(rpca_ctx ctx);
rpca_status rpca_set_stream(rpca_ctx ctx, void* hip_stream);
/* Cap on the workspace the context may hold (bytes; 0 = no cap).  A call
 * that needs more returns RPCA_ERR_NO_MEMORY before launching anything. */
rpca_status rpca_set_workspace_limit(rpca_ctx ctx, size_t bytes);
rpca_status rpca_workspace_size(rpca_ctx ctx, const rpca_matrix* A, int k, int l,
                                size_t* bytes);

/* Randomized SVD / PCA, Section 2 (formulas (i1)-(i4) and (approx)) with the
 * renormalized power iteration of Sections 2 and 5: Y = A Omega, then ``its``
 * times Z = A* Q, Y = A Q, renormalizing by pivoted LU after every
 * application except the last, which is orthonormalized (QR); then
 * B = Q* A and its SVD.  Omega (n x l, Gaussian) is a pure function of
 * ``seed``: Philox4x32-10 stream 0.  With RPCA_CENTER the result is the PCA of
 * A - 1 c (c = column means) without forming it (Section 5).
 * Outputs: U (m x k, row-major, ldu >= k), S (k doubles, descending),
 * V (n x k, row-major, ldv >= k); U diag(S) V^T approximates A.  Columns of U
 * are signed so that the largest-magnitude entry is positive. */
rpca_status rpca_svd(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                     uint64_t seed, unsigned flags, float* U, int64_t ldu, double* S,
                     float* V, int64_t ldv);

/* rpca_svd for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same solve, kernels and results as rpca_svd, with the working memory taken
 * from a static device array of 64 MiB (the last 64 KiB hold the pivot
 * tournament's counters) that each GPU the library runs on holds until the
 * process ends, instead of the context's workspace.  The call allocates
 * nothing (no hipMalloc, hipFree or allocating library routine); the
 * context must already exist.  Its first call on a device looks up the
 * array's address there.  A problem whose working memory exceeds the array
 * (rpca_workspace_size minus the second tall buffer, roughly
 * 12 * max(m, n) * 32*ceil(l/32) bytes) returns RPCA_ERR_NO_MEMORY before
 * anything is launched.  Every call on one GPU shares that array and leaves
 * its contents behind: calls that overlap on one GPU (several streams or
 * contexts at once) race and must be serialized by the caller.  Timing
 * (rpca_set_timing) is not recorded for this call. */
rpca_status rpca_svd_noalloc(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                             uint64_t seed, unsigned flags, float* U, int64_t ldu, double* S,
                             float* V, int64_t ldv);

/* Shift-stabilized Nystrom method for a symmetric positive semidefinite n x n
 * A (Section 3, formulas (start)-(finish), after the self-adjoint core loop of
 * Section 5): U (n x k) and lambda (k, descending) with A ~ U diag(lambda) U*.
 * The shift is nu = sqrt(n) * u * ||A Q||_F, with u the unit roundoff of the
 * product B1 = A Q (2^-16 for a float32 A, whose products are three bfloat16
 * products of split operands; 2^-8 for a bfloat16 copy, 2^-4 for E4M3),
 * multiplied by 10 up to rpca_set_nystrom_retries times (default 10) while
 * the Cholesky factor does not exist.  Whether it was found is known on the
 * device only: like every device-side failure it is reported as
 * RPCA_ERR_NOT_PSD by the next synchronizing call on the context -- this one
 * with RPCA_SYNC, else rpca_sync -- and lambda, U are then not meaningful. */
rpca_status rpca_eig_psd(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                         uint64_t seed, unsigned flags, float* U, int64_t ldu,
                         double* lambda);

/* Rayleigh-Ritz eigenpairs of a general self-adjoint n x n A (positive,
 * negative or indefinite), after the self-adjoint core loop of Section 5
 * (A applied ``its`` times to Omega with renormalization, the last an
 * orthonormalization): B2 = Q* A Q = W diag(lambda) W*, U = Q W.  Returns the
 * k eigenpairs largest in magnitude: U (n x k) and lambda (k, signed,
 * ordered by |lambda| descending) with A ~ U diag(lambda) U*.  Flags as for
 * rpca_eig_psd (not RPCA_NYSTROM_SQRT).  With eigenvalues of equal magnitude
 * and opposite signs among the k, the pair's vectors are not separated. */
rpca_status rpca_eig_sym(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                         uint64_t seed, unsigned flags, float* U, int64_t ldu, double* lambda);

/* One problem of a batch (rpca_svd_batched).  kind 0: rpca_svd of A with
 * outputs U, S, V; kind 1: rpca_eig_psd of A with outputs U and S (the
 * eigenvalues), V unused.  ``flags`` takes RPCA_CENTER / RPCA_RENORM_ORTH.
 * All pointers are device memory owned by the caller, except ``A`` (host). */
typedef struct {
  int32_t kind, k, l, its;
  uint64_t seed;
  uint32_t flags;
  int32_t reserved; /* 0 */
  const rpca_matrix* A;
  float* U;
  int64_t ldu;
  double* S;
  float* V;
  int64_t ldv;
} rpca_problem;

/* Many independent solves in one call.  Every problem is checked before
 * anything is launched; device-side failures of single problems (a Nystrom
 * factor never found, non-finite values) are reported per problem by
 * rpca_batch_status and for the whole batch by the next synchronizing call
 * (RPCA_SYNC, rpca_sync), which returns RPCA_ERR_NOT_PSD, RPCA_ERR_NUMERICAL
 * or RPCA_ERR_TIMEOUT (below); the other problems' outputs are valid.
 *
 * Problems with a dense float32 A, m, n <= 8192 and l <= 64 are solved by one
 * persistent launch on the context stream: each workgroup of 512 threads
 * solves a whole problem (Sections 2, 3 and 5 with the same steps as the
 * single calls) and then takes the next one from a device counter, largest
 * problems first.  Its results equal the single calls' up to rounding (the
 * renormalizations pick other, equivalent bases).  Each call writes its
 * problem table to device memory on the stream (kernel arguments carry it, so
 * a captured graph replays its own table); the table, the work counter and
 * the working memory (one slot per workgroup, sized by the largest m or n)
 * belong to the context and are sized by uncaptured calls, which only grow
 * them (memory a larger buffer replaces is kept until rpca_destroy, for the
 * graphs that use it).  Calls that overlap on several streams share these
 * buffers and must not run at the same time.
 *
 * A problem whose single-workgroup time would set the batch's end (cost
 * model below) is split over up to 8 workgroups
 * (rpca_set_batch_split) that share its passes over A, its Gram matrices and
 * triangular solves by row ranges and meet at a device counter between the
 * steps; the split problems come first in the table and the launch has a
 * workgroup for each of their shares, so they run together.  A share that
 * waits too long (another kernel holding the device's compute units, e.g. a
 * second batched call on another stream) gives up, and the problem reports
 * RPCA_ERR_TIMEOUT.  Problems with the pivoted-LU renormalization are not
 * split.
 *
 * The other problems (sparse, bfloat16/E4M3 storage, larger sizes), and every
 * problem after rpca_set_batch_mode(ctx, 1), run the single-problem kernels
 * concurrently on up to rpca_set_batch_streams internal HIP streams (default
 * priority) forked from and joined back into the context stream; the results
 * then equal the single calls' bit for bit.  Each stream has its own
 * workspace and pivot counters.
 *
 * The call is ordered on the context stream like a single solve and can be
 * captured into a HIP graph there once an uncaptured call of the same batch
 * has sized the tables and workspaces (a capture that would need new ones
 * returns RPCA_ERR_UNSUPPORTED).  ``flags`` takes RPCA_SYNC and
 * RPCA_DETERMINISTIC (for every problem); RPCA_CENTER and RPCA_RENORM_ORTH
 * are per problem. */
rpca_status rpca_svd_batched(rpca_ctx ctx, int count, const rpca_problem* problems,
                             unsigned flags);

/* Per-problem outcome of the last rpca_svd_batched call on the context
 * (synchronizes): status_host[i] (host, count <= that call's count) is
 * RPCA_OK, RPCA_ERR_NUMERICAL (non-finite values), RPCA_ERR_NOT_PSD
 * (Nystrom factor never found) or RPCA_ERR_TIMEOUT (a problem split over
 * workgroups whose shares did not run together) for problem i, in the order
 * of the problems array.  Does not clear what rpca_sync reports. */
rpca_status rpca_batch_status(rpca_ctx ctx, int32_t count, int32_t* status_host);

/* Synchronize the context stream and report the device-side failures of the
 * solves issued on the context since the last synchronizing call:
 * RPCA_ERR_NUMERICAL when non-finite values were met (for instance a NaN or
 * infinity in A), else RPCA_ERR_NOT_PSD when a Nystrom factor was never found
 * (Section 3's shift retries exhausted), else RPCA_OK.  The report is then
 * cleared.  Every device loop is bounded, so such inputs end normally with
 * non-finite outputs. */
rpca_status rpca_sync(rpca_ctx ctx);

/* Number of times the Nystrom shift is multiplied by 10 before the solve is
 * reported as not PSD (0 .. 30, default 10). */
rpca_status rpca_set_nystrom_retries(rpca_ctx ctx, int32_t retries);

/* Randomized power-method estimate of ||A - U diag(S) V^T||_2 (Section 4),
 * in float64: ``iters`` steps of X <- orth(E^T E X) from a Gaussian n x 4
 * start block (Philox stream 1), estimate = ||E X||_2 <= ||E||_2.
 * V == NULL means the symmetric residual A - U diag(S) U^T.  RPCA_CENTER
 * measures against the column-centered A.  ``err_host`` is a host pointer;
 * the call synchronizes. */
rpca_status rpca_spectral_err(rpca_ctx ctx, const rpca_matrix* A, int k, const float* U,
                              int64_t ldu, const double* S, const float* V, int64_t ldv,
                              int iters, uint64_t seed, unsigned flags, double* err_host);

/* Precision preparation, once per matrix (not part of a solve).  A is float32
 * m x n row-major (device, leading dimension lda); ``out`` (device, leading
 * dimension ldo elements) receives
 *   RPCA_BF16:     bfloat16(a_ij), rounded to nearest even;
 *   RPCA_FP8_E4M3: E4M3(a_ij / s_j), rounded to nearest even, with
 *                  s_j = max_i |a_ij| / 448 (1 for a zero column) written to
 *                  col_scale (device, length n), so |a_ij / s_j| <= 448.
 * E4M3 is the OCP 8-bit format (bias 7, largest finite 448, no infinities).
 * Stream-ordered; uses the context workspace for the E4M3 column maxima. */
rpca_status rpca_quantize(rpca_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                          rpca_dtype dtype, void* out, int64_t ldo, float* col_scale);

/* The Gaussian test matrix alone: out[i*ldo + j] = z[j*n + i] for i < n,
 * j < l, where z is Philox4x32-10 stream ``stream`` under key ``seed`` mapped
 * through the Box-Muller transform (evaluated in float64, rounded to float32).
 * Exposed so that the generator can be checked against an independent
 * implementation.  ``words_out`` (may be NULL) receives the raw 32-bit words
 * of blocks 0 .. ceil(n*l/4)-1, four per block. */
rpca_status rpca_gaussian(rpca_ctx ctx, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                          float* out, int64_t ldo, uint32_t* words_out);

/* The uniform test matrix of RPCA_OMEGA_UNIFORM: out[i*ldo + j] = v[j*n + i],
 * v[e] = (x + 1/2) 2^-31 - 1 for the 32-bit word x number e of Philox4x32-10
 * stream ``stream`` under key ``seed`` (word e % 4 of block e / 4), formed
 * exactly in float64 and rounded once to float32. */
rpca_status rpca_uniform(rpca_ctx ctx, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                         float* out, int64_t ldo);

/* ---- single steps of the method, exposed for testing ------------------- */

/* Y = A X (trans = 0; X is n x l, Y is m x l) or Y = A^T X (trans = 1; X is
 * m x l, Y is n x l), float32 X/Y row-major, using the same kernels as the
 * solvers.  With RPCA_CENTER, A is replaced by A - 1 c. */
rpca_status rpca_op_matmul(rpca_ctx ctx, const rpca_matrix* A, int trans, int l,
                           const float* X, int64_t ldx, float* Y, int64_t ldy,
                           unsigned flags);
/* Renormalization of a tall r x l float32 matrix Y, in place.
 * kind = 0: pivoted LU (Q = P L, tournament pivoting), ``piv`` (may be NULL,
 *           device int32[l]) receives the pivot rows;
 * kind = 1: orthonormalization (Cholesky QR with float64 Gram matrices),
 *           ``R`` (may be NULL, device double[l*l], row-major) receives the
 *           upper triangular R with Y_in = Q R. */
rpca_status rpca_op_renorm(rpca_ctx ctx, int kind, int64_t rows, int l, float* Y, int64_t ldy,
                           int32_t* piv, double* R);
/* SVD of an l x l float64 matrix M (row-major, device): M = W diag(s) X^T
 * with s descending; W, X are l x l row-major (device). */
rpca_status rpca_op_small_svd(rpca_ctx ctx, int l, const double* M, double* s, double* W,
                              double* X);

/* ---- diagnostics -------------------------------------------------------- */

typedef struct {
  int64_t calls;          /* solver calls since the last reset               */
  int64_t a_passes;       /* passes over A launched                          */
  int64_t timed_launches; /* launches of the A-pass kernels that were timed  */
  double ms_ax;           /* total device time of Y = A X kernels (ms)        */
  double ms_atx;          /* total device time of A^T X kernels (ms)          */
  int64_t n_ax, n_atx;    /* number of timed launches of each                */
  double bytes_ax;        /* algorithmic bytes of the timed A X launches      */
  double bytes_atx;       /* algorithmic bytes of the timed A^T X launches    */
  int64_t shift_retries;  /* Nystrom shift retries of the last Nystrom solve  */
  /* the same for passes over a bfloat16 / E4M3 copy of A                    */
  double ms_ax_lp, ms_atx_lp;
  int64_t n_ax_lp, n_atx_lp;
  double bytes_ax_lp, bytes_atx_lp;
} rpca_stats;

/* Record HIP events around every A-pass kernel launch (on the context
 * stream) when ``enable`` is nonzero. */
rpca_status rpca_set_timing(rpca_ctx ctx, int enable);
/* Synchronizes the stream, folds the recorded events into the totals. */
rpca_status rpca_get_stats(rpca_ctx ctx, rpca_stats* out);
rpca_status rpca_reset_stats(rpca_ctx ctx);

/* Batched mode: 0 (default) solves the problems the persistent launch takes
 * there and the others on streams; 1 runs every problem on streams. */
rpca_status rpca_set_batch_mode(rpca_ctx ctx, int32_t mode);
/* Splitting of problems in the persistent launch: at most max_parts
 * workgroups per problem (1 .. 16; 1 splits nothing; default 8); at least
 * min_parts (1 .. max_parts; default 1, the cost model decides) for every
 * problem that can be split (not LU-renormalized, 64 rows of its smaller side
 * per share) as long as all shares fit in one round of the grid; and the
 * polls of a share waiting for the others before it gives up (spin_limit >
 * 0; 0 keeps the default of 2^22, about a second).  RPCA_ERR_INVALID_ARG
 * outside those ranges.
 *
 * The cost model: a problem takes about 0.45 ms + 0.167 ns x passes x m x n
 * + 1.21 ns x steps x (m + n) x lp on one workgroup (lp = 32 or 64; fitted
 * on this device), and 0.9 ms + the variable part / g as one of g shares.
 * Among a few split targets the host keeps the one whose simulated list
 * schedule (the shares first, then the rest by decreasing cost, each to the
 * first free workgroup) ends first. */
rpca_status rpca_set_batch_split(rpca_ctx ctx, int32_t max_parts, int32_t min_parts,
                                 int32_t spin_limit);

/* Number of HIP streams rpca_svd_batched spreads a batch over (1..64,
 * default 8; each has its own workspace).  How many of them run at once is
 * bounded by the hardware queues HIP gives the process (GPU_MAX_HW_QUEUES). */
rpca_status rpca_set_batch_streams(rpca_ctx ctx, int32_t streams);

/* ---- autotuner -----------------------------------------------------------
 * The float32 A-pass kernels and the LU pivot tournament have tile
 * configurations whose best choice depends on the shape: waves per workgroup
 * and LDS ring depth of Y = A X and of A^T X, and rows per tournament block.
 * rpca_tune times every candidate on the caller's dense A with l sketch
 * columns (one warm-up and ``reps`` timed launches each, reps < 1 means 3),
 * using the context's stream and workspace (A is only read; the call
 * synchronizes the stream), and keeps the fastest in the context's table
 * under the shape class of A: (ceil log2 m, ceil log2 n, l padded to
 * 32/64/128, dtype).  Later rpca_svd, rpca_eig_psd and rpca_svd_batched
 * calls on matrices of that class use it.  Only a float32 A has A-pass
 * alternatives; for a low-precision copy the tournament alone is tuned.
 * ``out`` (nullable) receives the choice and the average launch time of each
 * chosen configuration.  Sparse A: RPCA_ERR_UNSUPPORTED. */
typedef struct {
  int32_t ax_waves, ax_ring;    /* Y = A X: 4 or 8 waves of 32 rows and the ring
                                   stages, or 16 (ring 0) for the tall form: 8
                                   waves of 64 rows, the built-in choice when
                                   every CU gets 256 rows or more */
  int32_t atx_waves, atx_ring;  /* A^T X                                     */
  int32_t lu_rows;              /* rows per tournament block                 */
  int32_t candidates;           /* configurations timed                      */
  double ms_ax, ms_atx;         /* ms per launch (A^T X with its reduction)  */
  double ms_lu;                 /* ms per tournament, m side plus n side     */
} rpca_tune_result;
rpca_status rpca_tune(rpca_ctx ctx, const rpca_matrix* A, int32_t l, int32_t reps,
                      rpca_tune_result* out);
/* The table as text, one shape class a line:
 *   log2m log2n lp dtype ax_waves ax_ring atx_waves atx_ring lu_rows
 * (lines starting with '#' are comments).  Loading adds to the table and
 * replaces entries of the same class; a malformed line fails with
 * RPCA_ERR_INVALID_ARG and leaves the table as it was.  A loaded line also
 * picks the A X form of a bfloat16 or E4M3 copy (dtype 1, 2): ax_waves 16
 * the tall form, 4 the 4-wave form; other fields of such a line besides
 * lu_rows are ignored. */
rpca_status rpca_tune_save(rpca_ctx ctx, const char* path);
rpca_status rpca_tune_load(rpca_ctx ctx, const char* path);
rpca_status rpca_tune_clear(rpca_ctx ctx);
/* Number of shape classes in the table. */
rpca_status rpca_tune_count(rpca_ctx ctx, int32_t* count);

const char* rpca_status_str(rpca_status s);
const char* rpca_last_error(rpca_ctx ctx);

#ifdef __cplusplus
}
#endif
#endif /* RPCA_H */
