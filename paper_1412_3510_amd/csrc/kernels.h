// Internal launchers (host side) for the HIP kernels of the randomized PCA.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpca {

// ---- Philox Gaussian (philox.hip) -------------------------------------------
// uniform: each word mapped to (x + 1/2) 2^-31 - 1 instead of Box-Muller
void launch_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                     float* out, int64_t ldo, uint32_t* words, bool uniform = false);

// ---- dense products (gemm.hip) ----------------------------------------------
// Fragment-ordered bfloat16 (hi, lo) copy of a tall float32 matrix, used as
// the small operand of both products.  ``nsteps`` 16-row steps are written
// (rows past ``rows`` are zero); ``mu`` (nullable, float[cols]) is subtracted
// from every valid row first; ``rscale`` (nullable, float[rows]) multiplies
// row r.
size_t packed_bytes(int64_t nsteps, int nb);
void launch_pack(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int cols, int nb,
                 const float* mu, const float* rscale, __bf16* out, int64_t nsteps);

// Tile configuration of the float32 A-pass kernels and of the LU tournament
// (0: the built-in choice).  The autotuner (rpca_tune) picks it per shape
// class; the launchers fall back to the built-in choice for values they do
// not support.
struct TuneCfg {
  int ax_waves = 0;   // Y = A X: 4 or 8 waves of 32 rows (8: lp = 64 or 128), or
                      // 16 for the tall form (8 waves of 64 rows, ax_tall.hip)
  int ax_ring = 0;    // LDS ring stages of the 4-wave form: 2, 3 or 4
  int atx_waves = 0;  // the same for A^T X
  int atx_ring = 0;
  int lu_rows = 0;    // rows per tournament block: 256, 512 or 1024 (lp <= 64)
};

// Y (m x 32*nb) = A (m x n) X, X packed with >= 2*ceil(n/32) steps.
void launch_ax(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
               const __bf16* Xp, float* Y, int64_t ldy, int nb, int num_cus,
               const TuneCfg* cfg = nullptr);
// the (waves, ring) pairs launch_ax and launch_atx can run for nb (the
// autotuner's candidates)
int ax_candidates(int nb, int (*out)[2]);
int atx_candidates(int nb, int (*out)[2]);
// Y = A X in the tall form (any dtype, nb 1, 2 or 4; the layout rules of the
// LDS-DMA kernels), and whether it is the built-in choice for m rows
void launch_ax_tall(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                    const __bf16* Xp, float* Y, int64_t ldy, int nb, int num_cus);
bool ax_tall_ok(int64_t m, int num_cus);
// whether float32 A in this layout takes the LDS-DMA kernels (which have the
// configurations above)
bool dma_ok_shape(const void* A, int64_t lda, int64_t n);

// Split-K partial products of A^T X (X packed on the m side).
struct AtxPlan {
  int ntiles;        // ceil(n / 128): the partials hold 4 * ntiles 32-column blocks per split
  int waves;         // waves per workgroup of the DMA kernel (4 or 8), or 16 for the
                     // wide form of a low-precision copy (8 waves, 512-column tiles)
  int ring;          // its LDS ring stages
  int gtiles;        // column tiles of that kernel, ceil(n / (32 * waves))
  int nsplit;        // number of row splits
  int64_t rows_per;  // rows per split (multiple of 32)
  size_t partial_bytes;
};
// dtype: 0 float32, 1 bfloat16, 2 E4M3 (the copy of A the pass reads)
AtxPlan plan_atx(int64_t m, int64_t n, int nb, int num_cus, int dtype,
                 const TuneCfg* cfg = nullptr);
// largest partial buffer over every configuration plan_atx can choose
size_t atx_partial_bytes_max(int64_t m, int64_t n, int nb, int num_cus, int dtype);
void launch_atx(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                const __bf16* Xp, float* P, const AtxPlan& plan, int nb);
// Z (n x 32*nb) = sum of the partials (fixed order); ``cscale`` (nullable,
// float[n]) multiplies row j of Z.
void launch_atx_reduce(hipStream_t st, const float* P, const AtxPlan& plan, int nb, int64_t n,
                       const float* cscale, float* Z, int64_t ldz);

// ---- passes over a bfloat16 / E4M3 copy of A (gemm_lp.hip) -------------------
// Shape rule of the low-precision kernels: n and lda multiples of 16 bytes of
// elements, A 16-byte aligned.
bool lp_shape_ok(const void* A, int dtype, int64_t lda, int64_t n);
int lp_rows_per_stage(int dtype);
int lp_per_cu(int nb, int dtype);
// whether the low-precision kernels have their 8-wave (256-row / 256-column
// tile) form for this nb and dtype
bool lp_atx_can8(int nb, int dtype);
// cfg (nullable): ax_waves 16 or 4 forces the tall or the 4-wave form
void launch_ax_lp(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                  const __bf16* Xp, float* Y, int64_t ldy, int nb, int num_cus,
                  const TuneCfg* cfg = nullptr);
void launch_atx_lp(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                   const __bf16* Xp, float* P, const AtxPlan& plan, int nb);
// the wide form (atx_wide.hip): rows per stage, and the launch
int atx_wide_rows_per_stage(int dtype);
void launch_atx_wide(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                     const __bf16* Xp, float* P, const AtxPlan& plan, int nb);
// float32 A -> bfloat16 (dtype 1) or E4M3 with column scales (dtype 2)
size_t quantize_work_bytes(int64_t m, int64_t n);
void launch_quantize(hipStream_t st, const float* A, int64_t lda, int64_t m, int64_t n, int dtype,
                     void* out, int64_t ldo, float* scale, float* work);

// ---- sparse A (sparse.hip) -----------------------------------------------------
// Y[i][:lp] = sum over k in [ptr[i], ptr[i+1]) of val[k] X[idx[k]][:lp]
// (CSR of A for A X, CSC of A = CSR of A^T for A^T X); dtype 0 float32, 1 bf16
void launch_spmm(hipStream_t st, const int* ptr, const int* idx, const void* val, int dtype,
                 int64_t nrows, int64_t nnz, int ncols, const float* X, int64_t ldx, float* Y,
                 int64_t ldy, int lp);
// the same with X, Y rows of 4 float64 (power-method blocks)
void launch_spmm4_f64(hipStream_t st, const int* ptr, const int* idx, const void* val, int dtype,
                      int64_t nrows, int64_t nnz, int ncols, const double* X, double* Y);

// ---- tall-skinny helpers (tall.hip)
// p[0 .. count) = 0 and dst[0 .. count) = src[...]; count a multiple of 4,
// pointers 16-byte aligned (kernel nodes only, for graph capture)
void launch_fill_zero(hipStream_t st, float* p, int64_t count);
void launch_copy(hipStream_t st, float* dst, const float* src, int64_t count);
// mu[c] = mean over rows of X[:, c] for c < cols (float64 accumulation).
void launch_colmean(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int cols,
                    double* partial, int nblk_max, float* mu);
int colmean_blocks(int64_t rows);
// X[r, c] -= mu[c]
void launch_sub_rowvec(hipStream_t st, float* X, int64_t ldx, int64_t rows, int cols,
                       const float* mu);
// Gram G = X^T X2 (float64; X2 = X when null), in two stages.  ``partial``
// holds gram_blocks(rows)*lp*lp doubles.  Skipped when *skip_flag == 0.
int gram_blocks(int64_t rows);
void launch_gram(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int lp,
                 const float* X2, int64_t ldx2, double* partial, double* G,
                 const int* skip_flag);
// fro2[0] = sum of squares of X (float64); psum/psq hold colmean_blocks(rows)*128 doubles
void launch_fro2_d(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int cols,
                   double* psum, double* psq, double* fro2);
// In-place right triangular solve X <- X U^-1 (U upper, float32, lp x lp),
// with the pivoted-LU convention for zero pivots (see tall.hip).
void launch_trsm(hipStream_t st, float* X, int64_t ldx, int64_t rows, int l, int lp,
                 const float* Ut, const int* piv, const int* skip_flag, const float* nu,
                 const float* addX, int64_t ldadd, int num_cus);
// Y (rows x k) = X (rows x lp) W (lp x k, float64, row-major ld ldw)
void launch_small_gemm(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int l,
                       const double* W, int ldw, int k, float* Y, int64_t ldy, int num_cus);
// Sign convention: flip columns of U (and V) so the largest-|.| entry of each
// U column is positive.  ``work`` holds sign_work_bytes(m) bytes.
size_t sign_work_bytes(int64_t m);
void launch_sign_fix(hipStream_t st, float* U, int64_t ldu, int64_t m, int k, float* V,
                     int64_t ldv, int64_t n, int* work);

// ---- pivoted LU by tournament (lu.hip) ---------------------------------------
struct LuPlan {
  int lp;
  int rows;            // rows per tournament block
  int levels;
  int nblk[16];        // blocks at each level (level 0 = leaves)
  int64_t cand_off[16];
  int64_t cand_total;  // ints
  int64_t counter_total;
};
// block_rows: 256, 512 or 1024 (lp <= 64); anything else takes 512
LuPlan plan_lu(int64_t rows, int lp, int block_rows = 0);
// Tournament pivoting over rows of X; writes the root's U (lp x lp float32,
// row-major), the pivot rows piv[l] and zero-pivot markers (U[j][j] == 0).
void launch_lu_tree(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int l,
                    const LuPlan& plan, int* cand, unsigned* counters, float* U, int* piv);

// ---- small dense float64 kernels (small.hip) ---------------------------------
// One Cholesky-QR step on the Gram G (lp x lp): upper R as float32 ``Rf``
// for the solve.  Pass 1 always runs; pass 2 too unless ``cond2``, which
// runs it only when pass 1 had to shift (state[0]); passes 3 and 4 only when
// state[1] is set (a shifted factorization or dependent columns met).  See
// small_core.h for ``state``.
void launch_chol_qr_step(hipStream_t st, const double* G, int l, int lp, int pass, float* Rf,
                         int* state, bool cond2 = false);
// Replace the dependent columns flagged in ``state`` by Gaussian columns.
void launch_complete(hipStream_t st, float* Q, int64_t ldq, int64_t rows, int l, const int* state,
                     uint64_t seed);
// Nystrom: B2 = sym(G) + nu I with nu = n_sqrt_u * sqrt(fro2[0]), Cholesky
// with nu <- 10 nu retries; writes C (float32 upper), nu (double and float).
void launch_chol_nystrom(hipStream_t st, const double* G, int l, int lp, const double* fro2,
                         double n_sqrt_u, float* Rf, double* nu_out, float* nu_f, int* state,
                         int max_retries);
// One-sided Jacobi SVD of M (l x l, float64 row-major ld lp) or of M^T:
// s (descending), Wacc (accumulated rotations, columns sorted), Xn
// (normalized columns of M Wacc, sorted).  ``work`` holds 2*lp*lp doubles.
// ``flag`` (device int, nullable): at lp = 128 the form without accumulated
// rotations (columns in LDS) runs first and the accumulating form (global
// memory) only when the ``kneed`` largest singular values (the columns of
// Wacc the caller reads) are too spread for its recovery of the rotations.
void launch_jacobi_svd(hipStream_t st, const double* M, int l, int lp, int transpose, double* s,
                       double* Wacc, double* Xn, double* work, int* flag = nullptr,
                       int kneed = 0);
// out[j] = s[j] (nu null) or max(s[j]^2 - nu, 0), j < k.  The solve's status
// (non-finite values; for Nystrom, no factor found) is OR-ed into status[0]
// and written to *slot; status[1] gets the Nystrom retry count (state,
// status and slot nullable; see small_core.h for the bits).
void launch_finish_values(hipStream_t st, const double* s, int k, const double* nu, double* out,
                          const int* state, int* status, int* slot);

// Self-adjoint variants: G <- (G + G^T)/2; the pseudoinverse factor
// M = W diag(s^-1/2) over the s_j above n_sqrt_u * sqrt(fro2[0]) (Section 3,
// square-root stabilization); eigenvalues lambda_j = s_j sign(w_j . x_j) of a
// symmetric matrix from its SVD (out[j], j < k), with the solve's status.
void launch_symmetrize(hipStream_t st, double* G, int l, int lp);
void launch_sqrt_pinv(hipStream_t st, const double* W, const double* s, int l, int lp,
                      const double* fro2, double n_sqrt_u, double* M);
void launch_sym_eig_finish(hipStream_t st, const double* s, const double* W, const double* X, int l,
                           int k, int lp, double* out, const int* state, int* status, int* slot);

// ---- spectral-norm estimate (spectral.hip) -------------------------------------
// a sparse A for the error estimate: CSR (ptr, idx, val) and CSC (ptr_t, ...)
struct SpecSparse {
  const int *ptr, *idx;
  const void* val;
  const int *ptr_t, *idx_t;
  const void* val_t;
  int dtype;
  int64_t nnz;
};
void launch_spectral(hipStream_t st, const float* A, int64_t lda, int64_t m, int64_t n, bool center,
                     const float* U, int64_t ldu, const double* S, const float* V, int64_t ldv,
                     int k, int iters, uint64_t seed, void* work, double* result,
                     const SpecSparse* sp);
size_t spectral_work_bytes(int64_t m, int64_t n, int k);

// ---- persistent batched solver (batch.hip) --------------------------------------
// One problem of the persistent launch (float32 A, row-major; all pointers
// device memory).  kind 0: randomized SVD (center: of the column-centered A);
// kind 1: Nystrom for a PSD A (m == n).  mid: the renormalization between
// applications -- 0 one Cholesky QR pass (repaired when it needs a shift),
// 1 pivoted LU, 2 the two-pass orthonormalization.
struct PersProblem {
  const float* A;
  int64_t lda;
  float* U;
  int64_t ldu;
  double* S;
  float* V;
  int64_t ldv;
  uint64_t seed;
  int32_t m, n, kind, k, l, its, center, mid;
  int32_t uniform;  // uniform test matrix (Section 5) instead of the Gaussian one
  int32_t parts;    // workgroups that share the problem (1: one workgroup solves it)
  int32_t part;     // this entry's share, 0 .. parts - 1
  int32_t pad_;
  int* status;   // the problem's status entry (bits of small_core.h), nullable
  int* gstatus;  // the caller's status word: [0] OR of the bits, [1] Nystrom retries
  float* sh;     // parts > 1: the problem's shared buffers (team_floats floats)
  int* bar;      // parts > 1: the team's arrival counter, zero at launch
};
static constexpr int kPersMaxDim = 8192;  // largest m, n
static constexpr int kPersMaxL = 64;      // largest l
static constexpr int kPersMaxParts = 16;  // most workgroups on one problem
// Floats of the shared buffers of a problem split over ``parts`` workgroups
// (rows: pers_rows of its larger dimension; np: n rounded up to 64): Y, Z, T
// and the packed operand (rows x 64 each), the A^T X partials (parts x np x
// 64), two sets of Gram partials (parts x 64 x 64 doubles) and of vector
// partials (parts x 64 doubles), and the sign keys and signs (parts x 128 x
// 8 bytes).
inline int64_t team_floats(int parts, int64_t rows, int64_t np) {
  return 4 * rows * 64 + (int64_t)parts * np * 64 + 2 * 2 * (int64_t)parts * (4096 + 64) +
         4 * (int64_t)parts * 64;
}
// rows of each slot buffer and floats per workgroup slot for problems up to maxdim
int64_t pers_rows(int64_t maxdim);
int64_t pers_slot_floats(int64_t maxdim);
// write ``count`` entries of the problem table to ``dev`` on the stream (kernel
// arguments carry the host entries, so the copy is graph-capturable)
void launch_pers_table(hipStream_t st, const PersProblem* host, int count, PersProblem* dev);
// ``count`` problems (device table) over ``grid`` workgroups; ``counter`` (device int,
// zero at launch) hands out the problems; ``ws`` holds grid * pers_slot_floats floats.
// max_retries: Nystrom shift retries before a problem is reported not PSD
// spin_limit: polls of a team's arrival counter before a workgroup gives up
// waiting (the problem then reports kErrTimeout)
void launch_persistent(hipStream_t st, const PersProblem* probs, int count, int* counter,
                       float* ws, int64_t maxdim, int grid, int max_retries, int spin_limit);

}  // namespace rpca
