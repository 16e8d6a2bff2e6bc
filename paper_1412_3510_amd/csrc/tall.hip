// Kernels on tall-skinny float32 matrices (rows x lp, lp = 32, 64 or 128,
// padding columns zero): column statistics for centering, the float64 Gram
// matrix for Cholesky QR, the right triangular solve shared by the LU and
// Cholesky-QR renormalizations and the Nystrom F = B1 C^-1, and the small
// products U = Q W of the final step.
#include "common.h"
#include "kernels.h"

namespace rpca {

// ------------------------------------------------------------------------
// column sums and sums of squares, float64 partials per row chunk
// ------------------------------------------------------------------------
static constexpr int kColChunk = 128;

int colmean_blocks(int64_t rows) { return (int)ceil_div(rows > 0 ? rows : 1, kColChunk); }

__global__ void __launch_bounds__(256) colstats_kernel(const float* __restrict__ X, int64_t ldx,
                                                       int64_t rows, int cols,
                                                       double* __restrict__ psum,
                                                       double* __restrict__ psq) {
  // thread -> (column c, row phase); 256 threads cover 256/ cpw columns
  const int cpw = (cols <= 32) ? 32 : (cols <= 64 ? 64 : 128);
  const int ph = 256 / cpw;
  const int c = threadIdx.x % cpw, p = threadIdx.x / cpw;
  const int64_t r0 = (int64_t)blockIdx.x * kColChunk;
  double s = 0.0, q = 0.0;
  if (c < cols) {
    const int64_t r1 = min(rows, r0 + kColChunk);
    double s1 = 0.0, q1 = 0.0;
    int64_t r = r0 + p;
    for (; r + ph < r1; r += 2 * ph) {  // two rows in flight per thread
      const double v = X[r * ldx + c], w = X[(r + ph) * ldx + c];
      s += v;
      q += v * v;
      s1 += w;
      q1 += w * w;
    }
    if (r < r1) {
      const double v = X[r * ldx + c];
      s += v;
      q += v * v;
    }
    s += s1;
    q += q1;
  }
  __shared__ double ss[256], sq[256];
  ss[threadIdx.x] = s;
  sq[threadIdx.x] = q;
  __syncthreads();
  if (p == 0 && c < cols) {
    for (int k = 1; k < ph; ++k) {
      s += ss[k * cpw + c];
      q += sq[k * cpw + c];
    }
    psum[(int64_t)blockIdx.x * 128 + c] = s;
    if (psq) psq[(int64_t)blockIdx.x * 128 + c] = q;
  }
}

// out[e] = scale * sum_b part[b * stride + e] for e < E.  A workgroup owns 64
// consecutive e; its sixteen waves split the b range (b = ph + 16 j, four
// loads in flight), then combine in LDS in a fixed order.
static constexpr int kRedWaves = 16;

__global__ void __launch_bounds__(64 * kRedWaves) reduce_partials_kernel(
    const double* __restrict__ part, int nblk, int64_t stride, int E, double scale,
    double* __restrict__ out_d, float* __restrict__ out_f, const int* __restrict__ skip_flag) {
  if (skip_flag && *skip_flag == 0) return;
  __shared__ double sh[kRedWaves][64];
  const int el = threadIdx.x & 63, ph = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + el;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
  if (e < E) {
    int b = ph;
    constexpr int W = kRedWaves;
    for (; b + 3 * W < nblk; b += 4 * W) {
      double v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = part[(int64_t)(b + W * u) * stride + e];
#pragma unroll
      for (int u = 0; u < 4; ++u) acc[u] += v[u];
    }
    for (; b < nblk; b += W) acc[0] += part[(int64_t)b * stride + e];
  }
  sh[ph][el] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
  __syncthreads();
  if (ph == 0 && e < E) {
    double s = 0.0;
#pragma unroll
    for (int w = 0; w < kRedWaves; ++w) s += sh[w][el];
    s *= scale;
    if (out_d) out_d[e] = s;
    if (out_f) out_f[e] = (float)s;
  }
}

static void launch_reduce(hipStream_t st, const double* part, int nblk, int64_t stride, int E,
                          double scale, double* out_d, float* out_f, const int* skip_flag) {
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)ceil_div(E, 64)), dim3(64 * kRedWaves),
                     0, st, part, nblk, stride, E, scale, out_d, out_f, skip_flag);
}

void launch_colmean(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int cols,
                    double* partial, int nblk_max, float* mu) {
  const int nblk = colmean_blocks(rows);
  (void)nblk_max;
  hipLaunchKernelGGL(colstats_kernel, dim3(nblk), dim3(256), 0, st, X, ldx, rows, cols, partial,
                     (double*)nullptr);
  launch_reduce(st, partial, nblk, 128, cols, 1.0 / (double)rows, nullptr, mu, nullptr);
}

__global__ void __launch_bounds__(256) sub_rowvec_kernel(float* __restrict__ X, int64_t ldx,
                                                         int64_t rows, int cols,
                                                         const float* __restrict__ mu) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = e / cols;
  const int c = (int)(e % cols);
  if (r < rows) X[r * ldx + c] -= mu[c];
}

void launch_sub_rowvec(hipStream_t st, float* X, int64_t ldx, int64_t rows, int cols,
                       const float* mu) {
  const int64_t total = rows * cols;
  if (total == 0) return;
  hipLaunchKernelGGL(sub_rowvec_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, X,
                     ldx, rows, cols, mu);
}

// sum of squares of all entries (float64) -> fro2[0]; colsq holds 128 doubles
__global__ void sum_cols_kernel(const double* __restrict__ colsq, int cols,
                                double* __restrict__ fro2) {
  __shared__ double sh[128];
  const int c = threadIdx.x;
  sh[c] = (c < cols) ? colsq[c] : 0.0;
  __syncthreads();
  if (c == 0) {
    double t = 0.0;
    for (int i = 0; i < 128; ++i) t += sh[i];
    fro2[0] = t;
  }
}

void launch_fro2_d(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int cols,
                   double* psum, double* psq, double* fro2) {
  const int nblk = colmean_blocks(rows);
  hipLaunchKernelGGL(colstats_kernel, dim3(nblk), dim3(256), 0, st, X, ldx, rows, cols, psum, psq);
  // per-column sums of squares into psum[0..127] (psum's partials are not needed)
  launch_reduce(st, psq, nblk, 128, cols, 1.0, psum, nullptr, nullptr);
  hipLaunchKernelGGL(sum_cols_kernel, dim3(1), dim3(128), 0, st, psum, cols, fro2);
}

// ------------------------------------------------------------------------
// Gram matrix G = X^T X2 in float64 (X2 = X when null).  The rows are split
// into at most kGramMaxBlocks equal contiguous ranges, one workgroup each
// (about one per CU).  A workgroup has NG groups of 256 threads (NG = 4 for
// tall inputs, so that four slices of loads are in flight per CU, else 1);
// within a group a 16 x 16 grid of threads owns T x T tiles of the lp x lp
// result (T = lp / 16).  The range is walked in slices of 32 rows, slice s
// going to group s % NG; a slice is widened to float64 once in LDS, and the
// next one is loaded into registers while the current one is used.  At the
// end the groups' sums are added in LDS in group order.  Products of float32
// values are exact in float64.
// ------------------------------------------------------------------------
static constexpr int kGramMaxBlocks = 256;
static constexpr int kGramSlice = 32;

template <int LP, int NG>
struct GramCfg {
  static constexpr int STAGE = 2 * kGramSlice * LP;  // doubles per group (X and X2 slices)
  static constexpr int COMB = (NG - 1) * LP * LP;    // doubles for the combination
  static constexpr int SHARED = NG * STAGE > COMB ? NG * STAGE : COMB;
};

static int gram_grid(int64_t rows, int ng) {
  const int64_t b = ceil_div(rows > 0 ? rows : 1, (int64_t)kGramSlice * ng);
  return (int)(b < kGramMaxBlocks ? b : kGramMaxBlocks);
}

int gram_blocks(int64_t rows) { return gram_grid(rows, 1); }  // an upper bound for any lp

template <int LP, int NG>
__global__ void __launch_bounds__(256 * NG) gram_kernel(const float* __restrict__ X, int64_t ldx,
                                                        const float* __restrict__ X2,
                                                        int64_t ldx2, int64_t rows,
                                                        double* __restrict__ partial,
                                                        const int* __restrict__ skip_flag) {
  if (skip_flag && *skip_flag == 0) return;
  constexpr int T = LP / 16;
  constexpr int PER = kGramSlice * LP / 256;  // values per thread per slice
  __shared__ __attribute__((aligned(16))) double sh[GramCfg<LP, NG>::SHARED];
  const int g = threadIdx.x >> 8, tid = threadIdx.x & 255, ti = tid >> 4, tj = tid & 15;
  const bool same = (X2 == nullptr);
  double* sa = sh + g * GramCfg<LP, NG>::STAGE;
  double* sb = same ? sa : sa + kGramSlice * LP;
  const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  double acc[T][T];
#pragma unroll
  for (int a = 0; a < T; ++a)
#pragma unroll
    for (int b = 0; b < T; ++b) acc[a][b] = 0.0;
  float pa[PER], pb[PER];
  auto load = [&](int64_t rc) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q, rr = e / LP, c = e % LP;
      const int64_t r = rc + rr;
      pa[q] = (r < r1) ? X[r * ldx + c] : 0.f;
      if (!same) pb[q] = (r < r1) ? X2[r * ldx2 + c] : 0.f;
    }
  };
  constexpr int64_t kStep = (int64_t)kGramSlice * NG;
  load(r0 + g * kGramSlice);
  for (int64_t rb = r0; rb < r1; rb += kStep) {
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int e = tid + 256 * q, rr = e / LP, c = e % LP;
      sa[rr * LP + c] = (double)pa[q];
      if (!same) sb[rr * LP + c] = (double)pb[q];
    }
    __syncthreads();
    if (rb + kStep < r1) load(rb + kStep + g * kGramSlice);
    for (int rr = 0; rr < kGramSlice; ++rr) {
      double a[T], b[T];
#pragma unroll
      for (int u = 0; u < T; u += 2) {
        const double2 va = *reinterpret_cast<const double2*>(&sa[rr * LP + ti * T + u]);
        const double2 vb = *reinterpret_cast<const double2*>(&sb[rr * LP + tj * T + u]);
        a[u] = va.x; a[u + 1] = va.y;
        b[u] = vb.x; b[u + 1] = vb.y;
      }
#pragma unroll
      for (int u = 0; u < T; ++u)
#pragma unroll
        for (int v = 0; v < T; ++v) acc[u][v] += a[u] * b[v];
    }
    __syncthreads();
  }
  if constexpr (NG > 1) {
    if (g > 0) {
      double* cb = sh + (g - 1) * LP * LP;
#pragma unroll
      for (int u = 0; u < T; ++u)
#pragma unroll
        for (int v = 0; v < T; ++v) cb[(ti * T + u) * LP + tj * T + v] = acc[u][v];
    }
    __syncthreads();
    if (g > 0) return;
#pragma unroll
    for (int h = 0; h < NG - 1; ++h)
#pragma unroll
      for (int u = 0; u < T; ++u)
#pragma unroll
        for (int v = 0; v < T; ++v) acc[u][v] += sh[h * LP * LP + (ti * T + u) * LP + tj * T + v];
  }
  double* out = partial + (int64_t)blockIdx.x * LP * LP;
#pragma unroll
  for (int u = 0; u < T; ++u)
#pragma unroll
    for (int v = 0; v < T; ++v) out[(ti * T + u) * LP + tj * T + v] = acc[u][v];
}

// The same Gram matrix on the float64 matrix cores (lp = 32, 64):
// v_mfma_f64_16x16x4f64 takes a 16 x 4 block of X^T and a 4 x 16 block of
// X2, lane L holding row r + L / 16 of both, and lane L's register q of the
// 16 x 16 result is entry (L / 16 + 4 q, L % 16).  Tile t of each dimension
// holds the columns T i + t (i = 0..15, T = lp / 16), so lane L's T entries
// of a row -- columns T (L % 16) .. T (L % 16) + T - 1 -- are contiguous and
// come in one 8- or 16-byte load, and result entry (i, j) of tile pair
// (ti, tj) is G[T i + ti][T j + tj].  A wave accumulates the T^2 tile pairs
// (those with ti <= tj when X2 = X: the rest follow by symmetry) over 4-row
// groups of its rows, U groups in flight; the waves of the workgroup then
// add their tiles in LDS in wave order (8 waves at lp = 32, 4 at lp = 64,
// where the wider tiles already keep the loads in flight).  Products of
// float32 values are exact in float64 and every sum is in float64, as in
// gram_kernel; only the order of the additions differs.
template <int LP>
__host__ __device__ constexpr int gram_waves() { return LP == 32 ? 8 : 4; }

template <int T>
__device__ __forceinline__ void gram_load_row(const float* __restrict__ p, bool ok, double* out) {
  if constexpr (T == 2) {
    const float2 v = *reinterpret_cast<const float2*>(p);
    out[0] = ok ? (double)v.x : 0.0;
    out[1] = ok ? (double)v.y : 0.0;
  } else {
#pragma unroll
    for (int h = 0; h < T / 4; ++h) {
      const float4 v = *reinterpret_cast<const float4*>(p + 4 * h);
      out[4 * h + 0] = ok ? (double)v.x : 0.0;
      out[4 * h + 1] = ok ? (double)v.y : 0.0;
      out[4 * h + 2] = ok ? (double)v.z : 0.0;
      out[4 * h + 3] = ok ? (double)v.w : 0.0;
    }
  }
}

template <int LP, bool SAME>
__global__ void __launch_bounds__(64 * gram_waves<LP>()) gram_mfma_kernel(
    const float* __restrict__ X, int64_t ldx, const float* __restrict__ X2, int64_t ldx2,
    int64_t rows, double* __restrict__ partial, const int* __restrict__ skip_flag) {
  if (skip_flag && *skip_flag == 0) return;
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int kGramWaves = gram_waves<LP>();
  constexpr int T = LP / 16;
  constexpr int NT2 = SAME ? T * (T + 1) / 2 : T * T;  // tiles a wave accumulates
  constexpr int U = 4;                                 // 4-row groups per step (loads in flight)
  __shared__ double sh[LP * LP];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane >> 4, lc = lane & 15;
  const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  d4 acc[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  const float* X2p = SAME ? X : X2;
  const int64_t ld2 = SAME ? ldx : ldx2;
  // wave w takes the 4-row groups w, w + W, w + 2 W, ... of the range
  for (int64_t g0 = r0 + 4 * wave; g0 < r1; g0 += 4 * kGramWaves * U) {
    double a[U][T], b[U][T];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = g0 + 4 * kGramWaves * u + lr;
      const bool ok = r < r1;
      const int64_t rc = ok ? r : r0;
      gram_load_row<T>(X + rc * ldx + T * lc, ok, a[u]);
      if (!SAME) gram_load_row<T>(X2p + rc * ld2 + T * lc, ok, b[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < T; ++ti)
#pragma unroll
        for (int tj = SAME ? ti : 0; tj < T; ++tj) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][ti], SAME ? a[u][tj] : b[u][tj],
                                                        acc[t], 0, 0, 0);
          ++t;
        }
    }
  }
  // the waves' tiles added in LDS in wave order (entry (i, j) of G at i * LP + j)
  for (int w = 0; w < kGramWaves; ++w) {
    if (wave == w) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < T; ++ti)
#pragma unroll
        for (int tj = SAME ? ti : 0; tj < T; ++tj) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = T * (lr + 4 * q) + ti, j = T * lc + tj;
            const double v = (w == 0) ? acc[t][q] : sh[i * LP + j] + acc[t][q];
            sh[i * LP + j] = v;
            if (SAME && ti != tj) sh[j * LP + i] = v;
          }
          ++t;
        }
    }
    __syncthreads();
  }
  double* out = partial + (int64_t)blockIdx.x * LP * LP;
  for (int e = threadIdx.x; e < LP * LP; e += 64 * kGramWaves) out[e] = sh[e];
}

// lp = 128 on the matrix cores: the 36 upper tiles (64 without symmetry)
// are dealt to the four waves in order, 9 (16) each; every wave walks all
// the workgroup's 4-row groups for its own tiles (the four waves read the
// same rows, mostly from L1) and writes its tiles, and their mirror images,
// straight to the workgroup's partial.  As at lp = 32 and 64, tile t holds
// the columns 8 i + t, so a lane reads its 8 entries of a row as two 16-byte
// loads.  A wave's tiles are compile-time constants (one instantiation per
// wave), so its operands are plain registers.
// upper tiles (ti <= tj) of the 8 x 8 tile grid in row order
__device__ constexpr int kG128Ti[36] = {0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1, 1, 1, 2, 2, 2, 2, 2, 2, 3, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5, 5, 6, 6, 7};
__device__ constexpr int kG128Tj[36] = {0, 1, 2, 3, 4, 5, 6, 7, 1, 2, 3, 4, 5, 6, 7, 2, 3, 4, 5, 6, 7, 3, 4, 5, 6, 7, 4, 5, 6, 7, 5, 6, 7, 6, 7, 7};
template <bool SAME>
__device__ __forceinline__ constexpr int g128_ti(int t) { return SAME ? kG128Ti[t] : t / 8; }
template <bool SAME>
__device__ __forceinline__ constexpr int g128_tj(int t) { return SAME ? kG128Tj[t] : t % 8; }

template <bool SAME, int W>
__device__ __forceinline__ void gram128_wave(const float* __restrict__ X, int64_t ldx,
                                             const float* __restrict__ X2, int64_t ld2,
                                             int64_t r0, int64_t r1, double* __restrict__ out) {
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int LP = 128, T = 8;
  constexpr int NTOT = SAME ? T * (T + 1) / 2 : T * T, PER = NTOT / 4;
  constexpr int U = SAME ? 4 : 2;  // 4-row groups per step (loads in flight)
  static_assert(PER * 4 == NTOT, "tiles per wave");
  const int lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
  d4 acc[PER];
#pragma unroll
  for (int t = 0; t < PER; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  for (int64_t g0 = r0; g0 < r1; g0 += 4 * U) {
    double a[U][T], b[U][T];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t r = g0 + 4 * u + lr;
      const bool ok = r < r1;
      const int64_t rc = ok ? r : r0;
      gram_load_row<T>(X + rc * ldx + T * lc, ok, a[u]);
      if constexpr (!SAME) gram_load_row<T>(X2 + rc * ld2 + T * lc, ok, b[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int ti = g128_ti<SAME>(W * PER + k), tj = g128_tj<SAME>(W * PER + k);
        acc[k] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][ti], SAME ? a[u][tj] : b[u][tj],
                                                      acc[k], 0, 0, 0);
      }
  }
#pragma unroll
  for (int k = 0; k < PER; ++k) {
    const int ti = g128_ti<SAME>(W * PER + k), tj = g128_tj<SAME>(W * PER + k);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = T * (lr + 4 * q) + ti, j = T * lc + tj;
      out[i * LP + j] = acc[k][q];
      if (SAME && ti != tj) out[j * LP + i] = acc[k][q];
    }
  }
}

template <bool SAME>
__global__ void __launch_bounds__(256) gram_mfma128_kernel(
    const float* __restrict__ X, int64_t ldx, const float* __restrict__ X2, int64_t ldx2,
    int64_t rows, double* __restrict__ partial, const int* __restrict__ skip_flag) {
  if (skip_flag && *skip_flag == 0) return;
  const int64_t r0 = rows * blockIdx.x / gridDim.x, r1 = rows * (blockIdx.x + 1) / gridDim.x;
  const float* X2p = SAME ? X : X2;
  const int64_t ld2 = SAME ? ldx : ldx2;
  double* out = partial + (int64_t)blockIdx.x * 128 * 128;
  switch (threadIdx.x >> 6) {  // (uniform per wave)
    case 0: gram128_wave<SAME, 0>(X, ldx, X2p, ld2, r0, r1, out); break;
    case 1: gram128_wave<SAME, 1>(X, ldx, X2p, ld2, r0, r1, out); break;
    case 2: gram128_wave<SAME, 2>(X, ldx, X2p, ld2, r0, r1, out); break;
    default: gram128_wave<SAME, 3>(X, ldx, X2p, ld2, r0, r1, out); break;
  }
}

void launch_gram(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int lp,
                 const float* X2, int64_t ldx2, double* partial, double* G,
                 const int* skip_flag) {
  int nblk;
  if (lp == 32 || lp == 64) {
    // the matrix-core form: one workgroup per 256 rows, at most
    // kGramMaxBlocks workgroups
    const int64_t b = ceil_div(rows > 0 ? rows : 1, (int64_t)256);
    nblk = (int)(b < kGramMaxBlocks ? b : kGramMaxBlocks);
#define GRAM_MF(LP_, SAME_)                                                                     \
  hipLaunchKernelGGL((gram_mfma_kernel<LP_, SAME_>), dim3(nblk), dim3(64 * gram_waves<LP_>()), 0, st, X, \
                     ldx, X2, ldx2, rows, partial, skip_flag)
    if (lp == 32) {
      if (X2) GRAM_MF(32, false); else GRAM_MF(32, true);
    } else {
      if (X2) GRAM_MF(64, false); else GRAM_MF(64, true);
    }
#undef GRAM_MF
  } else {
    // lp = 128: the tiles dealt to the waves, one workgroup per 256 rows
    const int64_t b = ceil_div(rows > 0 ? rows : 1, (int64_t)256);
    nblk = (int)(b < kGramMaxBlocks ? b : kGramMaxBlocks);
    if (X2)
      hipLaunchKernelGGL(gram_mfma128_kernel<false>, dim3(nblk), dim3(256), 0, st, X, ldx, X2,
                         ldx2, rows, partial, skip_flag);
    else
      hipLaunchKernelGGL(gram_mfma128_kernel<true>, dim3(nblk), dim3(256), 0, st, X, ldx, X2,
                         ldx2, rows, partial, skip_flag);
  }
  const int lp2 = lp * lp;
  launch_reduce(st, partial, nblk, lp2, lp2, 1.0, G, nullptr, skip_flag);
}

// ------------------------------------------------------------------------
// In-place right triangular solve X <- (X + nu * addX) U^-1, U upper
// triangular float32 (lp x lp, row-major).  A zero diagonal U[j][j] marks a
// zero pivot of the LU renormalization: column j of the result is then the
// unit vector of the pivot row piv[j] (LAPACK getrf leaves L's column as
// e_j when the pivot is zero).  A nonzero *skip_flag == 0 skips the launch's
// work (conditional third Cholesky-QR pass).  One thread per row.
// ------------------------------------------------------------------------
template <int LP>
__global__ void __launch_bounds__(256) trsm_kernel(float* __restrict__ X, int64_t ldx, int64_t rows,
                                                   int l, const float* __restrict__ Ut,
                                                   const int* __restrict__ piv,
                                                   const int* __restrict__ skip_flag,
                                                   const float* __restrict__ nu,
                                                   const float* __restrict__ addX, int64_t ldadd) {
  if (skip_flag && *skip_flag == 0) return;
  // column j of U stored contiguously (sUt[j][i] = U[i][j]) so the solve reads
  // four entries per LDS access
  __shared__ __attribute__((aligned(16))) float sU[LP * LP];
  __shared__ float sd[LP];
  __shared__ int sp[LP];
  // consecutive threads fill consecutive LDS words (the transposed writes of
  // consecutive U entries would all hit one bank); U itself is small and read
  // from L2
  for (int e = threadIdx.x; e < LP * LP; e += 256) {
    const int j = e / LP, i = e % LP;
    sU[e] = Ut[i * LP + j];
  }
  if (threadIdx.x < LP) {
    const int j = threadIdx.x;
    const float d = (j < l) ? Ut[j * LP + j] : 0.f;
    sd[j] = (d != 0.f) ? 1.0f / d : 0.f;
    sp[j] = (piv && j < l) ? piv[j] : -1;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (row >= rows) return;
  float x[LP];
  const float* src = X + row * ldx;
#pragma unroll
  for (int c = 0; c < LP; c += 4) {
    const float4 v = *reinterpret_cast<const float4*>(src + c);
    x[c] = v.x; x[c + 1] = v.y; x[c + 2] = v.z; x[c + 3] = v.w;
  }
  if (addX) {
    const float s = *nu;
    const float* a = addX + row * ldadd;
#pragma unroll
    for (int c = 0; c < LP; c += 4) {
      const float4 v = *reinterpret_cast<const float4*>(a + c);
      x[c] += s * v.x; x[c + 1] += s * v.y; x[c + 2] += s * v.z; x[c + 3] += s * v.w;
    }
  }
#pragma unroll
  for (int j = 0; j < LP; ++j) {
    if (j < l) {
      float s = x[j];
      const float* col = sU + j * LP;
#pragma unroll
      for (int i = 0; i < j; ++i) s -= x[i] * col[i];
      const float d = sd[j];
      x[j] = (d != 0.f) ? s * d : ((row == sp[j]) ? 1.f : 0.f);
    } else {
      x[j] = 0.f;
    }
  }
  float* dst = X + row * ldx;
#pragma unroll
  for (int c = 0; c < LP; c += 4)
    *reinterpret_cast<float4*>(dst + c) = make_float4(x[c], x[c + 1], x[c + 2], x[c + 3]);
}

// The same solve, right-looking and blocked: once x_i is final, row i of U
// updates the entries to its right, so each x_j still accumulates
// x_i U[i][j] in increasing i and the results are bitwise those of
// trsm_kernel.  Two choices make it the faster form for many rows:
//  * independent updates: the products of a step go to different x_j, so
//    they issue back to back (the left-looking form chains each x_j's sum);
//  * U in LDS, read at one address by the whole wave (a broadcast: four
//    entries per read, no bank conflicts), where scalar loads of U (64 KB
//    at lp = 128, more than the scalar cache) wait on L2 for most rows.
// The columns go in blocks of 16: the diagonal block is solved, stored, and
// used to update the blocks to its right; then the register window shifts
// one block down, so the loop over blocks stays rolled (about 27 KB of code
// at lp = 128, against 94 KB fully unrolled).
// ------------------------------------------------------------------------
template <int LP, int NT>
__global__ void __launch_bounds__(NT) trsm_blocked_kernel(float* __restrict__ X, int64_t ldx,
                                                          int64_t rows, int l,
                                                          const float* __restrict__ Ut,
                                                          const int* __restrict__ piv,
                                                          const int* __restrict__ skip_flag,
                                                          const float* __restrict__ nu,
                                                          const float* __restrict__ addX,
                                                          int64_t ldadd) {
  if (skip_flag && *skip_flag == 0) return;
  constexpr int B = 16, NBK = LP / B;
  static_assert(LP % B == 0, "whole blocks");
  __shared__ __attribute__((aligned(16))) float sU[LP * LP];
  __shared__ float sd[LP];
  __shared__ int sp[LP];
  {
    // up to 16 loads in flight per thread before their stores (a plain
    // copy loop waits out the memory latency once per 16 bytes)
    constexpr int PER = LP * LP / (4 * NT), GR = PER < 16 ? PER : 16;
    static_assert(PER * 4 * NT == LP * LP && PER % GR == 0, "U fill shape");
    const float4* u4 = reinterpret_cast<const float4*>(Ut);
    float4* s4 = reinterpret_cast<float4*>(sU);
#pragma unroll
    for (int g0 = 0; g0 < PER; g0 += GR) {
      float4 t[GR];
#pragma unroll
      for (int u = 0; u < GR; ++u) t[u] = u4[(g0 + u) * NT + threadIdx.x];
#pragma unroll
      for (int u = 0; u < GR; ++u) s4[(g0 + u) * NT + threadIdx.x] = t[u];
    }
  }
  for (int j = threadIdx.x; j < LP; j += NT) {
    const float d = (j < l) ? Ut[j * LP + j] : 0.f;
    sd[j] = (d != 0.f) ? 1.0f / d : 0.f;
    sp[j] = (piv && j < l) ? piv[j] : -1;
  }
  __syncthreads();
  const int64_t row = (int64_t)blockIdx.x * NT + threadIdx.x;
  if (row >= rows) return;
  float x[LP];
  const float* src = X + row * ldx;
#pragma unroll
  for (int c = 0; c < LP; c += 4) {
    const float4 v = *reinterpret_cast<const float4*>(src + c);
    x[c] = v.x; x[c + 1] = v.y; x[c + 2] = v.z; x[c + 3] = v.w;
  }
  if (addX) {
    const float s = *nu;
    const float* a = addX + row * ldadd;
#pragma unroll
    for (int c = 0; c < LP; c += 4) {
      const float4 v = *reinterpret_cast<const float4*>(a + c);
      x[c] += s * v.x; x[c + 1] += s * v.y; x[c + 2] += s * v.z; x[c + 3] += s * v.w;
    }
  }
  float* dst = X + row * ldx;
  // x[0 .. LP - 16 b) holds columns 16 b .. LP - 1 at the start of block b
#pragma unroll 1
  for (int b = 0; b < NBK; ++b) {
    const int i0 = b * B;
#pragma unroll
    for (int i = 0; i < B; ++i) {
      const int gi = i0 + i;
      if (gi < l) {
        const float d = sd[gi];
        x[i] = (d != 0.f) ? x[i] * d : ((row == sp[gi]) ? 1.f : 0.f);
        const float* ui = sU + gi * LP + i0;
#pragma unroll
        for (int j = i + 1; j < B; ++j) x[j] -= x[i] * ui[j];
      } else {
        x[i] = 0.f;
      }
    }
#pragma unroll
    for (int c = 0; c < B; c += 4)
      *reinterpret_cast<float4*>(dst + i0 + c) = make_float4(x[c], x[c + 1], x[c + 2], x[c + 3]);
    // blocks to the right (columns at or beyond l are updated too, and
    // zeroed when reached; none is left once the block reaches l)
    if (i0 + B < l) {
#pragma unroll
      for (int c = 1; c < NBK; ++c) {
        if (c < NBK - b) {
#pragma unroll
          for (int i = 0; i < B; ++i) {
            const float* ui = sU + (i0 + i) * LP + i0 + c * B;
#pragma unroll
            for (int j = 0; j < B; ++j) x[c * B + j] -= x[i] * ui[j];
          }
        }
      }
    }
#pragma unroll
    for (int t = 0; t < LP - B; ++t) x[t] = x[t + B];
  }
}

void launch_trsm(hipStream_t st, float* X, int64_t ldx, int64_t rows, int l, int lp,
                 const float* Ut, const int* piv, const int* skip_flag, const float* nu,
                 const float* addX, int64_t ldadd, int num_cus) {
  if (rows == 0) return;
  const dim3 grid((unsigned)ceil_div(rows, 256));
  // lp = 64 with a workgroup of rows per CU or more, and lp = 128: the
  // blocked form (lp = 128 on fewer rows in workgroups of 64 threads, which
  // spreads them over more CUs)
  const bool blocked = lp >= 64 && rows >= (int64_t)num_cus * 256;
#define TRSM_GO(K_) hipLaunchKernelGGL(K_, grid, dim3(256), 0, st, X, ldx, rows, l, Ut, piv, skip_flag, nu, addX, ldadd)
  switch (lp) {
    case 32: TRSM_GO(trsm_kernel<32>); break;
    case 64:
      if (blocked) TRSM_GO((trsm_blocked_kernel<64, 256>));
      else TRSM_GO(trsm_kernel<64>);
      break;
    case 128:
      if (blocked)
        TRSM_GO((trsm_blocked_kernel<128, 256>));
      else
        hipLaunchKernelGGL((trsm_blocked_kernel<128, 64>), dim3((unsigned)ceil_div(rows, 64)),
                           dim3(64), 0, st, X, ldx, rows, l, Ut, piv, skip_flag, nu, addX, ldadd);
      break;
    default: break;
  }
#undef TRSM_GO
}

// ------------------------------------------------------------------------
// Y (rows x k) = X (rows x lp) W (lp x k), W float64 rounded to float32 in
// LDS.  A workgroup walks tiles of 32 rows (grid-stride, about two
// workgroups per CU, so W is converted once per workgroup): the tile of X
// is loaded with coalesced 16-byte reads and kept transposed in LDS; thread
// (row group, column group) accumulates a (32 / RG) x 4 block of Y over
// i < l in order, and writes it back with 16-byte stores when the layout
// allows.
// ------------------------------------------------------------------------
static constexpr int kGemmRows = 32;

template <int LP>
__global__ void __launch_bounds__(256) small_gemm_kernel(const float* __restrict__ X, int64_t ldx,
                                                         int64_t rows, int l,
                                                         const double* __restrict__ W, int ldw,
                                                         int k, float* __restrict__ Y,
                                                         int64_t ldy, int vec) {
  constexpr int TR = kGemmRows;
  constexpr int CG = LP / 4;        // column groups of 4
  constexpr int RG = 256 / CG;      // row groups
  constexpr int RPG = TR / RG;      // rows per thread
  constexpr int WS = LP + 4;        // LDS row stride of W
  constexpr int XS = TR + 4;        // LDS row stride of the transposed tile
  constexpr int F4 = TR * LP / 4 / 256;  // float4 loads per thread per tile
  __shared__ __attribute__((aligned(16))) float sW[LP * WS];
  __shared__ __attribute__((aligned(16))) float sX[LP * XS];
  for (int e = threadIdx.x; e < LP * LP; e += 256) {
    const int i = e / LP, c = e % LP;
    sW[i * WS + c] = (i < l && c < k) ? (float)W[i * ldw + c] : 0.f;
  }
  const int tc = threadIdx.x % CG, tr = threadIdx.x / CG;
  const int64_t ntiles = ceil_div(rows, (int64_t)TR);
  // the next tile's X is loaded into registers while the current one is used
  float4 pre[F4];
  auto load = [&](int64_t t) {
#pragma unroll
    for (int q = 0; q < F4; ++q) {
      const int e = threadIdx.x + 256 * q, rr = e / (LP / 4), c4 = 4 * (e % (LP / 4));
      const int64_t r = t * TR + rr;
      pre[q] = (r < rows) ? *reinterpret_cast<const float4*>(X + r * ldx + c4)
                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  if ((int64_t)blockIdx.x < ntiles) load(blockIdx.x);
  for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const int64_t r0 = t * TR;
    __syncthreads();  // the previous tile's reads are done (and W is in place)
#pragma unroll
    for (int q = 0; q < F4; ++q) {
      const int e = threadIdx.x + 256 * q, rr = e / (LP / 4), c4 = 4 * (e % (LP / 4));
      sX[(c4 + 0) * XS + rr] = pre[q].x;
      sX[(c4 + 1) * XS + rr] = pre[q].y;
      sX[(c4 + 2) * XS + rr] = pre[q].z;
      sX[(c4 + 3) * XS + rr] = pre[q].w;
    }
    __syncthreads();
    if (t + gridDim.x < ntiles) load(t + gridDim.x);
    float acc[RPG][4];
#pragma unroll
    for (int a = 0; a < RPG; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0.f;
    for (int i = 0; i < l; ++i) {
      const float4 w4 = *reinterpret_cast<const float4*>(sW + i * WS + 4 * tc);
      float xa[RPG];
#pragma unroll
      for (int a = 0; a < RPG; ++a) xa[a] = sX[i * XS + tr * RPG + a];
#pragma unroll
      for (int a = 0; a < RPG; ++a) {
        acc[a][0] = fmaf(xa[a], w4.x, acc[a][0]);
        acc[a][1] = fmaf(xa[a], w4.y, acc[a][1]);
        acc[a][2] = fmaf(xa[a], w4.z, acc[a][2]);
        acc[a][3] = fmaf(xa[a], w4.w, acc[a][3]);
      }
    }
    const int c0 = 4 * tc;
    if (c0 < k) {
#pragma unroll
      for (int a = 0; a < RPG; ++a) {
        const int64_t r = r0 + tr * RPG + a;
        if (r >= rows) break;
        float* dst = Y + r * ldy + c0;
        if (vec && c0 + 4 <= k) {
          *reinterpret_cast<float4*>(dst) = make_float4(acc[a][0], acc[a][1], acc[a][2], acc[a][3]);
        } else {
#pragma unroll
          for (int b = 0; b < 4; ++b)
            if (c0 + b < k) dst[b] = acc[a][b];
        }
      }
    }
  }
}

void launch_small_gemm(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int l,
                       const double* W, int ldw, int k, float* Y, int64_t ldy, int num_cus) {
  if (rows == 0) return;
  const int64_t tiles = ceil_div(rows, (int64_t)kGemmRows);
  const int64_t cap = 2 * (int64_t)(num_cus > 0 ? num_cus : 256);
  const dim3 grid((unsigned)(tiles < cap ? tiles : cap));
  const int vec = (ldy % 4 == 0 && (reinterpret_cast<uintptr_t>(Y) & 15) == 0) ? 1 : 0;
  const int lp = (int)ldx;  // X is stored with ld = lp
  switch (lp) {
    case 32: hipLaunchKernelGGL(small_gemm_kernel<32>, grid, dim3(256), 0, st, X, ldx, rows, l, W, ldw, k, Y, ldy, vec); break;
    case 64: hipLaunchKernelGGL(small_gemm_kernel<64>, grid, dim3(256), 0, st, X, ldx, rows, l, W, ldw, k, Y, ldy, vec); break;
    case 128: hipLaunchKernelGGL(small_gemm_kernel<128>, grid, dim3(256), 0, st, X, ldx, rows, l, W, ldw, k, Y, ldy, vec); break;
    default: break;
  }
}

// ------------------------------------------------------------------------
// Sign convention for the output: the largest-|.| entry of each column of U
// is made positive (ties go to the smallest row index); V's column follows.
// ------------------------------------------------------------------------
static constexpr int kSignChunk = 64;

__global__ void __launch_bounds__(128) colabsmax_kernel(const float* __restrict__ U, int64_t ldu,
                                                        int64_t m, int k, float* __restrict__ pval,
                                                        int64_t* __restrict__ pidx) {
  const int c = threadIdx.x;
  if (c >= k) return;
  const int64_t r0 = (int64_t)blockIdx.x * kSignChunk;
  float best = -1.f, bval = 0.f;
  int64_t bidx = -1;
  for (int64_t r = r0; r < r0 + kSignChunk && r < m; ++r) {
    const float v = U[r * ldu + c];
    if (fabsf(v) > best) {
      best = fabsf(v);
      bval = v;
      bidx = r;
    }
  }
  pval[(int64_t)blockIdx.x * 128 + c] = (bidx >= 0) ? bval : 0.f;
  pidx[(int64_t)blockIdx.x * 128 + c] = bidx;
}

// One workgroup per column: first maximum of |U[:, c]| over the block partials.
__global__ void __launch_bounds__(256) sign_final_kernel(const float* __restrict__ pval,
                                                         const int64_t* __restrict__ pidx,
                                                         int nblk, int k, float* __restrict__ sgn) {
  const int c = blockIdx.x;
  float best = -1.f, bval = 0.f;
  int64_t bidx = 0x7fffffffffffffffLL;
  for (int b = threadIdx.x; b < nblk; b += 256) {
    const int64_t i = pidx[(int64_t)b * 128 + c];
    const float v = pval[(int64_t)b * 128 + c];
    if (i >= 0 && (fabsf(v) > best || (fabsf(v) == best && i < bidx))) {
      best = fabsf(v);
      bval = v;
      bidx = i;
    }
  }
  __shared__ float sb[256], sv[256];
  __shared__ int64_t si[256];
  sb[threadIdx.x] = best;
  sv[threadIdx.x] = bval;
  si[threadIdx.x] = bidx;
  __syncthreads();
  for (int o = 128; o > 0; o >>= 1) {
    if (threadIdx.x < o) {
      const int u = threadIdx.x + o;
      if (sb[u] > sb[threadIdx.x] || (sb[u] == sb[threadIdx.x] && si[u] < si[threadIdx.x])) {
        sb[threadIdx.x] = sb[u];
        sv[threadIdx.x] = sv[u];
        si[threadIdx.x] = si[u];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0 && c < k) sgn[c] = (sv[0] < 0.f) ? -1.f : 1.f;
}

__global__ void __launch_bounds__(256) flip_kernel(float* __restrict__ X, int64_t ldx, int64_t rows,
                                                   int k, const float* __restrict__ sgn) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = e / k;
  const int c = (int)(e % k);
  if (r < rows && sgn[c] < 0.f) X[r * ldx + c] = -X[r * ldx + c];
}

size_t sign_work_bytes(int64_t m) {
  const int nblk = (int)ceil_div(m > 0 ? m : 1, kSignChunk);
  return (size_t)nblk * 128 * (sizeof(float) + sizeof(int64_t)) + 128 * sizeof(float);
}

void launch_sign_fix(hipStream_t st, float* U, int64_t ldu, int64_t m, int k, float* V,
                     int64_t ldv, int64_t n, int* work) {
  const int nblk = (int)ceil_div(m > 0 ? m : 1, kSignChunk);
  float* pval = reinterpret_cast<float*>(work);
  int64_t* pidx = reinterpret_cast<int64_t*>(pval + (size_t)nblk * 128 + ((nblk * 128) & 1));
  float* sgn = reinterpret_cast<float*>(pidx + (size_t)nblk * 128);
  hipLaunchKernelGGL(colabsmax_kernel, dim3(nblk), dim3(128), 0, st, U, ldu, m, k, pval, pidx);
  hipLaunchKernelGGL(sign_final_kernel, dim3(k), dim3(256), 0, st, pval, pidx, nblk, k, sgn);
  hipLaunchKernelGGL(flip_kernel, dim3((unsigned)ceil_div(m * k, 256)), dim3(256), 0, st, U, ldu,
                     m, k, sgn);
  if (V)
    hipLaunchKernelGGL(flip_kernel, dim3((unsigned)ceil_div(n * k, 256)), dim3(256), 0, st, V, ldv,
                       n, k, sgn);
}

}  // namespace rpca

namespace rpca {

// Plain fills and copies as kernels (not hipMemsetAsync / hipMemcpyAsync), so
// that a captured graph of a solve holds kernel nodes only.
__global__ void __launch_bounds__(256) fill_zero_kernel(float4* __restrict__ p, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
}

__global__ void __launch_bounds__(256) copy_kernel(float4* __restrict__ d,
                                                   const float4* __restrict__ s, int64_t n4) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n4) d[i] = s[i];
}

void launch_fill_zero(hipStream_t st, float* p, int64_t count) {
  const int64_t n4 = count / 4;  // callers pass multiples of 4 floats (16-byte aligned)
  if (n4 <= 0) return;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)ceil_div(n4, 256)), dim3(256), 0, st,
                     reinterpret_cast<float4*>(p), n4);
}

void launch_copy(hipStream_t st, float* dst, const float* src, int64_t count) {
  const int64_t n4 = count / 4;
  if (n4 <= 0) return;
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)ceil_div(n4, 256)), dim3(256), 0, st,
                     reinterpret_cast<float4*>(dst), reinterpret_cast<const float4*>(src), n4);
}

}  // namespace rpca
