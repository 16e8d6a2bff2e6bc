// Spectral-norm error estimate of a low-rank approximation (Section 4): the
// paper measures accuracy by ||A - U Sigma V*|| and estimates it with the
// power method from a random start (Kuczynski and Wozniakowski: within a
// factor of two with overwhelming probability).
//
// Here the residual E = A_c - U diag(S) V^T (A_c = A, or A minus its column
// means; V = U for the symmetric residual) is never formed.  A block of SB = 4
// start vectors (Philox stream 1, the Gaussian map of the test matrix) is
// iterated as X <- orth(E^T E X) in float64, and the estimate is the largest
// singular value of E X, which never exceeds ||E||.
//
//   E X   = A X - 1 mean(A X) - U (S o V^T X)         (mean only with centering)
//   E^T Y = A^T (Y - 1 mean(Y)) - V (S o U^T Y)
//
// since A_c = (I - 1 1^T / m) A.  A is read in float32 and every product is
// accumulated in float64.  orth is Cholesky QR three times over (the first
// with a small diagonal shift), which returns the Q factor with a positive
// diagonal R, as Householder QR with the sign fixed would.
#include <cmath>

#include "common.h"
#include "kernels.h"
#include "philox.h"

namespace rpca {

static constexpr int SB = 4;           // power-method block size
static constexpr int kTnChunk = 512;   // rows per partial of the tall reductions
static constexpr int kAxRowsW = 8;     // rows per wave in E X
static constexpr int kAtxTile = 1024;  // columns per workgroup in E^T Y

// ---------------------------------------------------------------------------
// X0[i][j] = z[j n + i] of stream 1 (float32 normal, widened)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) spec_start_kernel(uint64_t seed, int64_t n,
                                                         double* __restrict__ X) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * SB) return;
  const int64_t i = e / SB;
  const int j = (int)(e - i * SB);
  X[e] = (double)philox_normal(seed, 1u, (uint64_t)j * (uint64_t)n + (uint64_t)i);
}

// ---------------------------------------------------------------------------
// Tall reductions: out[j][q] = sum_i U[i][j] T[i][q] (j < k) and
// out[k][q] = sum_i T[i][q]; T is rows x SB float64.  Partials per chunk of
// kTnChunk rows, then a fixed-order sum.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) spec_tn_partial_kernel(const float* __restrict__ U,
                                                              int64_t ldu, int k,
                                                              const double* __restrict__ T,
                                                              int64_t rows,
                                                              double* __restrict__ part) {
  const int nout = (k + 1) * SB;
  const int64_t r0 = (int64_t)blockIdx.x * kTnChunk;
  const int64_t r1 = min(rows, r0 + kTnChunk);
  for (int o = threadIdx.x; o < nout; o += blockDim.x) {
    const int j = o / SB, q = o - j * SB;
    // four independent partial sums keep several loads in flight
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t i = r0;
    if (j < k) {
      for (; i + 4 <= r1; i += 4) {
        s0 += (double)U[i * ldu + j] * T[i * SB + q];
        s1 += (double)U[(i + 1) * ldu + j] * T[(i + 1) * SB + q];
        s2 += (double)U[(i + 2) * ldu + j] * T[(i + 2) * SB + q];
        s3 += (double)U[(i + 3) * ldu + j] * T[(i + 3) * SB + q];
      }
      for (; i < r1; ++i) s0 += (double)U[i * ldu + j] * T[i * SB + q];
    } else {
      for (; i + 4 <= r1; i += 4) {
        s0 += T[i * SB + q];
        s1 += T[(i + 1) * SB + q];
        s2 += T[(i + 2) * SB + q];
        s3 += T[(i + 3) * SB + q];
      }
      for (; i < r1; ++i) s0 += T[i * SB + q];
    }
    part[(int64_t)blockIdx.x * nout + o] = (s0 + s1) + (s2 + s3);
  }
}

__global__ void __launch_bounds__(256) spec_sum_parts_kernel(const double* __restrict__ part,
                                                             int nparts, int nout,
                                                             double* __restrict__ out) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nout) return;
  double s = 0.0;
  for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * nout + o];
  out[o] = s;
}

static int tn_parts(int64_t rows) { return (int)ceil_div(rows, kTnChunk); }

static void tn_reduce(hipStream_t st, const float* U, int64_t ldu, int k, const double* T,
                      int64_t rows, double* part, double* out) {
  const int parts = tn_parts(rows);
  const int nout = (k + 1) * SB;
  hipLaunchKernelGGL(spec_tn_partial_kernel, dim3(parts), dim3(256), 0, st, U, ldu, k, T, rows,
                     part);
  hipLaunchKernelGGL(spec_sum_parts_kernel, dim3((unsigned)ceil_div(nout, 256)), dim3(256), 0, st,
                     part, parts, nout, out);
}

// ---------------------------------------------------------------------------
// P = A X  (m x SB, float64).  A wave takes kAxRowsW rows; VEC: lane reads
// float4 of each row at columns 4 lane + 256 s (needs n % 4 == 0, lda % 4 == 0
// and 16-byte alignment), else one float at column lane + 64 s.
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ void __launch_bounds__(256) spec_ax_kernel(const float* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      const double* __restrict__ X,
                                                      double* __restrict__ P) {
  constexpr int R = kAxRowsW;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * R;
  if (r0 >= m) return;
  const float* rowp[R];
#pragma unroll
  for (int r = 0; r < R; ++r) rowp[r] = A + min(r0 + r, m - 1) * lda;
  double acc[R][SB];
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < SB; ++q) acc[r][q] = 0.0;
  if (VEC) {
    for (int64_t c = 4 * lane; c < n; c += 256) {
      float4 a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = *reinterpret_cast<const float4*>(rowp[r] + c);
      const double2* xp = reinterpret_cast<const double2*>(X + c * SB);
      double x[4][SB];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const double2 u = xp[2 * t], v = xp[2 * t + 1];
        x[t][0] = u.x; x[t][1] = u.y; x[t][2] = v.x; x[t][3] = v.y;
      }
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < SB; ++q) {
          acc[r][q] += (double)a[r].x * x[0][q];
          acc[r][q] += (double)a[r].y * x[1][q];
          acc[r][q] += (double)a[r].z * x[2][q];
          acc[r][q] += (double)a[r].w * x[3][q];
        }
    }
  } else {
    for (int64_t c = lane; c < n; c += 64) {
      float a[R];
#pragma unroll
      for (int r = 0; r < R; ++r) a[r] = rowp[r][c];
      const double2* xp = reinterpret_cast<const double2*>(X + c * SB);
      const double2 u = xp[0], v = xp[1];
      const double x[SB] = {u.x, u.y, v.x, v.y};
#pragma unroll
      for (int r = 0; r < R; ++r)
#pragma unroll
        for (int q = 0; q < SB; ++q) acc[r][q] += (double)a[r] * x[q];
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < SB; ++q) acc[r][q] = wave_sum(acc[r][q]);
  // lane r * SB + q writes P[r0 + r][q]
  if (lane < R * SB) {
    double v = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r)
#pragma unroll
      for (int q = 0; q < SB; ++q)
        if (lane == r * SB + q) v = acc[r][q];
    const int r = lane / SB;
    if (r0 + r < m) P[(r0 + r) * SB + (lane % SB)] = v;
  }
}

// Y[i] = P[i] - mean(P) (centering) - U[i] W,  W = S o (V^T X) (k x SB),
// in place on P.  sums[k][q] holds the column sums of P when centering.
__global__ void __launch_bounds__(256) spec_fix_y_kernel(double* __restrict__ P, int64_t m,
                                                         const double* __restrict__ sums,
                                                         bool center,
                                                         const float* __restrict__ U,
                                                         int64_t ldu, int k,
                                                         const double* __restrict__ S,
                                                         const double* __restrict__ VtX) {
  __shared__ double W[129 * SB];
  for (int e = threadIdx.x; e < k * SB; e += blockDim.x) W[e] = S[e / SB] * VtX[e];
  __syncthreads();
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  double y[SB];
#pragma unroll
  for (int q = 0; q < SB; ++q) y[q] = P[i * SB + q] - (center ? sums[q] / (double)m : 0.0);
  for (int j = 0; j < k; ++j) {
    const double u = (double)U[i * ldu + j];
#pragma unroll
    for (int q = 0; q < SB; ++q) y[q] -= u * W[j * SB + q];
  }
#pragma unroll
  for (int q = 0; q < SB; ++q) P[i * SB + q] = y[q];
}

// ---------------------------------------------------------------------------
// Zpart[band][c][q] = sum over the band's rows i of A[i][c] (Y[i][q] - mean_q).
// Grid (column tiles of kAtxTile, row bands).  VEC: thread t owns columns
// tile + 4t .. +3 (float4); else columns tile + t + 256 u, u < 4.
// ---------------------------------------------------------------------------
template <bool VEC>
__global__ void __launch_bounds__(256) spec_atx_kernel(const float* __restrict__ A, int64_t lda,
                                                       int64_t m, int64_t n,
                                                       const double* __restrict__ Y,
                                                       const double* __restrict__ ysum,
                                                       bool center, int64_t band_rows,
                                                       double* __restrict__ Zpart) {
  const int t = threadIdx.x;
  const int64_t tile = (int64_t)blockIdx.x * kAtxTile;
  const int64_t i0 = (int64_t)blockIdx.y * band_rows;
  const int64_t i1 = min(m, i0 + band_rows);
  double mean[SB];
#pragma unroll
  for (int q = 0; q < SB; ++q) mean[q] = center ? ysum[q] / (double)m : 0.0;
  int64_t col[4];
  bool ok[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    col[u] = VEC ? tile + 4 * t + u : tile + t + 256 * u;
    ok[u] = col[u] < n;
  }
  double acc[4][SB];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int q = 0; q < SB; ++q) acc[u][q] = 0.0;
  for (int64_t i = i0; i < i1; ++i) {
    float a[4];
    const float* row = A + i * lda;
    if (VEC) {
      if (ok[0]) {
        const float4 v = *reinterpret_cast<const float4*>(row + col[0]);
        a[0] = v.x; a[1] = v.y; a[2] = v.z; a[3] = v.w;
      } else {
        a[0] = a[1] = a[2] = a[3] = 0.f;
      }
    } else {
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = ok[u] ? row[col[u]] : 0.f;
    }
    double y[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) y[q] = Y[i * SB + q] - mean[q];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < SB; ++q) acc[u][q] += (double)a[u] * y[q];
  }
  double* out = Zpart + (int64_t)blockIdx.y * n * SB;
#pragma unroll
  for (int u = 0; u < 4; ++u)
    if (ok[u])
#pragma unroll
      for (int q = 0; q < SB; ++q) out[col[u] * SB + q] = acc[u][q];
}

// Z[c][q] = sum_band Zpart[band][c][q] - V[c] (S o U^T Y)
__global__ void __launch_bounds__(256) spec_atx_reduce_kernel(const double* __restrict__ Zpart,
                                                              int bands, int64_t n,
                                                              const float* __restrict__ V,
                                                              int64_t ldv, int k,
                                                              const double* __restrict__ S,
                                                              const double* __restrict__ UtY,
                                                              double* __restrict__ Z) {
  __shared__ double W[129 * SB];
  for (int e = threadIdx.x; e < k * SB; e += blockDim.x) W[e] = S[e / SB] * UtY[e];
  __syncthreads();
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * SB) return;
  const int64_t c = e / SB;
  const int q = (int)(e - c * SB);
  double s = 0.0;
  for (int b = 0; b < bands; ++b) s += Zpart[(int64_t)b * n * SB + e];
  for (int j = 0; j < k; ++j) s -= (double)V[c * ldv + j] * W[j * SB + q];
  Z[e] = s;
}

// ---------------------------------------------------------------------------
// Yc = Y - 1 mean(Y) (sparse A^T Y with centering); sums[q] = column sums
__global__ void __launch_bounds__(256) spec_center_kernel(const double* __restrict__ Y, int64_t m,
                                                          const double* __restrict__ sums,
                                                          double* __restrict__ Yc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= m * SB) return;
  Yc[e] = Y[e] - sums[e % SB] / (double)m;
}

// Cholesky QR of X (rows x SB, float64)
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) spec_gram_partial_kernel(const double* __restrict__ X,
                                                                int64_t rows,
                                                                double* __restrict__ part) {
  constexpr int NO = SB * (SB + 1) / 2;
  __shared__ double red[4][NO];
  const int64_t r0 = (int64_t)blockIdx.x * kTnChunk;
  const int64_t r1 = min(rows, r0 + kTnChunk);
  double g[NO];
#pragma unroll
  for (int o = 0; o < NO; ++o) g[o] = 0.0;
  for (int64_t i = r0 + threadIdx.x; i < r1; i += blockDim.x) {
    double x[SB];
#pragma unroll
    for (int q = 0; q < SB; ++q) x[q] = X[i * SB + q];
    int o = 0;
#pragma unroll
    for (int a = 0; a < SB; ++a)
#pragma unroll
      for (int b = a; b < SB; ++b) g[o++] += x[a] * x[b];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 0; o < NO; ++o) {
    const double v = wave_sum(g[o]);
    if (lane == 0) red[wave][o] = v;
  }
  __syncthreads();
  if (threadIdx.x < NO) {
    const int o = threadIdx.x;
    part[(int64_t)blockIdx.x * NO + o] = red[0][o] + red[1][o] + red[2][o] + red[3][o];
  }
}

// Sum the Gram partials, factor G + s I = R^T R (s > 0 on the first pass, or
// when a pivot is not positive), write R^-1 (upper, row-major SB x SB).  An
// all-zero block gives R^-1 = I.
__global__ void __launch_bounds__(64) spec_chol_kernel(const double* __restrict__ part, int nparts,
                                                       int64_t rows, int shifted,
                                                       double* __restrict__ Rinv) {
  constexpr int NO = SB * (SB + 1) / 2;
  __shared__ double gs[NO];
  if (threadIdx.x < NO) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * NO + threadIdx.x];
    gs[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double G[SB][SB];
  {
    int o = 0;
    for (int a = 0; a < SB; ++a)
      for (int b = a; b < SB; ++b) {
        G[a][b] = gs[o];
        G[b][a] = gs[o];
        ++o;
      }
  }
  double tr = 0.0;
  for (int a = 0; a < SB; ++a) tr += G[a][a];
  double R[SB][SB];
  for (int a = 0; a < SB; ++a)
    for (int b = 0; b < SB; ++b) R[a][b] = (a == b) ? 1.0 : 0.0;
  if (tr > 0.0 && tr < 1e300) {
    const double u = 1.1102230246251565e-16;  // 2^-53
    double s = shifted ? 11.0 * ((double)rows * SB + SB * (SB + 1)) * u * tr : 0.0;
    for (int attempt = 0; attempt < 8; ++attempt) {
      bool ok = true;
      for (int a = 0; a < SB; ++a)
        for (int b = 0; b < SB; ++b) R[a][b] = 0.0;
      for (int j = 0; j < SB && ok; ++j) {
        double d = G[j][j] + s;
        for (int p = 0; p < j; ++p) d -= R[p][j] * R[p][j];
        if (!(d > 0.0)) {
          ok = false;
          break;
        }
        const double r = sqrt(d);
        R[j][j] = r;
        for (int c = j + 1; c < SB; ++c) {
          double v = G[j][c];
          for (int p = 0; p < j; ++p) v -= R[p][j] * R[p][c];
          R[j][c] = v / r;
        }
      }
      if (ok) break;
      s = (s > 0.0) ? 100.0 * s : 1e-15 * tr;
    }
  }
  // R^-1 by back substitution, column by column
  double Ri[SB][SB];
  for (int a = 0; a < SB; ++a)
    for (int b = 0; b < SB; ++b) Ri[a][b] = 0.0;
  for (int c = 0; c < SB; ++c) {
    for (int a = c; a >= 0; --a) {
      double v = (a == c) ? 1.0 : 0.0;
      for (int p = a + 1; p <= c; ++p) v -= R[a][p] * Ri[p][c];
      Ri[a][c] = v / R[a][a];
    }
  }
  for (int a = 0; a < SB; ++a)
    for (int b = 0; b < SB; ++b) Rinv[a * SB + b] = Ri[a][b];
}

__global__ void __launch_bounds__(256) spec_apply_kernel(double* __restrict__ X, int64_t rows,
                                                         const double* __restrict__ Rinv) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double x[SB], y[SB];
#pragma unroll
  for (int q = 0; q < SB; ++q) x[q] = X[i * SB + q];
#pragma unroll
  for (int c = 0; c < SB; ++c) {
    double v = 0.0;
#pragma unroll
    for (int a = 0; a <= c; ++a) v += x[a] * Rinv[a * SB + c];
    y[c] = v;
  }
#pragma unroll
  for (int q = 0; q < SB; ++q) X[i * SB + q] = y[q];
}

// Largest eigenvalue of the SB x SB Gram of Y (cyclic Jacobi), sqrt -> result.
__global__ void __launch_bounds__(64) spec_final_kernel(const double* __restrict__ part, int nparts,
                                                        double* __restrict__ result) {
  constexpr int NO = SB * (SB + 1) / 2;
  __shared__ double gs[NO];
  if (threadIdx.x < NO) {
    double s = 0.0;
    for (int p = 0; p < nparts; ++p) s += part[(int64_t)p * NO + threadIdx.x];
    gs[threadIdx.x] = s;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double G[SB][SB];
  int o = 0;
  for (int a = 0; a < SB; ++a)
    for (int b = a; b < SB; ++b) {
      G[a][b] = gs[o];
      G[b][a] = gs[o];
      ++o;
    }
  for (int sweep = 0; sweep < 30; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int a = 0; a < SB; ++a) {
      diag += G[a][a] * G[a][a];
      for (int b = a + 1; b < SB; ++b) off += G[a][b] * G[a][b];
    }
    if (!(off > 1e-32 * diag)) break;
    for (int p = 0; p < SB; ++p)
      for (int q = p + 1; q < SB; ++q) {
        if (G[p][q] == 0.0) continue;
        const double theta = (G[q][q] - G[p][p]) / (2.0 * G[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < SB; ++r) {  // columns p, q
          const double gp = G[r][p], gq = G[r][q];
          G[r][p] = c * gp - s * gq;
          G[r][q] = s * gp + c * gq;
        }
        for (int r = 0; r < SB; ++r) {  // rows p, q
          const double gp = G[p][r], gq = G[q][r];
          G[p][r] = c * gp - s * gq;
          G[q][r] = s * gp + c * gq;
        }
      }
  }
  double lmax = 0.0;
  for (int a = 0; a < SB; ++a) lmax = fmax(lmax, G[a][a]);
  result[0] = sqrt(lmax);
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
namespace {

struct SpecLayout {
  int64_t off_X, off_Y, off_Yc, off_Zp, off_part, off_vtx, off_uty, off_sum, off_rinv, total;
  int tiles, bands, parts;
  int64_t band_rows;
};

SpecLayout spec_layout(int64_t m, int64_t n, int k) {
  SpecLayout L{};
  L.tiles = (int)ceil_div(n, kAtxTile);
  int bands = (int)std::max<int64_t>(1, 1024 / L.tiles);
  bands = (int)std::min<int64_t>(bands, ceil_div(m, 64));
  L.band_rows = ceil_div(m, bands);
  L.bands = (int)ceil_div(m, L.band_rows);
  L.parts = tn_parts(std::max(m, n));
  int64_t off = 0;
  auto take = [&](int64_t doubles) {
    const int64_t o = off;
    off = round_up(off + doubles, 32);
    return o;
  };
  L.off_X = take(n * SB);
  L.off_Y = take(m * SB);
  L.off_Yc = take(m * SB);
  L.off_Zp = take((int64_t)L.bands * n * SB);
  L.off_part = take((int64_t)L.parts * (k + 1) * SB);
  L.off_vtx = take((int64_t)(k + 1) * SB);
  L.off_uty = take((int64_t)(k + 1) * SB);
  L.off_sum = take((int64_t)(k + 1) * SB);
  L.off_rinv = take(SB * SB);
  L.total = off;
  return L;
}

void orth(hipStream_t st, double* X, int64_t rows, double* part, double* Rinv) {
  const int parts = tn_parts(rows);
  const unsigned g = (unsigned)ceil_div(rows, 256);
  for (int pass = 0; pass < 3; ++pass) {
    hipLaunchKernelGGL(spec_gram_partial_kernel, dim3(parts), dim3(256), 0, st, X, rows, part);
    hipLaunchKernelGGL(spec_chol_kernel, dim3(1), dim3(64), 0, st, part, parts, rows,
                       pass == 0 ? 1 : 0, Rinv);
    hipLaunchKernelGGL(spec_apply_kernel, dim3(g), dim3(256), 0, st, X, rows, Rinv);
  }
}

}  // namespace

size_t spectral_work_bytes(int64_t m, int64_t n, int k) {
  return (size_t)spec_layout(m, n, k).total * sizeof(double) + 256;
}

void launch_spectral(hipStream_t st, const float* A, int64_t lda, int64_t m, int64_t n, bool center,
                     const float* U, int64_t ldu, const double* S, const float* V, int64_t ldv,
                     int k, int iters, uint64_t seed, void* work, double* result,
                     const SpecSparse* sp) {
  const SpecLayout L = spec_layout(m, n, k);
  double* base = static_cast<double*>(work);
  double* X = base + L.off_X;
  double* Y = base + L.off_Y;
  double* Yc = base + L.off_Yc;
  double* Zp = base + L.off_Zp;
  double* part = base + L.off_part;
  double* vtx = base + L.off_vtx;
  double* uty = base + L.off_uty;
  double* sums = base + L.off_sum;
  double* Rinv = base + L.off_rinv;
  const float* Vs = V ? V : U;
  const int64_t ldvs = V ? ldv : ldu;
  const bool vec = (n % 4 == 0) && (lda % 4 == 0) && ((reinterpret_cast<uintptr_t>(A) & 15) == 0);
  const unsigned ax_grid = (unsigned)ceil_div(m, 4 * kAxRowsW);

  hipLaunchKernelGGL(spec_start_kernel, dim3((unsigned)ceil_div(n * SB, 256)), dim3(256), 0, st,
                     seed, n, X);
  orth(st, X, n, part, Rinv);

  // Y = E X
  auto apply_e = [&]() {
    tn_reduce(st, Vs, ldvs, k, X, n, part, vtx);
    if (sp)
      launch_spmm4_f64(st, sp->ptr, sp->idx, sp->val, sp->dtype, m, sp->nnz, (int)n, X, Y);
    else if (vec)
      hipLaunchKernelGGL(spec_ax_kernel<true>, dim3(ax_grid), dim3(256), 0, st, A, lda, m, n, X, Y);
    else
      hipLaunchKernelGGL(spec_ax_kernel<false>, dim3(ax_grid), dim3(256), 0, st, A, lda, m, n, X,
                         Y);
    if (center) tn_reduce(st, nullptr, 0, 0, Y, m, part, sums);
    hipLaunchKernelGGL(spec_fix_y_kernel, dim3((unsigned)ceil_div(m, 256)), dim3(256), 0, st, Y, m,
                       sums, center, U, ldu, k, S, vtx);
  };
  for (int it = 0; it < iters; ++it) {
    apply_e();
    // X = E^T Y, then orthonormalized
    tn_reduce(st, U, ldu, k, Y, m, part, uty);
    if (sp) {
      // A^T (Y - 1 mean(Y)) by the CSC gather, then the low-rank correction
      const double* src = Y;
      if (center) {
        hipLaunchKernelGGL(spec_center_kernel, dim3((unsigned)ceil_div(m * SB, 256)), dim3(256), 0,
                           st, Y, m, uty + k * SB, Yc);
        src = Yc;
      }
      launch_spmm4_f64(st, sp->ptr_t, sp->idx_t, sp->val_t, sp->dtype, n, sp->nnz, (int)m, src, Zp);
      hipLaunchKernelGGL(spec_atx_reduce_kernel, dim3((unsigned)ceil_div(n * SB, 256)), dim3(256),
                         0, st, Zp, 1, n, Vs, ldvs, k, S, uty, X);
      orth(st, X, n, part, Rinv);
      continue;
    }
    const dim3 grid((unsigned)L.tiles, (unsigned)L.bands);
    if (vec)
      hipLaunchKernelGGL(spec_atx_kernel<true>, grid, dim3(256), 0, st, A, lda, m, n, Y,
                         uty + k * SB, center, L.band_rows, Zp);
    else
      hipLaunchKernelGGL(spec_atx_kernel<false>, grid, dim3(256), 0, st, A, lda, m, n, Y,
                         uty + k * SB, center, L.band_rows, Zp);
    hipLaunchKernelGGL(spec_atx_reduce_kernel, dim3((unsigned)ceil_div(n * SB, 256)), dim3(256), 0,
                       st, Zp, L.bands, n, Vs, ldvs, k, S, uty, X);
    orth(st, X, n, part, Rinv);
  }
  apply_e();
  const int parts = tn_parts(m);
  hipLaunchKernelGGL(spec_gram_partial_kernel, dim3(parts), dim3(256), 0, st, Y, m, part);
  hipLaunchKernelGGL(spec_final_kernel, dim3(1), dim3(64), 0, st, part, parts, result);
}

}  // namespace rpca
