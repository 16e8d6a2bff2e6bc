// Passes over a sparse A (Section 8 applies the method to sparse matrices:
// only products with A and A* are needed, so A is never densified).
//
// A is given in CSR (rows of A) and CSC (rows of A^T); both products are the
// same gather kernel: out[i][:] = sum over the stored entries k of row i of
// val[k] X[idx[k]][:], for X tall and skinny (n x lp float32, row-major, zero
// beyond column l).  A row of the output is owned by TPR = min(lp, 64) lanes,
// lane c accumulating columns c, c + TPR, ... in float32; the entry's index
// and value are uniform over those lanes, the gathered X row is one coalesced
// segment.  Entries are taken four at a time so that four gathers are in
// flight per lane.  The order of accumulation is fixed (ascending k), so the
// result does not depend on scheduling.  Offsets are clamped to [0, nnz] and
// indices to [0, ncols): malformed arrays give wrong numbers, never an
// access outside them.
#include "common.h"
#include "kernels.h"

namespace rpca {

template <typename V>
__device__ __forceinline__ float ldval(const V* p, int64_t k);
template <>
__device__ __forceinline__ float ldval<float>(const float* p, int64_t k) { return p[k]; }
template <>
__device__ __forceinline__ float ldval<__bf16>(const __bf16* p, int64_t k) {
  return static_cast<float>(p[k]);
}

template <int LP, typename V>
__global__ void __launch_bounds__(256) spmm_kernel(const int* __restrict__ ptr,
                                                   const int* __restrict__ idx,
                                                   const V* __restrict__ val, int64_t nrows,
                                                   int64_t nnz, int ncols,
                                                   const float* __restrict__ X, int64_t ldx,
                                                   float* __restrict__ Y, int64_t ldy) {
  constexpr int TPR = LP < 64 ? LP : 64;  // lanes per output row
  constexpr int CPT = LP / TPR;           // columns per lane
  constexpr int RPB = 256 / TPR;          // rows per workgroup
  const int c = threadIdx.x % TPR;
  const int64_t i = (int64_t)blockIdx.x * RPB + threadIdx.x / TPR;
  if (i >= nrows) return;
  const int64_t k0 = min<int64_t>(max(ptr[i], 0), nnz);
  const int64_t k1 = max<int64_t>(min<int64_t>(ptr[i + 1], nnz), k0);
  float acc[CPT];
#pragma unroll
  for (int u = 0; u < CPT; ++u) acc[u] = 0.f;
  int64_t k = k0;
  for (; k + 4 <= k1; k += 4) {
    int j[4];
    float v[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      j[t] = min(max(idx[k + t], 0), ncols - 1);
      v[t] = ldval<V>(val, k + t);
    }
    float x[4][CPT];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < CPT; ++u) x[t][u] = X[(int64_t)j[t] * ldx + c + TPR * u];
#pragma unroll
    for (int t = 0; t < 4; ++t)
#pragma unroll
      for (int u = 0; u < CPT; ++u) acc[u] += v[t] * x[t][u];
  }
  for (; k < k1; ++k) {
    const int j = min(max(idx[k], 0), ncols - 1);
    const float v = ldval<V>(val, k);
#pragma unroll
    for (int u = 0; u < CPT; ++u) acc[u] += v * X[(int64_t)j * ldx + c + TPR * u];
  }
#pragma unroll
  for (int u = 0; u < CPT; ++u) Y[i * ldy + c + TPR * u] = acc[u];
}

void launch_spmm(hipStream_t st, const int* ptr, const int* idx, const void* val, int dtype,
                 int64_t nrows, int64_t nnz, int ncols, const float* X, int64_t ldx, float* Y,
                 int64_t ldy, int lp) {
  if (nrows <= 0) return;
  const int tpr = lp < 64 ? lp : 64;
  const unsigned grid = (unsigned)ceil_div(nrows, 256 / tpr);
#define SPMM_GO(LP_, V_)                                                                       \
  hipLaunchKernelGGL((spmm_kernel<LP_, V_>), dim3(grid), dim3(256), 0, st, ptr, idx,           \
                     static_cast<const V_*>(val), nrows, nnz, ncols, X, ldx, Y, ldy)
  if (dtype == 1) {
    switch (lp) {
      case 32: SPMM_GO(32, __bf16); break;
      case 64: SPMM_GO(64, __bf16); break;
      case 128: SPMM_GO(128, __bf16); break;
      default: break;
    }
  } else {
    switch (lp) {
      case 32: SPMM_GO(32, float); break;
      case 64: SPMM_GO(64, float); break;
      case 128: SPMM_GO(128, float); break;
      default: break;
    }
  }
#undef SPMM_GO
}

// out[i][q] = sum_k val[k] X[idx[k]][q], q < 4, float64 accumulation (the
// power method of the error estimate); one thread per row.
template <typename V>
__global__ void __launch_bounds__(256) spmm4_f64_kernel(const int* __restrict__ ptr,
                                                        const int* __restrict__ idx,
                                                        const V* __restrict__ val, int64_t nrows,
                                                        int64_t nnz, int ncols,
                                                        const double* __restrict__ X,
                                                        double* __restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nrows) return;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int64_t k0 = min<int64_t>(max(ptr[i], 0), nnz);
  const int64_t k1 = max<int64_t>(min<int64_t>(ptr[i + 1], nnz), k0);
  for (int64_t k = k0; k < k1; ++k) {
    const double v = (double)ldval<V>(val, k);
    const int j = min(max(idx[k], 0), ncols - 1);
    const double2* x = reinterpret_cast<const double2*>(X + (int64_t)j * 4);
    const double2 p = x[0], q = x[1];
    a0 += v * p.x;
    a1 += v * p.y;
    a2 += v * q.x;
    a3 += v * q.y;
  }
  double2* y = reinterpret_cast<double2*>(Y + i * 4);
  y[0] = make_double2(a0, a1);
  y[1] = make_double2(a2, a3);
}

void launch_spmm4_f64(hipStream_t st, const int* ptr, const int* idx, const void* val, int dtype,
                      int64_t nrows, int64_t nnz, int ncols, const double* X, double* Y) {
  if (nrows <= 0) return;
  const unsigned grid = (unsigned)ceil_div(nrows, 256);
  if (dtype == 1)
    hipLaunchKernelGGL(spmm4_f64_kernel<__bf16>, dim3(grid), dim3(256), 0, st, ptr, idx,
                       static_cast<const __bf16*>(val), nrows, nnz, ncols, X, Y);
  else
    hipLaunchKernelGGL(spmm4_f64_kernel<float>, dim3(grid), dim3(256), 0, st, ptr, idx,
                       static_cast<const float*>(val), nrows, nnz, ncols, X, Y);
}

}  // namespace rpca
