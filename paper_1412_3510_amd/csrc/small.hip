// Small dense float64 steps on the device: the l x l Cholesky factorizations
// of Cholesky QR and of the Nystrom method, and the l x l SVD of the
// Rayleigh-Ritz step.  Each runs in one workgroup; none needs the host.
#include "common.h"
#include "kernels.h"
#include "philox.h"

namespace rpca {

// state[] layout (int):
//   0  the current orthonormalization shifted a Cholesky factorization
//   1  extra passes 3 and 4 are needed
//   2  dependent columns were replaced by random ones
//   3  Nystrom shift retries
//   4  Nystrom: no positive definite shifted B2 found
//   5  non-finite values met
//   8..11  bit mask of dependent columns (128 bits)
static constexpr double kTauRel = 1e-10;   // relative Cholesky pivot that marks dependence
static constexpr double kShiftRel = 1e-8;  // relative diagonal shift when dependence is met
static constexpr double kJunkNorm2 = 1e-2; // squared column norm after a shifted pass

// Cholesky G = R^T R of the leading l x l block held in LDS (row-major,
// stride LP), in place (upper triangle).  Returns false at the first pivot
// d_j <= tau * ref[j] (or non-finite); all threads agree.
template <int LP>
__device__ bool chol_lds(double* A, int l, const double* ref, double tau, int* s_flag) {
  const int tid = threadIdx.x;
  for (int j = 0; j < l; ++j) {
    __syncthreads();
    const double d = A[j * LP + j];
    if (!(d > tau * ref[j]) || !(d > 0.0) || !(d < 1e300)) return false;
    const double r = sqrt(d);
    const double ri = 1.0 / r;
    __syncthreads();
    for (int c = j + 1 + tid; c < l; c += blockDim.x) A[j * LP + c] *= ri;
    if (tid == 0) A[j * LP + j] = r;
    __syncthreads();
    const int w = l - j - 1;
    for (int e = tid; e < w * w; e += blockDim.x) {
      const int i = j + 1 + e / w, c = j + 1 + e % w;
      if (c >= i) A[i * LP + c] -= A[j * LP + i] * A[j * LP + c];
    }
  }
  __syncthreads();
  (void)s_flag;
  return true;
}

template <int LP>
__global__ void __launch_bounds__(256) chol_qr_kernel(const double* __restrict__ G, int l, int pass,
                                                      float* __restrict__ Rf,
                                                      double* __restrict__ Racc,
                                                      int* __restrict__ state) {
  if (pass >= 3 && state[1] == 0) return;
  __shared__ double A[LP * LP];
  __shared__ double diag[LP];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  if (pass == 1) {
    __syncthreads();
    if (tid < 12) state[tid] = 0;
  }
  for (int j = tid; j < LP; j += blockDim.x) diag[j] = (j < l) ? G[j * LP + j] : 0.0;
  __syncthreads();
  double maxd = 0.0;
  for (int j = 0; j < l; ++j) maxd = fmax(maxd, diag[j]);
  bool shifted = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    __syncthreads();
    const double srel = attempt ? kShiftRel : 0.0;
    const double sabs = attempt ? (1e-30 * maxd + 1e-300) : 0.0;
    for (int e = tid; e < LP * LP; e += blockDim.x) {
      const int i = e / LP, c = e % LP;
      double v = (i < l && c < l) ? G[e] : 0.0;
      if (i == c && i < l) v += srel * diag[i] + sabs;
      A[e] = v;
    }
    __syncthreads();
    const bool ok = chol_lds<LP>(A, l, diag, attempt ? 0.0 : kTauRel, &s_flag);
    if (ok) break;
    if (attempt == 1) {  // only non-finite input can get here
      if (tid == 0) state[5] = 1;
    }
    shifted = true;
  }
  __syncthreads();
  if (tid == 0) {
    if (shifted) state[0] = 1;
    if (pass == 2) {
      // dependent columns of the first pass show up as short columns here
      unsigned mask[4] = {0u, 0u, 0u, 0u};
      int any = 0;
      if (state[0]) {
        for (int j = 0; j < l; ++j)
          if (!(diag[j] >= kJunkNorm2)) {
            mask[j >> 5] |= 1u << (j & 31);
            any = 1;
          }
      }
      for (int w = 0; w < 4; ++w) state[8 + w] = (int)mask[w];
      state[2] = any;
      state[1] = state[0] | any;
    }
  }
  // float32 copy of R for the solve
  for (int e = tid; e < LP * LP; e += blockDim.x) {
    const int i = e / LP, c = e % LP;
    Rf[e] = (i < l && c < l && c >= i) ? (float)A[e] : 0.f;
  }
  if (Racc) {
    __syncthreads();
    if (pass == 1) {
      for (int e = tid; e < LP * LP; e += blockDim.x) {
        const int i = e / LP, c = e % LP;
        Racc[e] = (i < l && c < l && c >= i) ? A[e] : 0.0;
      }
    } else {
      // Racc <- R Racc (both upper triangular)
      constexpr int PER = (LP * LP + 255) / 256;
      double outv[PER];
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = tid + 256 * u;
        double s = 0.0;
        if (e < LP * LP) {
          const int i = e / LP, c = e % LP;
          if (i < l && c < l && c >= i)
            for (int t = i; t <= c; ++t) s += A[i * LP + t] * Racc[t * LP + c];
        }
        outv[u] = s;
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int e = tid + 256 * u;
        if (e < LP * LP) Racc[e] = outv[u];
      }
      __syncthreads();
      if (pass == 2 && state[2]) {
        for (int e = tid; e < LP * LP; e += blockDim.x) {
          const int i = e / LP;
          if (i < l && ((unsigned)state[8 + (i >> 5)] >> (i & 31)) & 1u) Racc[e] = 0.0;
        }
      }
    }
  }
}

void launch_chol_qr_step(hipStream_t st, const double* G, int l, int lp, int pass, float* Rf,
                         double* Racc, int* state) {
  switch (lp) {
    case 32: hipLaunchKernelGGL(chol_qr_kernel<32>, dim3(1), dim3(256), 0, st, G, l, pass, Rf, Racc, state); break;
    case 64: hipLaunchKernelGGL(chol_qr_kernel<64>, dim3(1), dim3(256), 0, st, G, l, pass, Rf, Racc, state); break;
    case 128: hipLaunchKernelGGL(chol_qr_kernel<128>, dim3(1), dim3(256), 0, st, G, l, pass, Rf, Racc, state); break;
    default: break;
  }
}

// Replace the dependent columns (state mask) of Q by Gaussian columns.
__global__ void __launch_bounds__(256) complete_kernel(float* __restrict__ Q, int64_t ldq,
                                                       int64_t rows, int l,
                                                       const int* __restrict__ state,
                                                       uint64_t seed) {
  if (state[2] == 0) return;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t r = e / l;
  const int j = (int)(e % l);
  if (r >= rows) return;
  if ((((unsigned)state[8 + (j >> 5)]) >> (j & 31)) & 1u)
    Q[r * ldq + j] = philox_normal(seed, 3u, (uint64_t)r * 128u + (uint64_t)j);
}

void launch_complete(hipStream_t st, float* Q, int64_t ldq, int64_t rows, int l, const int* state,
                     uint64_t seed) {
  const int64_t total = rows * l;
  if (total == 0) return;
  hipLaunchKernelGGL(complete_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, Q,
                     ldq, rows, l, state, seed);
}

// ------------------------------------------------------------------------
// Nystrom (Section 3): B2 = Q* B1 + nu I (symmetrized), C = chol(B2) upper;
// nu = sqrt(n) u ||B1||_F, multiplied by 10 while the factor does not exist.
// ------------------------------------------------------------------------
template <int LP>
__global__ void __launch_bounds__(256) chol_nystrom_kernel(const double* __restrict__ G, int l,
                                                           const double* __restrict__ fro2,
                                                           double n_sqrt_u, float* __restrict__ Rf,
                                                           double* __restrict__ nu_out,
                                                           float* __restrict__ nu_f,
                                                           int* __restrict__ state,
                                                           int max_retries) {
  __shared__ double A[LP * LP];
  __shared__ double zero[LP];
  __shared__ int s_flag;
  const int tid = threadIdx.x;
  for (int j = tid; j < LP; j += blockDim.x) zero[j] = 0.0;
  double nu = n_sqrt_u * sqrt(fro2[0]);
  if (!(nu > 0.0)) nu = 1e-300;
  int retry = 0;
  bool ok = false;
  for (; retry <= max_retries; ++retry) {
    __syncthreads();
    for (int e = tid; e < LP * LP; e += blockDim.x) {
      const int i = e / LP, c = e % LP;
      double v = 0.0;
      if (i < l && c < l) v = 0.5 * (G[i * LP + c] + G[c * LP + i]) + (i == c ? nu : 0.0);
      A[e] = v;
    }
    __syncthreads();
    ok = chol_lds<LP>(A, l, zero, 0.0, &s_flag);
    if (ok) break;
    if (retry < max_retries) nu *= 10.0;
  }
  __syncthreads();
  if (tid == 0) {
    state[3] = ok ? retry : max_retries;
    state[4] = ok ? 0 : 1;
    nu_out[0] = nu;
    nu_f[0] = (float)nu;
  }
  for (int e = tid; e < LP * LP; e += blockDim.x) {
    const int i = e / LP, c = e % LP;
    Rf[e] = (ok && i < l && c < l && c >= i) ? (float)A[e] : (i == c ? 1.f : 0.f);
  }
}

void launch_chol_nystrom(hipStream_t st, const double* G, int l, int lp, const double* fro2,
                         double n_sqrt_u, float* Rf, double* nu_out, float* nu_f, int* state,
                         int max_retries) {
  switch (lp) {
    case 32: hipLaunchKernelGGL(chol_nystrom_kernel<32>, dim3(1), dim3(256), 0, st, G, l, fro2, n_sqrt_u, Rf, nu_out, nu_f, state, max_retries); break;
    case 64: hipLaunchKernelGGL(chol_nystrom_kernel<64>, dim3(1), dim3(256), 0, st, G, l, fro2, n_sqrt_u, Rf, nu_out, nu_f, state, max_retries); break;
    case 128: hipLaunchKernelGGL(chol_nystrom_kernel<128>, dim3(1), dim3(256), 0, st, G, l, fro2, n_sqrt_u, Rf, nu_out, nu_f, state, max_retries); break;
    default: break;
  }
}

// ------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of M (or M^T), l <= LP, in float64.
// Columns are stored contiguously (Mc[j*LP + i] = column j, row i).  Column
// pairs follow the round-robin (circle) ordering, l/2 disjoint pairs per
// round, each pair on a group of G lanes.  With M Wacc = Xn diag(s):
//   s    -- column norms, sorted descending
//   Wacc -- accumulated rotations (orthogonal), columns in the same order
//   Xn   -- normalized columns of M Wacc (zero where s = 0)
// For M = R (B^T = Q2 R) the left singular vectors of B are Wacc and the
// right ones Q2 Xn; for M = R^T (F = QF R) the left ones of F are QF Wacc.
// ------------------------------------------------------------------------
template <int LP, bool GLOBAL>
__global__ void __launch_bounds__(256) jacobi_kernel(const double* __restrict__ M, int l,
                                                     int transpose, double* __restrict__ s_out,
                                                     double* __restrict__ Wacc,
                                                     double* __restrict__ Xn,
                                                     double* __restrict__ gwork) {
  // column stride padded by one double in LDS so that the columns of
  // different pairs fall in different banks
  constexpr int CS = GLOBAL ? LP : LP + 1;
  __shared__ double sM[GLOBAL ? 1 : LP * CS];
  __shared__ double sV[GLOBAL ? 1 : LP * CS];
  __shared__ double sig[LP];
  __shared__ int perm[LP];
  __shared__ int s_rot;
  double* Mc = GLOBAL ? gwork : sM;
  double* Vc = GLOBAL ? gwork + LP * CS : sV;
  const int tid = threadIdx.x;
  for (int e = tid; e < LP * LP; e += 256) {
    const int j = e / LP, i = e % LP;
    double v = 0.0;
    if (i < l && j < l) v = transpose ? M[j * LP + i] : M[i * LP + j];
    Mc[j * CS + i] = v;
    Vc[j * CS + i] = (i == j) ? 1.0 : 0.0;
  }
  const int lp2 = l + (l & 1);
  const int npairs = lp2 / 2;
  int G = 64;
  while (G > 1 && G * npairs > 256) G >>= 1;
  const int k = tid / G, gl = tid % G;
  const bool active = (k < npairs);
  const double tol = 1e-13;
  for (int sweep = 0; sweep < 60; ++sweep) {
    __syncthreads();
    if (tid == 0) s_rot = 0;
    __syncthreads();
    for (int r = 0; r < lp2 - 1; ++r) {
      int p = 0, q = 0;
      if (active) {
        const int a = k, b = lp2 - 1 - k;
        p = (a == 0) ? 0 : 1 + (a - 1 + r) % (lp2 - 1);
        q = (b == 0) ? 0 : 1 + (b - 1 + r) % (lp2 - 1);
      }
      double al = 0.0, be = 0.0, ga = 0.0;
      if (active && p < l && q < l) {
        for (int i = gl; i < l; i += G) {
          const double mp = Mc[p * CS + i], mq = Mc[q * CS + i];
          al += mp * mp;
          be += mq * mq;
          ga += mp * mq;
        }
      }
      al = group_sum(al, G);
      be = group_sum(be, G);
      ga = group_sum(ga, G);
      if (active && p < l && q < l && al > 0.0 && be > 0.0 && fabs(ga) > tol * sqrt(al * be)) {
        const double zeta = (be - al) / (2.0 * ga);
        const double t = ((zeta >= 0.0) ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        for (int i = gl; i < l; i += G) {
          const double mp = Mc[p * CS + i], mq = Mc[q * CS + i];
          Mc[p * CS + i] = c * mp - s * mq;
          Mc[q * CS + i] = s * mp + c * mq;
          const double vp = Vc[p * CS + i], vq = Vc[q * CS + i];
          Vc[p * CS + i] = c * vp - s * vq;
          Vc[q * CS + i] = s * vp + c * vq;
        }
        if (gl == 0) s_rot = 1;
      }
      __syncthreads();
    }
    if (s_rot == 0) break;
  }
  __syncthreads();
  if (tid < LP) {
    double s = 0.0;
    if (tid < l)
      for (int i = 0; i < l; ++i) s += Mc[tid * CS + i] * Mc[tid * CS + i];
    sig[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < l) {
    int rank = 0;
    for (int i = 0; i < l; ++i)
      if (sig[i] > sig[tid] || (sig[i] == sig[tid] && i < tid)) ++rank;
    perm[rank] = tid;
  }
  __syncthreads();
  for (int e = tid; e < LP * LP; e += 256) {
    const int i = e / LP, rr = e % LP;  // output row i, column rr
    double w = 0.0, x = 0.0;
    if (i < l && rr < l) {
      const int j = perm[rr];
      w = Vc[j * CS + i];
      x = (sig[j] > 0.0) ? Mc[j * CS + i] / sig[j] : 0.0;
    }
    Wacc[e] = w;
    Xn[e] = x;
  }
  if (tid < LP) s_out[tid] = (tid < l) ? sig[perm[tid]] : 0.0;
}

void launch_jacobi_svd(hipStream_t st, const double* M, int l, int lp, int transpose, double* s,
                       double* Wacc, double* Xn, double* work) {
  switch (lp) {
    case 32: hipLaunchKernelGGL((jacobi_kernel<32, false>), dim3(1), dim3(256), 0, st, M, l, transpose, s, Wacc, Xn, work); break;
    case 64: hipLaunchKernelGGL((jacobi_kernel<64, false>), dim3(1), dim3(256), 0, st, M, l, transpose, s, Wacc, Xn, work); break;
    case 128: hipLaunchKernelGGL((jacobi_kernel<128, true>), dim3(1), dim3(256), 0, st, M, l, transpose, s, Wacc, Xn, work); break;
    default: break;
  }
}

// out[j] = s[j] (nu == nullptr) or max(s[j]^2 - nu, 0)
__global__ void finish_values_kernel(const double* __restrict__ s, int k,
                                     const double* __restrict__ nu, double* __restrict__ out) {
  const int j = threadIdx.x;
  if (j >= k) return;
  out[j] = nu ? fmax(s[j] * s[j] - nu[0], 0.0) : s[j];
}

void launch_finish_values(hipStream_t st, const double* s, int k, const double* nu, double* out) {
  hipLaunchKernelGGL(finish_values_kernel, dim3(1), dim3(128), 0, st, s, k, nu, out);
}

}  // namespace rpca
