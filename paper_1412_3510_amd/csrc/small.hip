// Small dense float64 steps on the device: the l x l Cholesky factorizations
// of Cholesky QR and of the Nystrom method, and the l x l SVD of the
// Rayleigh-Ritz step.  Each runs in one workgroup; none needs the host.
#include "common.h"
#include "kernels.h"
#include "philox.h"
#include "small_core.h"

namespace rpca {

// cond2: pass 2 runs only when pass 1 had to shift (a single Cholesky QR pass
// otherwise)
template <int LP>
__global__ void __launch_bounds__(kCholThreads) chol_qr_kernel(const double* __restrict__ G,
                                                               int l, int pass, int cond2,
                                                               float* __restrict__ Rf,
                                                               int* __restrict__ state) {
  if (pass >= 3 && state[1] == 0) return;
  if (pass == 2 && cond2 && state[0] == 0) return;
  __shared__ __attribute__((aligned(16))) double ubuf[2 * LP];
  __shared__ double diag[LP];
  __shared__ float Rs[LP * LP];
  __shared__ double s_maxd;
  const int tid = threadIdx.x;
  if (pass == 1 && tid < 12) state[tid] = 0;
  if (tid < LP) diag[tid] = (tid < l) ? G[tid * LP + tid] : 0.0;
  __syncthreads();
  if (tid < 64) {  // largest diagonal entry: one wave, shuffle reduction
    double mx = 0.0;
    for (int j = tid; j < l; j += 64) mx = fmax(mx, diag[j]);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
    if (tid == 0) s_maxd = mx;
  }
  __syncthreads();
  const double maxd = s_maxd;
  bool shifted = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    __syncthreads();
    const double srel = attempt ? kShiftRel : 0.0;
    const double sabs = attempt ? (1e-30 * maxd + 1e-300) : 0.0;
    const bool ok = chol_par<LP>(G, false, l, srel, sabs, diag, attempt ? 0.0 : kTauRel, Rs, ubuf);
    if (ok) break;
    if (attempt == 1 && tid == 0) {  // only non-finite input gets here
      state[5] = 1;
      state[kStNonFinite] = 1;  // kept for the rest of the solve
    }
    shifted = true;
  }
  __syncthreads();
  // the float32 factor; rows l .. LP-1 are zero
  for (int e = tid; e < LP * LP; e += kCholThreads) Rf[e] = (e < l * LP) ? Rs[e] : 0.f;
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
}

void launch_chol_qr_step(hipStream_t st, const double* G, int l, int lp, int pass, float* Rf,
                         int* state, bool cond2) {
  const int c2 = cond2 ? 1 : 0;
  switch (lp) {
    case 32: hipLaunchKernelGGL(chol_qr_kernel<32>, dim3(1), dim3(kCholThreads), 0, st, G, l, pass, c2, Rf, state); break;
    case 64: hipLaunchKernelGGL(chol_qr_kernel<64>, dim3(1), dim3(kCholThreads), 0, st, G, l, pass, c2, Rf, state); break;
    case 128: hipLaunchKernelGGL(chol_qr_kernel<128>, dim3(1), dim3(kCholThreads), 0, st, G, l, pass, c2, Rf, state); break;
    default: break;
  }
}

// Replace the dependent columns (state mask) of Q by Gaussian columns.
__global__ void __launch_bounds__(256) complete_kernel(float* __restrict__ Q, int64_t ldq,
                                                       int64_t rows, int l,
                                                       const int* __restrict__ state,
                                                       uint64_t seed) {
  if (state[2] == 0) return;
  const int64_t total = rows * l;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t r = e / l;
    const int j = (int)(e % l);
    if ((((unsigned)state[8 + (j >> 5)]) >> (j & 31)) & 1u)
      Q[r * ldq + j] = philox_normal(seed, 3u, (uint64_t)r * 128u + (uint64_t)j);
  }
}

void launch_complete(hipStream_t st, float* Q, int64_t ldq, int64_t rows, int l, const int* state,
                     uint64_t seed) {
  const int64_t total = rows * l;
  if (total == 0) return;
  // grid-stride: at most 64 K workgroups whatever the size
  const int64_t blocks = ceil_div(total, 256) < 65536 ? ceil_div(total, 256) : 65536;
  hipLaunchKernelGGL(complete_kernel, dim3((unsigned)blocks), dim3(256), 0, st, Q, ldq, rows, l,
                     state, seed);
}

// ------------------------------------------------------------------------
// Nystrom (Section 3): B2 = Q* B1 + nu I (symmetrized), C = chol(B2) upper;
// nu = sqrt(n) u ||B1||_F, multiplied by 10 while the factor does not exist.
// ------------------------------------------------------------------------
template <int LP>
__global__ void __launch_bounds__(kCholThreads) chol_nystrom_kernel(
    const double* __restrict__ G, int l, const double* __restrict__ fro2, double n_sqrt_u,
    float* __restrict__ Rf, double* __restrict__ nu_out, float* __restrict__ nu_f,
    int* __restrict__ state, int max_retries) {
  __shared__ __attribute__((aligned(16))) double ubuf[2 * LP];
  __shared__ double zero[LP];
  __shared__ float Rs[LP * LP];
  const int tid = threadIdx.x;
  if (tid < LP) zero[tid] = 0.0;
  __syncthreads();
  double nu = n_sqrt_u * sqrt(fro2[0]);
  if (!(nu > 0.0)) nu = 1e-300;
  int retry = 0;
  bool ok = false;
  for (; retry <= max_retries; ++retry) {
    __syncthreads();
    // B2 = (G + G^T)/2 + nu I
    ok = chol_par<LP>(G, true, l, 0.0, nu, zero, 0.0, Rs, ubuf);
    if (ok) break;
    if (retry < max_retries) nu *= 10.0;
  }
  __syncthreads();
  if (tid == 0) {
    state[kStRetries] = ok ? retry : max_retries;
    state[kStNotPsd] = ok ? 0 : 1;
    nu_out[0] = nu;
    nu_f[0] = (float)nu;
  }
  // rows l .. LP-1 zero; the identity where no factor was found
  for (int e = tid; e < LP * LP; e += kCholThreads) {
    const int i = e / LP, c = e % LP;
    Rf[e] = ok ? ((i < l) ? Rs[e] : 0.f) : ((i == c && i < l) ? 1.f : 0.f);
  }
}

void launch_chol_nystrom(hipStream_t st, const double* G, int l, int lp, const double* fro2,
                         double n_sqrt_u, float* Rf, double* nu_out, float* nu_f, int* state,
                         int max_retries) {
  switch (lp) {
    case 32: hipLaunchKernelGGL(chol_nystrom_kernel<32>, dim3(1), dim3(kCholThreads), 0, st, G, l, fro2, n_sqrt_u, Rf, nu_out, nu_f, state, max_retries); break;
    case 64: hipLaunchKernelGGL(chol_nystrom_kernel<64>, dim3(1), dim3(kCholThreads), 0, st, G, l, fro2, n_sqrt_u, Rf, nu_out, nu_f, state, max_retries); break;
    case 128: hipLaunchKernelGGL(chol_nystrom_kernel<128>, dim3(1), dim3(kCholThreads), 0, st, G, l, fro2, n_sqrt_u, Rf, nu_out, nu_f, state, max_retries); break;
    default: break;
  }
}


template <int LP, bool GLOBAL, int G, bool ACC>
__global__ void __launch_bounds__(G * LP / 2) jacobi_kernel(const double* __restrict__ M, int l,
                                                     int transpose, double* __restrict__ s_out,
                                                     double* __restrict__ Wacc,
                                                     double* __restrict__ Xn,
                                                     double* __restrict__ gwork, int* flag,
                                                     const int* __restrict__ skip_unless,
                                                     int kneed) {
  if (skip_unless && *skip_unless == 0) return;
  constexpr int CS = jacobi_cs<LP, GLOBAL>();
  __shared__ __attribute__((aligned(16))) double sM[GLOBAL ? 2 : LP * CS];
  __shared__ __attribute__((aligned(16))) double sV[(GLOBAL || !ACC) ? 2 : LP * CS];
  __shared__ double sig[LP];
  __shared__ int perm[LP];
  __shared__ int s_rot, s_big;
  double* Mc = GLOBAL ? gwork : sM;
  double* Vc = GLOBAL ? gwork + LP * CS : sV;
  jacobi_body<LP, GLOBAL, G, ACC>(M, l, transpose, s_out, Wacc, Xn, Mc, Vc, sig, perm, s_rot,
                                  s_big, flag, kneed);
}

void launch_jacobi_svd(hipStream_t st, const double* M, int l, int lp, int transpose, double* s,
                       double* Wacc, double* Xn, double* work, int* flag, int kneed) {
  // lp <= 64: the accumulating form in LDS (a round costs its barrier and
  // reductions, not the rotation of W).  lp = 128, with a flag: rotate the
  // columns alone (in LDS) and recover the rotations by a product; the
  // accumulating form (global memory) runs after it only when the flag says
  // the product is not accurate enough.  Without a flag: the accumulating form.
#define JAC_GO(LP_, GL_, ACC_, NT_, FLAG_, SKIP_, KN_)                                           \
  hipLaunchKernelGGL((jacobi_kernel<LP_, GL_, 16, ACC_>), dim3(1), dim3(NT_), 0, st, M, l,      \
                     transpose, s, Wacc, Xn, work, FLAG_, SKIP_, KN_)
  switch (lp) {
    case 32: JAC_GO(32, false, true, 256, nullptr, nullptr, 0); break;
    case 64: JAC_GO(64, false, true, 512, nullptr, nullptr, 0); break;
    case 128:
      if (flag) JAC_GO(128, false, false, 1024, flag, nullptr, kneed);
      JAC_GO(128, true, true, 1024, nullptr, flag, 0);
      break;
    default: break;
  }
#undef JAC_GO
}

// out[j] = s[j] (nu == nullptr) or max(s[j]^2 - nu, 0).  The status of the
// solve -- kErrNotPsd when the Nystrom factor was never found (state slot
// kStNotPsd), kErrNonFinite when a value returned here, the shift, or an
// earlier Cholesky step (state slot kStNonFinite) was not finite -- is
// OR-ed into status[0] (the caller's sticky word, read at its next
// synchronization) and stored in *slot (nullable: the problem's entry of a
// batch); status[1] receives the Nystrom retry count.
__global__ void finish_values_kernel(const double* __restrict__ s, int k,
                                     const double* __restrict__ nu, double* __restrict__ out,
                                     const int* __restrict__ state, int* __restrict__ status,
                                     int* __restrict__ slot) {
  __shared__ int bad;
  const int j = threadIdx.x;
  if (j == 0) bad = 0;
  __syncthreads();
  if (j < k) {
    const double v = nu ? fmax(s[j] * s[j] - nu[0], 0.0) : s[j];
    out[j] = v;
    if (!isfinite(s[j]) || (nu && !isfinite(nu[0]))) bad = 1;
  }
  __syncthreads();
  if (j == 0) {
    int bits = bad ? kErrNonFinite : 0;
    if (state) {
      if (state[kStNonFinite]) bits |= kErrNonFinite;
      if (nu && state[kStNotPsd]) bits |= kErrNotPsd;
    }
    if (status) {
      if (bits) atomicOr(status, bits);
      if (nu && state) status[1] = state[kStRetries];
    }
    if (slot) *slot = bits;
  }
}

void launch_finish_values(hipStream_t st, const double* s, int k, const double* nu, double* out,
                          const int* state, int* status, int* slot) {
  hipLaunchKernelGGL(finish_values_kernel, dim3(1), dim3(128), 0, st, s, k, nu, out, state,
                     status, slot);
}

// ------------------------------------------------------------------------
// Self-adjoint variants (Section 3's square-root stabilization; the
// Rayleigh-Ritz eigenpairs of a general self-adjoint A).
// ------------------------------------------------------------------------
// G (l x l, stride lp) <- (G + G^T) / 2
__global__ void __launch_bounds__(256) symmetrize_kernel(double* __restrict__ G, int l, int lp) {
  for (int e = threadIdx.x; e < l * l; e += 256) {
    const int i = e / l, j = e % l;
    if (i < j) {
      const double a = 0.5 * (G[i * lp + j] + G[j * lp + i]);
      G[i * lp + j] = a;
      G[j * lp + i] = a;
    }
  }
}

void launch_symmetrize(hipStream_t st, double* G, int l, int lp) {
  hipLaunchKernelGGL(symmetrize_kernel, dim3(1), dim3(256), 0, st, G, l, lp);
}

// M = W diag(w_j^-1/2) over the eigenvalues w_j = s[j] above the cut
// n_sqrt_u * sqrt(fro2[0]) (zero columns for the others): the regularized
// pseudoinverse of the self-adjoint square root C = W diag(w^1/2) W^T of
// B2, applied as B1 C^+ = (B1 M) W^T.  W, M: lp x lp, row-major.
__global__ void __launch_bounds__(256) sqrt_pinv_kernel(const double* __restrict__ W,
                                                        const double* __restrict__ s, int l, int lp,
                                                        const double* __restrict__ fro2,
                                                        double n_sqrt_u, double* __restrict__ M) {
  const double cut = n_sqrt_u * sqrt(fro2[0]);
  for (int e = threadIdx.x; e < lp * lp; e += 256) {
    const int i = e / lp, j = e % lp;
    double v = 0.0;
    if (i < l && j < l && s[j] > cut) v = W[i * lp + j] * rsqrt_nr(s[j]);
    M[e] = v;
  }
}

void launch_sqrt_pinv(hipStream_t st, const double* W, const double* s, int l, int lp,
                      const double* fro2, double n_sqrt_u, double* M) {
  hipLaunchKernelGGL(sqrt_pinv_kernel, dim3(1), dim3(256), 0, st, W, s, l, lp, fro2, n_sqrt_u, M);
}

// Eigenvalues of a symmetric M from its SVD M W = X diag(s): for an
// eigenvector w_j, M w_j = lambda_j w_j, so x_j = sign(lambda_j) w_j and
// lambda_j = s_j sign(w_j . x_j); out[j] for j < k (ordered by |lambda|).
// The status of the solve goes to status / slot as in finish_values_kernel.
__global__ void __launch_bounds__(128) sym_eig_finish_kernel(
    const double* __restrict__ s, const double* __restrict__ W, const double* __restrict__ X,
    int l, int k, int lp, double* __restrict__ out, const int* __restrict__ state,
    int* __restrict__ status, int* __restrict__ slot) {
  __shared__ int bad;
  const int j = threadIdx.x;
  if (j == 0) bad = 0;
  __syncthreads();
  if (j < k) {
    double d = 0.0;
    for (int i = 0; i < l; ++i) d += W[i * lp + j] * X[i * lp + j];
    out[j] = (d < 0.0) ? -s[j] : s[j];
    if (!isfinite(s[j])) bad = 1;
  }
  __syncthreads();
  if (j == 0) {
    int bits = bad ? kErrNonFinite : 0;
    if (state && state[kStNonFinite]) bits |= kErrNonFinite;
    if (status && bits) atomicOr(status, bits);
    if (slot) *slot = bits;
  }
}

void launch_sym_eig_finish(hipStream_t st, const double* s, const double* W, const double* X, int l,
                           int k, int lp, double* out, const int* state, int* status, int* slot) {
  hipLaunchKernelGGL(sym_eig_finish_kernel, dim3(1), dim3(128), 0, st, s, W, X, l, k, lp, out, state,
                     status, slot);
}

}  // namespace rpca
