// Gaussian test matrix from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
//
// The paper draws the test vectors i.i.d. N(0,1) (Section 2) and notes the
// method does not depend on the generator's quality (Section 5).  The
// generator is counter based so that every entry is a pure function of
// (seed, stream, index): one thread produces one 4-word block.
//
//   key     = (seed mod 2^32, seed >> 32)
//   counter = (t mod 2^32, t >> 32, stream, 0)  for block t
//   words (x0, x1) -> (z0, z1), (x2, x3) -> (z2, z3) by Box-Muller in float64:
//       u = (x + 1/2) 2^-32, r = sqrt(-2 ln u_a), theta = 2 pi u_b,
//       (r cos theta, r sin theta), then rounded once to float32
//   Omega[i, j] = z[j*n + i]
// or, for the uniform test matrix, each word on its own:
//   v = (x + 1/2) 2^-31 - 1 (float64, exact), rounded to float32
#include "common.h"
#include "kernels.h"
#include "philox.h"

namespace rpca {

// One thread per block of four normals; element e = 4t + q maps to
// Omega[e % n, e / n].
__global__ void __launch_bounds__(256) gaussian_kernel(uint64_t seed, uint32_t stream, int64_t n,
                                                       int64_t l, float* __restrict__ out,
                                                       int64_t ldo, uint32_t* __restrict__ words,
                                                       int uniform) {
  const int64_t total = n * l;
  const int64_t nb = (total + 3) / 4;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nb) return;
  uint32_t c[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), stream, 0u};
  philox_block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  if (words) {
#pragma unroll
    for (int q = 0; q < 4; ++q) words[4 * t + q] = c[q];
  }
  float z[4];
  if (uniform) {
#pragma unroll
    for (int q = 0; q < 4; ++q) z[q] = word_uniform(c[q]);
  } else {
    box_muller(c[0], c[1], z[0], z[1]);
    box_muller(c[2], c[3], z[2], z[3]);
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int64_t e = 4 * t + q;
    if (e < total) {
      const int64_t j = e / n, i = e - j * n;
      out[i * ldo + j] = z[q];
    }
  }
}

void launch_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                     float* out, int64_t ldo, uint32_t* words, bool uniform) {
  const int64_t nb = (n * l + 3) / 4;
  if (nb == 0) return;
  const int64_t grid = (nb + 255) / 256;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)grid), dim3(256), 0, st, seed, stream, n, l,
                     out, ldo, words, uniform ? 1 : 0);
}

}  // namespace rpca
