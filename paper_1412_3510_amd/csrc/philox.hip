// Gaussian test matrix from Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).
//
// The paper draws the test vectors i.i.d. N(0,1) (Section 2) and notes the
// method does not depend on the generator's quality (Section 5).  The
// generator is counter based so that every entry is a pure function of
// (seed, stream, index), whichever thread computes it.
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

// A workgroup owns a tile of Omega (row-major, leading dimension ldo): R
// consecutive rows and up to kGaussCols consecutive columns, and writes it
// row by row.  Variate e = j n + i is entry (i, j), so the rows of one
// column j are the consecutive variates j n + r0 .. j n + r1 - 1: the
// workgroup runs the Philox blocks that cover them (R / 4 + 1 per column at
// most; a block that straddles two columns or two tiles is run by each, with
// the same result) and keeps the entries of its tile in LDS.  Writing each
// block's four entries straight to Omega would put them in four different
// rows, one 4-byte piece of a cache line each.
constexpr int kGaussTile = 8448;  // LDS floats: R (columns + 1) <= kGaussTile
constexpr int kGaussCols = 128;

__global__ void __launch_bounds__(256) gaussian_kernel(uint64_t seed, uint32_t stream, int64_t n,
                                                       int64_t l, int R, int rtiles,
                                                       float* __restrict__ out, int64_t ldo,
                                                       uint32_t* __restrict__ words, int uniform) {
  __shared__ float tile[kGaussTile];
  const int64_t r0 = (int64_t)(blockIdx.x % rtiles) * R;
  const int64_t r1 = (r0 + R < n) ? r0 + R : n;
  const int64_t c0 = (int64_t)(blockIdx.x / rtiles) * kGaussCols;
  const int cw = (int)((c0 + kGaussCols < l) ? kGaussCols : l - c0);
  const int LT = cw + 1;      // tile row stride
  const int CB = R / 4 + 1;   // blocks per column, at most
  for (int k = threadIdx.x; k < CB * cw; k += 256) {
    const int jl = k / CB;
    const int64_t j = c0 + jl;
    const int64_t elo = j * n + r0, ehi = j * n + r1;  // this column's variates here
    const int64_t t = elo / 4 + (k - jl * CB);
    if (4 * t >= ehi) continue;
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
      if (e >= elo && e < ehi) tile[(int)(e - elo) * LT + jl] = z[q];
    }
  }
  __syncthreads();
  const int nr = (int)(r1 - r0);
  for (int idx = threadIdx.x; idx < nr * cw; idx += 256) {
    const int rr = idx / cw, jl = idx - rr * cw;
    out[(r0 + rr) * ldo + c0 + jl] = tile[rr * LT + jl];
  }
}

void launch_gaussian(hipStream_t st, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                     float* out, int64_t ldo, uint32_t* words, bool uniform) {
  if (n <= 0 || l <= 0) return;
  // rows per tile: a multiple of 4, at most 256, with the tile in LDS; for
  // small n fewer (down to 8), so that about 1024 workgroups share the work
  // (each block of four variates is a long float64 computation)
  const int64_t cw = l < kGaussCols ? l : kGaussCols;
  int R = (int)(kGaussTile / (cw + 1)) & ~3;
  R = R > 256 ? 256 : R;
  const int64_t rpar = ((n + 1023) / 1024 + 3) & ~(int64_t)3;
  if (rpar < R) R = rpar > 8 ? (int)rpar : 8;
  const int64_t rtiles = (n + R - 1) / R;
  const int64_t ctiles = (l + kGaussCols - 1) / kGaussCols;
  hipLaunchKernelGGL(gaussian_kernel, dim3((unsigned)(rtiles * ctiles)), dim3(256), 0, st, seed,
                     stream, n, l, R, (int)rtiles, out, ldo, words, uniform ? 1 : 0);
}

}  // namespace rpca
