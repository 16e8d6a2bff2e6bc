// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the Box-Muller map
// used for every random matrix the method draws.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rpca {

static constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
static constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;

__device__ __forceinline__ void philox_block(uint32_t c[4], uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += kW0;
      k1 += kW1;
    }
    const uint32_t lo0 = kM0 * c[0], hi0 = __umulhi(kM0, c[0]);
    const uint32_t lo1 = kM1 * c[2], hi1 = __umulhi(kM1, c[2]);
    const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
  }
}

__device__ __forceinline__ void box_muller(uint32_t xa, uint32_t xb, float& z0, float& z1) {
  const double two_m32 = 2.3283064365386963e-10;  // 2^-32
  const double ua = ((double)xa + 0.5) * two_m32;
  const double ub = ((double)xb + 0.5) * two_m32;
  const double r = sqrt(-2.0 * log(ua));
  const double th = 6.283185307179586 * ub;
  z0 = (float)(r * cos(th));
  z1 = (float)(r * sin(th));
}


// The uniform alternative (Section 5: uniform draws on [-1, 1] serve as well):
// word x -> (x + 1/2) 2^-31 - 1, exact in float64, rounded once to float32.
__device__ __forceinline__ float word_uniform(uint32_t x) {
  return (float)(((double)x + 0.5) * 4.656612873077393e-10 - 1.0);  // 2^-31
}

// Normal variate number e (e = 4t + q) of stream ``stream`` under ``seed``.
__device__ __forceinline__ float philox_normal(uint64_t seed, uint32_t stream, uint64_t e) {
  const uint64_t t = e >> 2;
  uint32_t c[4] = {(uint32_t)t, (uint32_t)(t >> 32), stream, 0u};
  philox_block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
  float z0, z1;
  const int q = (int)(e & 3);
  if (q < 2) box_muller(c[0], c[1], z0, z1);
  else box_muller(c[2], c[3], z0, z1);
  return (q & 1) ? z1 : z0;
}

}  // namespace rpca
