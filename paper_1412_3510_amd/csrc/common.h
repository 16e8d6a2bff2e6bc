// Shared device helpers for the randomized PCA kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

#define RPCA_WAVE 64

// Split a float into a bfloat16 pair (hi, lo) with x ~ hi + lo; both rounded
// to nearest even.  hi + lo carries 16 significant bits of x; the products
// hi*hi' + hi*lo' + lo*hi' reproduce x*x' to about 2^-16 relative.
__device__ __forceinline__ void split_bf16(float x, __bf16& hi, __bf16& lo) {
  hi = static_cast<__bf16>(x);
  lo = static_cast<__bf16>(x - static_cast<float>(hi));
}

// Wave-wide reductions (64 lanes).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double group_sum(double v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Argmax of (key, idx) over a wave: larger key wins, ties go to the smaller
// idx.  Keys below zero mark "no candidate".
__device__ __forceinline__ void wave_argmax(float& key, int& idx) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    float k2 = __shfl_xor(key, o, 64);
    int i2 = __shfl_xor(idx, o, 64);
    if (k2 > key || (k2 == key && i2 < idx)) {
      key = k2;
      idx = i2;
    }
  }
}

// The same argmax with DPP lane permutations: quad swaps, half-row and row
// mirrors inside each 16-lane row, then row_bcast:15 / row_bcast:31 across
// rows; lane 63 ends with the wave's result, read back with one readlane.
// Branch-free (selects), so the chain is a few dozen dependent VALU ops.
__device__ __forceinline__ int dpp_sel(int v, int ctrl_sel) {
  switch (ctrl_sel) {
    case 0: return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    case 1: return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    case 2: return __builtin_amdgcn_update_dpp(v, v, 0x141, 0xF, 0xF, false);  // row_half_mirror
    case 3: return __builtin_amdgcn_update_dpp(v, v, 0x140, 0xF, 0xF, false);  // row_mirror
    case 4: return __builtin_amdgcn_update_dpp(v, v, 0x142, 0xA, 0xF, false);  // row_bcast:15
    default: return __builtin_amdgcn_update_dpp(v, v, 0x143, 0xC, 0xF, false); // row_bcast:31
  }
}

__device__ __forceinline__ void argmax_combine(float& key, int& idx, int ctrl_sel) {
  const float k2 = __int_as_float(dpp_sel(__float_as_int(key), ctrl_sel));
  const int i2 = dpp_sel(idx, ctrl_sel);
  const bool take = (k2 > key) | ((k2 == key) & (i2 < idx));
  key = take ? k2 : key;
  idx = take ? i2 : idx;
}

__device__ __forceinline__ void wave_argmax_fast(float& key, int& idx) {
#pragma unroll
  for (int s = 0; s < 6; ++s) argmax_combine(key, idx, s);
  key = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(key), 63));
  idx = __builtin_amdgcn_readlane(idx, 63);
}

__host__ __device__ inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
__host__ __device__ inline int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
