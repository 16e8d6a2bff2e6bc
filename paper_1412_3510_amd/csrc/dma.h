// Helpers shared by the passes over A (gemm.hip, gemm_lp.hip, ax_tall.hip):
// LDS-DMA copies and waits, the split product and the E4M3 widening.
#pragma once
#include "common.h"

namespace rpca {

static constexpr int kFragElems = 512;  // bf16 per 1 KB fragment

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of logical tile ids so tiles that share operands share an
// L2.
__device__ __forceinline__ int xcd_remap(int b, int nwg) {
  if (nwg % 8 != 0) return b;
  return (b % 8) * (nwg / 8) + b / 8;
}

typedef __attribute__((address_space(3))) char lds_char;

// 16 bytes per lane, global -> LDS at lds_block + 16 * lane.  Written as
// inline assembly (M0 = LDS base, no VGPR result) so that the compiler does
// not guard every later LDS read with a wait for all outstanding copies; the
// kernels wait for exactly the stage they read with wait_vm_barrier.
__device__ __forceinline__ void dma16(const void* g, char* lds_block) {
  const unsigned la = __builtin_amdgcn_readfirstlane((unsigned)(size_t)((lds_char*)lds_block));
  asm volatile("s_mov_b32 m0, %1\n\tglobal_load_lds_dwordx4 %0, off" ::"v"(g), "s"(la)
               : "memory", "m0");
}

// Wait until at most N DMA instructions of this wave are outstanding, then
// synchronize the workgroup.  The memory clobber keeps LDS reads below.
template <int N>
__device__ __forceinline__ void wait_vm_barrier() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  asm volatile("s_waitcnt vmcnt(%0)\n\ts_barrier" ::"n"(N) : "memory");
}
__device__ __forceinline__ void barrier_mem() { asm volatile("s_barrier" ::: "memory"); }

// Wait for the oldest issued stage when ``ahead`` later stages (0 .. S-1) are
// already in flight, PER DMA instructions per stage and wave.
template <int PER, int S>
__device__ __forceinline__ void wait_ahead(int ahead) {
  constexpr int M = S - 1;
  switch (ahead) {
    case 0: wait_vm_barrier<0>(); break;
    case 1: wait_vm_barrier<PER>(); break;
    case 2: wait_vm_barrier<(M >= 2 ? 2 : M) * PER>(); break;
    case 3: wait_vm_barrier<(M >= 3 ? 3 : M) * PER>(); break;
    case 4: wait_vm_barrier<(M >= 4 ? 4 : M) * PER>(); break;
    case 5: wait_vm_barrier<(M >= 5 ? 5 : M) * PER>(); break;
    default: wait_vm_barrier<(M >= 6 ? 6 : M) * PER>(); break;
  }
}

// Wait as wait_vm_barrier for a count known only at run time (at most 32;
// a larger count waits for 32, which is stricter).
__device__ __forceinline__ void wait_vm_barrier_n(int n) {
#define RPCA_WN(N) case N: wait_vm_barrier<N>(); break;
  switch (n) {
    RPCA_WN(0) RPCA_WN(1) RPCA_WN(2) RPCA_WN(3) RPCA_WN(4) RPCA_WN(5) RPCA_WN(6) RPCA_WN(7)
    RPCA_WN(8) RPCA_WN(9) RPCA_WN(10) RPCA_WN(11) RPCA_WN(12) RPCA_WN(13) RPCA_WN(14)
    RPCA_WN(15) RPCA_WN(16) RPCA_WN(17) RPCA_WN(18) RPCA_WN(19) RPCA_WN(20) RPCA_WN(21)
    RPCA_WN(22) RPCA_WN(23) RPCA_WN(24) RPCA_WN(25) RPCA_WN(26) RPCA_WN(27) RPCA_WN(28)
    RPCA_WN(29) RPCA_WN(30) RPCA_WN(31)
    default: wait_vm_barrier<32>(); break;
  }
#undef RPCA_WN
}

// A B with A and B split into bfloat16 (hi, lo) pairs: hi hi + hi lo + lo hi
// on v_mfma_f32_32x32x16_bf16, smallest terms first.
__device__ __forceinline__ f32x16 mfma3(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                        const bf16x8& bl, f32x16 acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
  return acc;
}

// split_bf16 of eight floats, two at a time: one packed conversion for the
// high parts, their float values by shifting and masking the packed word, the
// exact differences, one packed conversion for the low parts (the same
// round-to-nearest-even results as split_bf16, in 24 instead of 32 VALU ops).
__device__ __forceinline__ void split_bf16x8(const float4& a0, const float4& a1, bf16x8& hi,
                                             bf16x8& lo) {
  typedef float f32x2v __attribute__((ext_vector_type(2)));
  typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
  const float v[8] = {a0.x, a0.y, a0.z, a0.w, a1.x, a1.y, a1.z, a1.w};
  unsigned hw[4], lw[4];
#pragma unroll
  for (int p = 0; p < 4; ++p) {
    const f32x2v x = {v[2 * p], v[2 * p + 1]};
    const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector(x, bf16x2v));
    const f32x2v r = {x[0] - __uint_as_float(h << 16), x[1] - __uint_as_float(h & 0xffff0000u)};
    hw[p] = h;
    lw[p] = __builtin_bit_cast(unsigned, __builtin_convertvector(r, bf16x2v));
  }
  hi = __builtin_bit_cast(bf16x8, hw);
  lo = __builtin_bit_cast(bf16x8, lw);
}

// 8 E4M3 values (two dwords, low byte first) -> 8 bfloat16, exact: every
// E4M3 value is a bfloat16 value, and v_cvt_scalef32_pk_bf16_fp8 with a
// scale of 1 widens two bytes (the low or the high half of the dword) at once.
__device__ __forceinline__ bf16x8 fp8x8_to_bf16(unsigned w0, unsigned w1) {
  unsigned p[4];
  p[0] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, false));
  p[1] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w0, 1.0f, true));
  p[2] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, false));
  p[3] = __builtin_bit_cast(unsigned, __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w1, 1.0f, true));
  return __builtin_bit_cast(bf16x8, p);
}

}  // namespace rpca
