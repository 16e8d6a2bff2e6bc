// LDS-DMA helpers shared by the passes over A (gemm.hip, gemm_lp.hip).
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


}  // namespace rpca
