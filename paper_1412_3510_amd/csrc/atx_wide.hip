// Partials of A^T X, wide form, for the float32 A (products as three
// bfloat16 terms of the split operands) and its bfloat16 and E4M3 copies
// (one term on the operand's high part; the E4M3 column scales apply to the
// rows of the reduced result).  Section 2 prices the method by its passes over A;
// what this kernel changes against the 128- and 256-column tiles of
// gemm_lp.hip is the share of each stage that the packed m-side operand
// takes, and how often that operand is read:
//
//  * 8 waves own two 32-column blocks each: tiles of 512 columns.  A stage
//    is 32 KB of A -- 16 rows of float32, 32 of bfloat16 or 64 of E4M3 --
//    and the operand fragments of those rows (8 KB, 16 KB for E4M3 at
//    lp = 128)
//    serve all 512 columns; at 128 columns, E4M3 stages held 16 KB of A and
//    32 KB of operand.  The operand is read once per column tile, so 16
//    times at n = 8000 instead of 63.
//  * One barrier per stage both publishes a stage and frees the slot of the
//    stage before (as in the tall form of A X); the wait before a stage
//    counts this wave's copies issued after it.
//
// LDS: row k of a stage occupies RB = 512 E bytes; its 16-byte chunk c sits
// at position c ^ (2 E ((k >> 3) & 1)), so that the two halves of a wave,
// which read 32 E bytes each in rows 8 apart, fall on different banks.  A
// 1 KB DMA block is half a float32 row, one bfloat16 row or two E4M3 rows;
// block q is issued by wave q % 8.  Each
// lane gathers the 8 entries of its column in 8 consecutive rows of a K16
// step (the B operand of v_mfma_f32_32x32x16_bf16); the operand fragment is
// the A operand.  Partials are laid out by 32-column block, ntiles * 4
// blocks per row split (ntiles = ceil(n / 128)), as for the other forms.
#include <algorithm>

#include "common.h"
#include "dma.h"
#include "kernels.h"

namespace rpca {

template <int E, int NB>
struct WideCfg {
  static constexpr int TC = 512;                      // tile columns
  static constexpr int RB = TC * E;                   // bytes per tile row
  static constexpr int KR = 32768 / RB;               // rows per stage
  static constexpr int KS = KR / 16;                  // K16 steps per stage
  static constexpr int XF = KS * NB * (E == 4 ? 2 : 1);  // 1 KB operand fragments per stage
  static constexpr int ABYTES = 32768;
  static constexpr int STAGE = ABYTES + XF * 1024;
  static constexpr int S = (160 * 1024) / STAGE > 4 ? 4 : (160 * 1024) / STAGE;
};

template <int E>
__device__ __forceinline__ int wide_swz(int k) { return 2 * E * ((k >> 3) & 1); }

template <int NB, int E>
__global__ void __launch_bounds__(512) atx_wide_kernel(const unsigned char* __restrict__ A,
                                                       int64_t lda, int64_t m, int64_t n,
                                                       const __bf16* __restrict__ Xp,
                                                       float* __restrict__ P, int gtiles,
                                                       int ntiles, int64_t rows_per) {
  using C = WideCfg<E, NB>;
  constexpr int RB = C::RB, KR = C::KR, KS = C::KS, XF = C::XF, S = C::S, STAGE = C::STAGE;
  constexpr int ABYTES = C::ABYTES;
  constexpr int XFW = (XF + 7) / 8;
  constexpr int XSTRIDE = E == 4 ? 1 : 2;  // KB between consecutive fragments in Xp
  static_assert(S >= 2 && S * STAGE <= 160 * 1024 && KR % 16 == 0, "stage shape");
  __shared__ __attribute__((aligned(1024))) char ring[S * STAGE];

  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 5, jl = lane & 31;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int split = t / gtiles, tile = t % gtiles;
  const int64_t col0 = (int64_t)tile * C::TC;
  const int64_t rbeg = (int64_t)split * rows_per;
  const int64_t rend = (rbeg + rows_per < m) ? rbeg + rows_per : m;
  const int64_t nstage = (rend > rbeg) ? ceil_div(rend - rbeg, KR) : 0;
  const char* xg = reinterpret_cast<const char*>(Xp) + (rbeg / 16) * NB * 2 * 1024;
  const int64_t nbytes = n * E;
  const int nxw = XF / 8 + (wave < XF % 8 ? 1 : 0);

  // this lane's four DMA chunks: row of the stage and byte offset in A's row
  int rr[4];
  int64_t cbyte[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int byte = 1024 * (wave + 8 * i) + 16 * lane;
    const int k = byte / RB, pos = (byte % RB) / 16;
    rr[i] = k;
    const int64_t cb = col0 * E + 16 * (pos ^ wide_swz<E>(k));
    cbyte[i] = (cb + 16 <= nbytes) ? cb : 0;  // past n: any valid chunk (columns never stored)
  }
  int issued = 0, done = 0, islot = 0;
  int64_t ist = 0;
  const int per = 4 + nxw;
  auto issue = [&]() {
    char* slot = ring + islot * STAGE;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t row = min(rbeg + ist * KR + rr[i], rend - 1);
      dma16(A + row * lda * E + cbyte[i], slot + (wave + 8 * i) * 1024);
    }
#pragma unroll
    for (int jx = 0; jx < XFW; ++jx) {
      const int f = wave + 8 * jx;
      if (f < XF)
        dma16(xg + ((ist * XF + f) * XSTRIDE) * 1024 + 16 * lane, slot + ABYTES + f * 1024);
    }
    issued += per;
    islot = islot + 1 == S ? 0 : islot + 1;
    ++ist;
  };

  f32x16 acc[2][NB];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][i][r] = 0.f;

#pragma unroll
  for (int u = 0; u < S - 1; ++u)
    if (u < nstage) issue();
  int cslot = 0;
  for (int64_t q = 0; q < nstage; ++q) {
    // stage q's copies are complete when at most the copies issued after it
    // are outstanding; the barrier publishes them and frees the slot of
    // stage q - 1 for the copy of stage q + S - 1
    wait_vm_barrier_n(issued - done - per);
    done += per;
    if (q + S - 1 < nstage) issue();
    const char* As = ring + cslot * STAGE;
    const char* Xs = As + ABYTES;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      bf16x8 xh[NB], xl[NB];
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        if (E == 4) {
          xh[cb] = *reinterpret_cast<const bf16x8*>(Xs + ((s * NB + cb) * 2) * 1024 + 16 * lane);
          xl[cb] = *reinterpret_cast<const bf16x8*>(Xs + ((s * NB + cb) * 2 + 1) * 1024 + 16 * lane);
        } else {
          xh[cb] = *reinterpret_cast<const bf16x8*>(Xs + (s * NB + cb) * 1024 + 16 * lane);
        }
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int cbt = (64 * wave + 32 * b + jl) * E;  // byte of the column in a tile row
        const int chunk = cbt / 16, off = cbt % 16;
        bf16x8 bop, bopl;
        if (E == 4) {
          float v[8];
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) {
            const int k = 16 * s + 8 * g + jj;
            v[jj] = *reinterpret_cast<const float*>(As + k * RB + 16 * (chunk ^ wide_swz<E>(k)) + off);
          }
          split_bf16x8(make_float4(v[0], v[1], v[2], v[3]), make_float4(v[4], v[5], v[6], v[7]),
                       bop, bopl);
        } else if (E == 2) {
          unsigned short h[8];
#pragma unroll
          for (int jj = 0; jj < 8; ++jj) {
            const int k = 16 * s + 8 * g + jj;
            h[jj] = *reinterpret_cast<const unsigned short*>(As + k * RB + 16 * (chunk ^ wide_swz<E>(k)) + off);
          }
          bop = __builtin_bit_cast(bf16x8, h);
        } else {
          unsigned w[2];
#pragma unroll
          for (int qq = 0; qq < 2; ++qq) {
            unsigned v = 0;
#pragma unroll
            for (int jj = 0; jj < 4; ++jj) {
              const int k = 16 * s + 8 * g + 4 * qq + jj;
              const unsigned byte = *reinterpret_cast<const unsigned char*>(
                  As + k * RB + 16 * (chunk ^ wide_swz<E>(k)) + off);
              v |= byte << (8 * jj);
            }
            w[qq] = v;
          }
          bop = fp8x8_to_bf16(w[0], w[1]);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          if (E == 4) acc[b][cb] = mfma3(xh[cb], xl[cb], bop, bopl, acc[b][cb]);
          else acc[b][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh[cb], bop, acc[b][cb], 0, 0, 0);
        }
      }
    }
    cslot = cslot + 1 == S ? 0 : cslot + 1;
  }
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    const int blk32 = tile * 16 + wave * 2 + b;  // 32-column block of this wave
    if (blk32 >= ntiles * 4) continue;            // columns past the partial layout (beyond n)
    float* out = P + ((int64_t)split * ntiles * 4 + blk32) * NB * 1024;
#pragma unroll
    for (int cb = 0; cb < NB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) out[(cb * 16 + r) * 64 + lane] = acc[b][cb][r];
  }
}

int atx_wide_rows_per_stage(int dtype) {
  return dtype == 2 ? WideCfg<1, 4>::KR : dtype == 1 ? WideCfg<2, 4>::KR : WideCfg<4, 4>::KR;
}

void launch_atx_wide(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                     const __bf16* Xp, float* P, const AtxPlan& plan, int nb) {
  const unsigned char* a = static_cast<const unsigned char*>(A);
  const dim3 grid((unsigned)(plan.gtiles * plan.nsplit));
#define RPCA_WIDE(E_)                                                                              \
  switch (nb) {                                                                                    \
    case 1: hipLaunchKernelGGL((atx_wide_kernel<1, E_>), grid, dim3(512), 0, st, a, lda, m, n, Xp, P, plan.gtiles, plan.ntiles, plan.rows_per); break; \
    case 2: hipLaunchKernelGGL((atx_wide_kernel<2, E_>), grid, dim3(512), 0, st, a, lda, m, n, Xp, P, plan.gtiles, plan.ntiles, plan.rows_per); break; \
    case 4: hipLaunchKernelGGL((atx_wide_kernel<4, E_>), grid, dim3(512), 0, st, a, lda, m, n, Xp, P, plan.gtiles, plan.ntiles, plan.rows_per); break; \
    default: break;                                                                                \
  }
  if (dtype == 2) { RPCA_WIDE(1) }
  else if (dtype == 1) { RPCA_WIDE(2) }
  else { RPCA_WIDE(4) }
#undef RPCA_WIDE
}

}  // namespace rpca
