// Y = A X, tall form, for the three copies of A the passes read: float32
// (products as three bfloat16 terms of the split operands), bfloat16 and
// E4M3 (one term on the operand's high part; the E4M3 column scales are
// folded into the rows of the packed X).  Section 2 prices the method by its
// passes over A, so this kernel only has to keep HBM busy; what it changes
// against the 32-rows-per-wave kernels of gemm.hip and gemm_lp.hip is the
// share of LDS that holds A:
//
//  * 8 waves own two 32-row blocks each (tiles of up to 512 rows), and a
//    stage is a 64-byte segment of every row (16 float32, 32 bfloat16 or 64
//    E4M3 columns).  The X fragments of a stage serve all 512 rows, so at
//    lp = 128 a stage is 32 KB of A and 8 KB of X (16 KB for E4M3) and the
//    LDS ring holds four stages (three for E4M3) instead of three of 32 + 16.
//  * A workgroup's row range is cut into tiles of equal height (one tile of
//    391 rows for 100000 rows on 256 CUs, two for 200000 rows), so no CU
//    streams the whole of X for a short last tile.
//  * The stages of all tiles form one stream: the first stages of the next
//    tile are in flight while a tile's Y is stored, and Y goes out with
//    non-temporal stores (it is read once, by the next kernel).
//
// The K16 steps are accumulated in the same order as in the other kernels,
// so all forms give the same Y bit for bit.
//
// LDS: row R of a stage occupies 64 bytes at 64 R; its 16-byte chunk c sits
// at position c ^ ((R >> 2) & 3), which keeps the MFMA operand reads of 16
// consecutive rows on distinct banks.  A 1 KB DMA block holds 16 rows; block
// q is issued by wave q % 8, X fragment f by wave f % 8, so the number of
// copies a wave issues per stage depends on the tile height and the wave,
// and the wait before a stage counts this wave's copies issued after it.
// The one barrier of a stage both publishes its copies and frees the slot of
// the stage before, which then takes the copy S - 1 stages ahead.
//
// What bounds it: copies alone stream at 5.5-5.7 TB/s, and the products
// (LDS reads, the bfloat16 split of A, MFMAs at about 20 ns each per SIMD
// under load) take 70% of that time for float32 at lp = 64, more than all of
// it for float32 at lp = 128 and E4M3; the two overlap only in part.
#include <algorithm>

#include "common.h"
#include "dma.h"
#include "kernels.h"

namespace rpca {

template <int E, int NB>
struct TallCfg {
  static constexpr int KC = 64 / E;                            // A columns per stage
  static constexpr int KS = KC / 16;                           // K16 steps per stage
  static constexpr int XF = KS * NB * (E == 4 ? 2 : 1);        // 1 KB X fragments per stage
  static constexpr int ABYTES = 512 * 64;
  static constexpr int STAGE = ABYTES + XF * 1024;
  static constexpr int S = (160 * 1024) / STAGE > 4 ? 4 : (160 * 1024) / STAGE;
};

// live 16-row DMA blocks of wave w in a tile of height hg (blocks w, w + 8,
// w + 16, w + 24: a prefix)
__device__ __forceinline__ int tall_blocks(int wave, int64_t hg) {
  int na = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i)
    if (16 * (wave + 8 * i) < hg) na = i + 1;
  return na;
}

template <int NB, int E>
__global__ void __launch_bounds__(512) ax_tall_kernel(const unsigned char* __restrict__ A,
                                                      int64_t lda, int64_t m, int64_t n,
                                                      const __bf16* __restrict__ Xp,
                                                      float* __restrict__ Y, int64_t ldy,
                                                      int64_t rows_per_wg) {
  using C = TallCfg<E, NB>;
  constexpr int KC = C::KC, KS = C::KS, XF = C::XF, S = C::S, STAGE = C::STAGE;
  constexpr int ABYTES = C::ABYTES;
  constexpr int XFW = (XF + 7) / 8;          // X fragments per wave per stage, at most
  constexpr int XSTRIDE = E == 4 ? 1 : 2;    // KB between consecutive fragments in Xp
  static_assert(S >= 2 && S * STAGE <= 160 * 1024, "LDS ring");
  __shared__ __attribute__((aligned(1024))) char ring[S * STAGE];

  // the wave index is uniform: scalar, so every per-wave choice below (live
  // blocks, copy counts, the wait) is a scalar branch, not an exec mask
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int g = lane >> 5;
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t rend = min(m, rbeg + rows_per_wg);
  if (rbeg >= rend) return;  // whole workgroup
  const int64_t rows = rend - rbeg;
  const int ntile = (int)ceil_div(rows, 512);
  const int64_t h = ceil_div(rows, ntile);  // tile height, at most 512
  const int64_t nstage = ceil_div(n, KC);
  const int64_t total = (int64_t)ntile * nstage;
  const int64_t nbytes = n * E;
  const char* xg = reinterpret_cast<const char*>(Xp);
  const int nxw = XF / 8 + (wave < XF % 8 ? 1 : 0);  // X fragments this wave issues
  // byte offset of this lane's chunk in its row segment: LDS position lane & 3
  // of row 16 q + lane / 4 holds chunk (lane & 3) ^ ((lane >> 4) & 3)
  const int coff = 16 * ((lane & 3) ^ ((lane >> 4) & 3));

  // ---- issue side: the next stage to copy is stage ist of tile itile
  int itile = 0, islot = 0, na = 0;
  int64_t ist = 0;
  const unsigned char* rowp[4];
  auto issue_tile = [&](int t) {
    const int64_t r0 = rbeg + (int64_t)t * h;
    na = tall_blocks(wave, min(h, rend - r0));
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int64_t r = min(r0 + 16 * (wave + 8 * i) + (lane >> 2), rend - 1);
      rowp[i] = A + r * lda * E;
    }
  };
  int issued = 0;  // copies this wave has issued (all stages so far)
  auto issue = [&]() {
    char* slot = ring + islot * STAGE;
    const int64_t cb = ist * 64 + coff;
    const int64_t cofs = cb < nbytes ? cb : 0;  // past n: any valid chunk (times zero X)
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (i < na) dma16(rowp[i] + cofs, slot + (wave + 8 * i) * 1024);
#pragma unroll
    for (int j = 0; j < XFW; ++j) {
      const int f = wave + 8 * j;
      if (f < XF)
        dma16(xg + ((ist * XF + f) * XSTRIDE) * 1024 + 16 * lane, slot + ABYTES + f * 1024);
    }
    issued += na + nxw;
    islot = islot + 1 == S ? 0 : islot + 1;
    if (++ist == nstage) {
      ist = 0;
      if (++itile < ntile) issue_tile(itile);
    }
  };

  // ---- compute side: stage cst of tile ctile
  int ctile = 0, cslot = 0;
  int64_t cst = 0;
  int64_t crow0 = rbeg, chg = min(h, rows);
  int cper = tall_blocks(wave, chg) + nxw;  // copies per stage of this wave in the tile
  int done = 0;                             // copies of the stages consumed so far

  f32x16 acc[2][NB];
#pragma unroll
  for (int b = 0; b < 2; ++b)
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[b][i][r] = 0.f;

  issue_tile(0);
#pragma unroll
  for (int t = 0; t < S - 1; ++t)
    if (t < total) issue();

  for (int64_t q = 0; q < total; ++q) {
    // this stage's copies are complete when at most the copies issued after
    // it are outstanding (copies complete in issue order); the barrier then
    // makes every wave's copies visible, and every wave is past the products
    // of stage q - 1 (whose LDS reads fed its MFMAs), so its slot takes the
    // copy of stage q + S - 1: one barrier per stage
    wait_vm_barrier_n(issued - done - cper);
    done += cper;
    if (q + S - 1 < total) issue();
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
        const int j = wave + 8 * b;  // 32-row block
        if (32 * j >= chg) continue;
        const int R = 32 * j + (lane & 31);
        const char* rowl = As + R * 64;
        const int sw = (R >> 2) & 3;
        if (E == 4) {
          const float4 a0 = *reinterpret_cast<const float4*>(rowl + 16 * ((2 * g) ^ sw));
          const float4 a1 = *reinterpret_cast<const float4*>(rowl + 16 * ((2 * g + 1) ^ sw));
          bf16x8 ah, al;
          split_bf16x8(a0, a1, ah, al);
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) acc[b][cb] = mfma3(ah, al, xh[cb], xl[cb], acc[b][cb]);
        } else {
          bf16x8 a;
          if (E == 2) {
            a = *reinterpret_cast<const bf16x8*>(rowl + 16 * ((2 * s + g) ^ sw));
          } else {
            const uint2 w = *reinterpret_cast<const uint2*>(rowl + 16 * (s ^ sw) + 8 * g);
            a = fp8x8_to_bf16(w.x, w.y);
          }
#pragma unroll
          for (int cb = 0; cb < NB; ++cb)
            acc[b][cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xh[cb], acc[b][cb], 0, 0, 0);
        }
      }
    }
    cslot = cslot + 1 == S ? 0 : cslot + 1;
    if (++cst == nstage) {
      // tile done: its Y (the next tile's first stages are already in flight)
      const int64_t cend = crow0 + chg;
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int j = wave + 8 * b;
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          const int col = 32 * cb + (lane & 31);
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            const int64_t row = crow0 + 32 * j + (r & 3) + 4 * g + 8 * (r >> 2);
            if (row < cend) __builtin_nontemporal_store(acc[b][cb][r], Y + row * ldy + col);
            acc[b][cb][r] = 0.f;
          }
        }
      }
      cst = 0;
      ++ctile;
      crow0 = rbeg + (int64_t)ctile * h;
      chg = min(h, rend - crow0);
      cper = tall_blocks(wave, chg) + nxw;
    }
  }
}

template <int NB, int E>
static void ax_tall_go(hipStream_t st, const unsigned char* A, int64_t lda, int64_t m, int64_t n,
                       const __bf16* Xp, float* Y, int64_t ldy, int num_cus) {
  // one workgroup per CU (the ring fills the LDS), row ranges as equal as
  // possible
  int64_t G = std::min<int64_t>(num_cus, ceil_div(m, 32));
  const int64_t rows_per = ceil_div(m, G);
  G = ceil_div(m, rows_per);
  hipLaunchKernelGGL((ax_tall_kernel<NB, E>), dim3((unsigned)G), dim3(512), 0, st, A, lda, m, n,
                     Xp, Y, ldy, rows_per);
}

bool ax_tall_ok(int64_t m, int num_cus) { return m >= (int64_t)num_cus * 256; }

void launch_ax_tall(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                    const __bf16* Xp, float* Y, int64_t ldy, int nb, int num_cus) {
  const unsigned char* a = static_cast<const unsigned char*>(A);
  const int e = dtype == 0 ? 4 : dtype == 1 ? 2 : 1;
#define RPCA_TALL(E_)                                                          \
  switch (nb) {                                                                \
    case 1: ax_tall_go<1, E_>(st, a, lda, m, n, Xp, Y, ldy, num_cus); break;   \
    case 2: ax_tall_go<2, E_>(st, a, lda, m, n, Xp, Y, ldy, num_cus); break;   \
    case 4: ax_tall_go<4, E_>(st, a, lda, m, n, Xp, Y, ldy, num_cus); break;   \
    default: break;                                                            \
  }
  if (e == 4) { RPCA_TALL(4) }
  else if (e == 2) { RPCA_TALL(2) }
  else { RPCA_TALL(1) }
#undef RPCA_TALL
}

}  // namespace rpca
