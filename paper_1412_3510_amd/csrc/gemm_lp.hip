// Passes over a low-precision copy of A: Y = A X and the partials of A^T X
// for A stored in bfloat16 (E = 2 bytes) or in OCP float8 E4M3 with a float32
// scale per column (E = 1 byte; A = A8 diag(s), the scales are applied to the
// packed X of A X and to the rows of A^T X, so the kernels see A8 only).
//
// The paper's cost model is the number of passes over A (Section 2) and the
// speed of each pass; a copy of A in half or a quarter of the bytes makes the
// passes of the range finder (all but the Rayleigh-Ritz product, which reads
// the float32 A) proportionally cheaper.  The range finder only needs
// span(Q) close to the dominant subspace, so the rounding of A to 2^-8
// (bfloat16) or 2^-4 (E4M3) relative acts as a perturbation of A far below
// sigma_{k+1} for the workloads here; X enters as its bfloat16 high part
// (one MFMA per K16 step), whose rounding is of the same order as A's.
//
// Same structure as the float32 kernels (gemm.hip): A streamed once through an
// LDS ring filled by global_load_lds_dwordx4 (128-byte row segments, 16-byte
// chunks XOR-swizzled), packed X fragments streamed beside it, products on
// v_mfma_f32_32x32x16_bf16 with float32 accumulation.  E4M3 bytes are widened
// to bfloat16 exactly, two at a time (v_cvt_scalef32_pk_bf16_fp8, scale 1).
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "dma.h"
#include "kernels.h"

namespace rpca {

template <int E>
struct LpCfg {
  static constexpr int ROWB = 128;           // bytes per A row segment in the ax stage
  static constexpr int KC = ROWB / E;        // A columns per ax stage
  static constexpr int KS = KC / 16;         // K16 steps per stage (both kernels)
  static constexpr int RS = 16384 / (128 * E);  // A rows per atx stage (128 columns)
  static constexpr int ABYTES = 16384;
};

// stage bytes: A (4 NW KB: 32 NW rows of 128 bytes in the ax kernel, RS rows
// of 128 columns in the atx kernel, NW = 4) plus the KS x NB X fragments
template <int NB, int E, int NW = 4>
constexpr int lp_stage_bytes() {
  return NW * 4096 + LpCfg<E>::KS * NB * 1024;
}

// ---------------- Y = A X --------------------------------------------------
// NW waves on a 32 NW-row tile.  Stage: KC columns of the tile (rows 8b..8b+7
// per 1 KB DMA block b; the 16-byte chunk c of row R sits at position
// c ^ ((R >> 1) & 7)) plus the matching KS x NB high-part X fragments.  The X
// fragments of a stage serve every row of the tile, so the 256-row tile of
// NW = 8 moves half the X bytes per byte of A of the 128-row one.  As in the
// float32 kernel, a wave whose rows are all past the end of a short last
// tile loads only its X fragments and skips its products.
template <int NB, int S, int E, int NW>
__global__ void __launch_bounds__(64 * NW) ax_lp_kernel(const unsigned char* __restrict__ A,
                                                        int64_t lda, int64_t m, int64_t n,
                                                        const __bf16* __restrict__ Xp,
                                                        float* __restrict__ Y, int64_t ldy,
                                                        int64_t rows_per_wg) {
  using C = LpCfg<E>;
  constexpr int KC = C::KC, KS = C::KS;
  constexpr int TR = 32 * NW;       // tile rows
  constexpr int ABYTES = TR * 128;
  constexpr int XFR = KS * NB;  // X fragments per stage
  constexpr int STAGE = lp_stage_bytes<NB, E, NW>();
  constexpr int XPW = XFR / NW;
  constexpr int PER = 4 + XPW;
  static_assert(XPW * NW == XFR && (S - 1) * PER < 64, "stage shape");
  static_assert(S * STAGE <= 160 * 1024, "LDS ring");
  __shared__ __attribute__((aligned(1024))) char ring[S * STAGE];

  // scalar wave index: the per-wave choices (live rows) are scalar branches
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t rend = min(m, rbeg + rows_per_wg);
  const int64_t nstage = ceil_div(n, KC);
  const char* xg = reinterpret_cast<const char*>(Xp);
  const int lrow = lane >> 3;
  const int g = lane >> 5;

  for (int64_t row0 = rbeg; row0 < rend; row0 += TR) {
    const unsigned char* rowp[4];
    int cofs[4];  // element offset of this lane's chunk within the stage
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = 8 * (4 * wave + i) + lrow;
      const int64_t grow = min(row0 + R, rend - 1);
      rowp[i] = A + grow * lda * E;
      cofs[i] = ((lane & 7) ^ ((R >> 1) & 7)) * (16 / E);
    }
    const bool live = row0 + 32 * wave < rend;  // this wave has rows in the tile
#define AXL_ISSUE(STG)                                                                    \
  do {                                                                                    \
    const int64_t stg_ = (STG);                                                           \
    char* slot_ = ring + (int)(stg_ % S) * STAGE;                                         \
    if (live) {                                                                           \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                     \
        const int64_t col_ = stg_ * KC + cofs[i];                                         \
        dma16(rowp[i] + (col_ < n ? col_ : 0) * E, slot_ + (4 * wave + i) * 1024);        \
      }                                                                                   \
    }                                                                                     \
    _Pragma("unroll") for (int i = 0; i < XPW; ++i) {                                     \
      const int blk_ = wave + NW * i;                                                     \
      dma16(xg + ((stg_ * XFR + blk_) * 2) * 1024 + 16 * lane, slot_ + ABYTES + blk_ * 1024); \
    }                                                                                     \
  } while (0)

    f32x16 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

#pragma unroll
    for (int t = 0; t < S - 1; ++t)
      if (t < nstage) AXL_ISSUE(t);
    const int R = 32 * wave + (lane & 31);
    const int sw = (R >> 1) & 7;
    for (int64_t stg = 0; stg < nstage; ++stg) {
      if (stg + S - 1 < nstage) AXL_ISSUE(stg + S - 1);
      const int64_t last = min(nstage - 1, stg + S - 1);
      // (both waits end in the workgroup barrier; a wave without rows
      // still takes every barrier of the stage)
      if (live) wait_ahead<PER, S>((int)(last - stg));
      else wait_ahead<XPW, S>((int)(last - stg));
      const char* As = ring + (int)(stg % S) * STAGE;
      const char* Xs = As + ABYTES;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        if (!live) break;
        bf16x8 a;
        if (E == 2) {
          a = *reinterpret_cast<const bf16x8*>(As + R * 128 + 16 * ((2 * s + g) ^ sw));
        } else {
          const uint2 w = *reinterpret_cast<const uint2*>(As + R * 128 + 16 * (s ^ sw) + 8 * g);
          a = fp8x8_to_bf16(w.x, w.y);
        }
#pragma unroll
        for (int cb = 0; cb < NB; ++cb) {
          const bf16x8 xh = *reinterpret_cast<const bf16x8*>(Xs + (s * NB + cb) * 1024 + 16 * lane);
          acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xh, acc[cb], 0, 0, 0);
        }
      }
      barrier_mem();
    }
#pragma unroll
    for (int cb = 0; cb < NB; ++cb) {
      const int col = 32 * cb + (lane & 31);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int64_t row = row0 + 32 * wave + (r & 3) + 4 * g + 8 * (r >> 2);
        if (row < rend) Y[row * ldy + col] = acc[cb][r];
      }
    }
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");  // no stores in flight under the next ring
  }
#undef AXL_ISSUE
}

// ---------------- partials of A^T X -----------------------------------------
// NW waves on a 32 NW-column tile (wave w: columns 32w..32w+31 of it).
// Stage: RS rows of the tile (4 NW KB; DMA block b holds rows RB b ..
// RB b + RB - 1, LPR lanes of 16 bytes per row; chunk c of row r sits at
// c ^ (LPR/2 ((r >> 3) & 1))) plus the matching KS x NB fragments of the
// packed m-side operand, which serve every column of the tile: the 256-column
// tile of NW = 8 moves half their bytes per byte of A.  The workgroup index
// gives (split, tile) over gtiles tiles per split; partials are laid out by
// 32-column block, ntiles * 4 blocks per split (ntiles = ceil(n / 128)).
template <int NB, int S, int E, int NW>
__global__ void __launch_bounds__(64 * NW) atx_lp_kernel(const unsigned char* __restrict__ A,
                                                         int64_t lda, int64_t m, int64_t n,
                                                         const __bf16* __restrict__ Xp,
                                                         float* __restrict__ P, int gtiles,
                                                         int ntiles, int64_t rows_per) {
  using C = LpCfg<E>;
  constexpr int RS = C::RS, KS = C::KS;
  constexpr int TC = 32 * NW;          // tile columns
  constexpr int ABYTES = NW * 4096;
  constexpr int ROWB = TC * E;         // bytes per row of the tile
  constexpr int LPR = ROWB / 16;       // lanes per row in a DMA block
  constexpr int RB = 64 / LPR;         // rows per DMA block
  constexpr int SWZ = LPR / 2;
  constexpr int XFR = KS * NB;
  constexpr int STAGE = lp_stage_bytes<NB, E, NW>();
  constexpr int XPW = XFR / NW;
  constexpr int PER = 4 + XPW;
  static_assert(RB * 4 * NW == RS && XPW * NW == XFR && (S - 1) * PER < 64, "stage shape");
  static_assert(S * STAGE <= 160 * 1024, "LDS ring");
  __shared__ __attribute__((aligned(1024))) char ring[S * STAGE];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int split = t / gtiles, tile = t % gtiles;
  const int64_t col0 = (int64_t)tile * TC;
  const int64_t rbeg = (int64_t)split * rows_per;
  const int64_t rend = (rbeg + rows_per < m) ? rbeg + rows_per : m;
  const int64_t nstage = (rend > rbeg) ? ceil_div(rend - rbeg, RS) : 0;
  const char* xg = reinterpret_cast<const char*>(Xp) + (rbeg / 16) * NB * 2 * 1024;

  int64_t colc[4];
  int rr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = 4 * wave + i;
    rr[i] = RB * b + lane / LPR;
    const int chunk = (lane % LPR) ^ (SWZ * ((rr[i] >> 3) & 1));
    const int64_t c = col0 + chunk * (16 / E);
    colc[i] = (c + 16 / E <= n) ? c : 0;
  }
#define ATXL_ISSUE(STG)                                                                   \
  do {                                                                                    \
    const int64_t stg_ = (STG);                                                           \
    char* slot_ = ring + (int)(stg_ % S) * STAGE;                                         \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                       \
      const int64_t grow_ = min(rbeg + stg_ * RS + rr[i], rend - 1);                      \
      dma16(A + (grow_ * lda + colc[i]) * E, slot_ + (4 * wave + i) * 1024);              \
    }                                                                                     \
    _Pragma("unroll") for (int i = 0; i < XPW; ++i) {                                     \
      const int blk_ = wave + NW * i;                                                     \
      dma16(xg + ((stg_ * XFR + blk_) * 2) * 1024 + 16 * lane, slot_ + ABYTES + blk_ * 1024); \
    }                                                                                     \
  } while (0)

  f32x16 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

#pragma unroll
  for (int u = 0; u < S - 1; ++u)
    if (u < nstage) ATXL_ISSUE(u);
  const int j = lane & 31, g = lane >> 5;
  // byte of (row 8g + jj of a K16 step, column 32 wave + j) within its row
  const int cbyte = (32 * wave + j) * E;
  const int pos = 16 * ((cbyte / 16) ^ (SWZ * g)) + (cbyte % 16);
  for (int64_t stg = 0; stg < nstage; ++stg) {
    if (stg + S - 1 < nstage) ATXL_ISSUE(stg + S - 1);
    const int64_t last = min(nstage - 1, stg + S - 1);
    wait_ahead<PER, S>((int)(last - stg));
    const char* As = ring + (int)(stg % S) * STAGE;
    const char* Xs = As + ABYTES;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const char* base = As + (16 * s + 8 * g) * ROWB + pos;
      bf16x8 b;
      if (E == 2) {
        unsigned short h[8];
#pragma unroll
        for (int jj = 0; jj < 8; ++jj) h[jj] = *reinterpret_cast<const unsigned short*>(base + jj * ROWB);
        b = __builtin_bit_cast(bf16x8, h);
      } else {
        unsigned w[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
          const unsigned b0 = *reinterpret_cast<const unsigned char*>(base + (4 * q + 0) * ROWB);
          const unsigned b1 = *reinterpret_cast<const unsigned char*>(base + (4 * q + 1) * ROWB);
          const unsigned b2 = *reinterpret_cast<const unsigned char*>(base + (4 * q + 2) * ROWB);
          const unsigned b3 = *reinterpret_cast<const unsigned char*>(base + (4 * q + 3) * ROWB);
          w[q] = b0 | (b1 << 8) | (b2 << 16) | (b3 << 24);
        }
        b = fp8x8_to_bf16(w[0], w[1]);
      }
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const bf16x8 xh = *reinterpret_cast<const bf16x8*>(Xs + (s * NB + cb) * 1024 + 16 * lane);
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xh, b, acc[cb], 0, 0, 0);
      }
    }
    barrier_mem();
  }
  const int blk32 = tile * NW + wave;  // 32-column block of this wave
  if (blk32 >= ntiles * 4) return;      // columns past the partial layout (beyond n)
  float* out = P + ((int64_t)split * ntiles * 4 + blk32) * NB * 1024;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) out[(cb * 16 + r) * 64 + lane] = acc[cb][r];
#undef ATXL_ISSUE
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
static int lp_elem_bytes(int dtype) { return dtype == 2 ? 1 : 2; }

template <int NB, int E, int NW = 4>
constexpr int lp_ring() {
  constexpr int st = lp_stage_bytes<NB, E, NW>();
  constexpr int s = (160 * 1024) / st;
  return s > 6 ? 6 : s;
}

// the 8-wave form of the low-precision A^T X kernel: the X fragments of a
// stage split evenly over 8 waves and the ring still holds three stages
template <int NB, int E>
constexpr bool lp_can8() {
  return (LpCfg<E>::KS * NB) % 8 == 0 && lp_ring<NB, E, 8>() >= 3;
}

bool lp_atx_can8(int nb, int dtype) {
  if (dtype == 2) return nb == 1 ? lp_can8<1, 1>() : nb == 2 ? lp_can8<2, 1>() : lp_can8<4, 1>();
  return nb == 1 ? lp_can8<1, 2>() : nb == 2 ? lp_can8<2, 2>() : lp_can8<4, 2>();
}

int lp_rows_per_stage(int dtype) { return dtype == 2 ? LpCfg<1>::RS : LpCfg<2>::RS; }

bool lp_shape_ok(const void* A, int dtype, int64_t lda, int64_t n) {
  const int per = 16 / lp_elem_bytes(dtype);
  return (lda % per) == 0 && (n % per) == 0 && (reinterpret_cast<uintptr_t>(A) % 16) == 0;
}

// resident workgroups per CU (one: the ring fills the LDS)
int lp_per_cu(int nb, int dtype) {
  int st = 0, s = 0;
  if (dtype == 2) {
    st = nb == 1 ? lp_stage_bytes<1, 1>() : nb == 2 ? lp_stage_bytes<2, 1>() : lp_stage_bytes<4, 1>();
    s = nb == 1 ? lp_ring<1, 1>() : nb == 2 ? lp_ring<2, 1>() : lp_ring<4, 1>();
  } else {
    st = nb == 1 ? lp_stage_bytes<1, 2>() : nb == 2 ? lp_stage_bytes<2, 2>() : lp_stage_bytes<4, 2>();
    s = nb == 1 ? lp_ring<1, 2>() : nb == 2 ? lp_ring<2, 2>() : lp_ring<4, 2>();
  }
  return std::max(1, (160 * 1024) / (s * st));
}

template <int NB, int E, int NW>
static void ax_lp_launch(hipStream_t st, const unsigned char* A, int64_t lda, int64_t m,
                         int64_t n, const __bf16* Xp, float* Y, int64_t ldy, int num_cus) {
  constexpr int S = lp_ring<NB, E, NW>();
  const int per_cu = std::max(1, (160 * 1024) / (S * lp_stage_bytes<NB, E, NW>()));
  int64_t G = (int64_t)num_cus * per_cu;
  G = std::min<int64_t>(G, ceil_div(m, 32));
  const int64_t rows_per = ceil_div(m, G);
  G = ceil_div(m, rows_per);
  hipLaunchKernelGGL((ax_lp_kernel<NB, S, E, NW>), dim3((unsigned)G), dim3(64 * NW), 0, st, A,
                     lda, m, n, Xp, Y, ldy, rows_per);
}

// the tall form (ax_tall.hip) where every CU gets 256 rows or more, else
// 4 waves on 128-row tiles (either one when the configuration names it)
template <int NB, int E>
static void ax_lp_go(hipStream_t st, const unsigned char* A, int64_t lda, int64_t m, int64_t n,
                     const __bf16* Xp, float* Y, int64_t ldy, int num_cus, const TuneCfg* cfg) {
  bool tall = ax_tall_ok(m, num_cus);
  if (cfg && cfg->ax_waves == 16) tall = true;
  if (cfg && cfg->ax_waves == 4) tall = false;
  if (tall) {
    launch_ax_tall(st, A, E == 2 ? 1 : 2, lda, m, n, Xp, Y, ldy, NB, num_cus);
    return;
  }
  ax_lp_launch<NB, E, 4>(st, A, lda, m, n, Xp, Y, ldy, num_cus);
}

void launch_ax_lp(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                  const __bf16* Xp, float* Y, int64_t ldy, int nb, int num_cus,
                  const TuneCfg* cfg) {
  const unsigned char* a = static_cast<const unsigned char*>(A);
  if (dtype == 2) {
    switch (nb) {
      case 1: ax_lp_go<1, 1>(st, a, lda, m, n, Xp, Y, ldy, num_cus, cfg); break;
      case 2: ax_lp_go<2, 1>(st, a, lda, m, n, Xp, Y, ldy, num_cus, cfg); break;
      case 4: ax_lp_go<4, 1>(st, a, lda, m, n, Xp, Y, ldy, num_cus, cfg); break;
      default: break;
    }
  } else {
    switch (nb) {
      case 1: ax_lp_go<1, 2>(st, a, lda, m, n, Xp, Y, ldy, num_cus, cfg); break;
      case 2: ax_lp_go<2, 2>(st, a, lda, m, n, Xp, Y, ldy, num_cus, cfg); break;
      case 4: ax_lp_go<4, 2>(st, a, lda, m, n, Xp, Y, ldy, num_cus, cfg); break;
      default: break;
    }
  }
}

template <int NB, int E>
static void atx_lp_go(hipStream_t st, const unsigned char* A, int64_t lda, int64_t m, int64_t n,
                      const __bf16* Xp, float* P, const AtxPlan& plan) {
  if constexpr (lp_can8<NB, E>()) {
    if (plan.waves == 8) {
      constexpr int S = lp_ring<NB, E, 8>();
      hipLaunchKernelGGL((atx_lp_kernel<NB, S, E, 8>), dim3((unsigned)(plan.gtiles * plan.nsplit)),
                         dim3(512), 0, st, A, lda, m, n, Xp, P, plan.gtiles, plan.ntiles,
                         plan.rows_per);
      return;
    }
  }
  constexpr int S = lp_ring<NB, E>();
  const dim3 grid((unsigned)(plan.ntiles * plan.nsplit));
  hipLaunchKernelGGL((atx_lp_kernel<NB, S, E, 4>), grid, dim3(256), 0, st, A, lda, m, n, Xp, P,
                     plan.ntiles, plan.ntiles, plan.rows_per);
}

void launch_atx_lp(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                   const __bf16* Xp, float* P, const AtxPlan& plan, int nb) {
  if (plan.waves == 16) {
    launch_atx_wide(st, A, dtype, lda, m, n, Xp, P, plan, nb);
    return;
  }
  const unsigned char* a = static_cast<const unsigned char*>(A);
  if (dtype == 2) {
    switch (nb) {
      case 1: atx_lp_go<1, 1>(st, a, lda, m, n, Xp, P, plan); break;
      case 2: atx_lp_go<2, 1>(st, a, lda, m, n, Xp, P, plan); break;
      case 4: atx_lp_go<4, 1>(st, a, lda, m, n, Xp, P, plan); break;
      default: break;
    }
  } else {
    switch (nb) {
      case 1: atx_lp_go<1, 2>(st, a, lda, m, n, Xp, P, plan); break;
      case 2: atx_lp_go<2, 2>(st, a, lda, m, n, Xp, P, plan); break;
      case 4: atx_lp_go<4, 2>(st, a, lda, m, n, Xp, P, plan); break;
      default: break;
    }
  }
}

// ---------------------------------------------------------------------------
// Precision preparation (once per matrix): A -> bfloat16 (round to nearest
// even), or A -> E4M3 with s_j = max_i |a_ij| / 448 (s_j = 1 for a zero
// column) and a8_ij = E4M3(a_ij / s_j), rounded to nearest even.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) to_bf16_kernel(const float* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      __bf16* __restrict__ out, int64_t ldo) {
  const int64_t total = m * n, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / n, j = e - i * n;
    out[i * ldo + j] = static_cast<__bf16>(A[i * lda + j]);
  }
}

// column max |a| over row chunks of ``chunk`` rows: part[c][j]
__global__ void __launch_bounds__(256) colabs_partial_kernel(const float* __restrict__ A,
                                                             int64_t lda, int64_t m, int64_t n,
                                                             int64_t chunk,
                                                             float* __restrict__ part) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const int64_t r0 = (int64_t)blockIdx.y * chunk, r1 = min(m, r0 + chunk);
  float v = 0.f;
  for (int64_t i = r0; i < r1; ++i) v = fmaxf(v, fabsf(A[i * lda + j]));
  part[(int64_t)blockIdx.y * n + j] = v;
}

__global__ void __launch_bounds__(256) colscale_kernel(const float* __restrict__ part, int nchunk,
                                                       int64_t n, float* __restrict__ scale) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  float v = 0.f;
  for (int c = 0; c < nchunk; ++c) v = fmaxf(v, part[(int64_t)c * n + j]);
  scale[j] = (v > 0.f) ? v / 448.0f : 1.0f;
}

// float -> E4M3 (OCP: bias 7, no infinities, max 448), round to nearest even,
// saturating at 448.
__device__ __forceinline__ unsigned char e4m3_encode(float x) {
  const unsigned sign = (__float_as_uint(x) >> 24) & 0x80u;
  float a = fabsf(x);
  if (!(a < 448.0f)) return (unsigned char)(sign | 0x7Eu);  // 448 (and NaN input -> 448)
  if (a < 0.015625f) {  // below 2^-6: subnormal steps of 2^-9
    const unsigned q = (unsigned)rintf(a * 512.0f);  // 0 .. 8; 8 is the smallest normal
    return (unsigned char)(sign | q);
  }
  int e;
  const float f = frexpf(a, &e);  // a = f 2^e, f in [0.5, 1)
  // a = (1 + m/8) 2^(e-1)
  unsigned mq = (unsigned)rintf((2.0f * f - 1.0f) * 8.0f);
  int ee = e - 1;
  if (mq == 8u) {
    mq = 0u;
    ++ee;
  }
  unsigned code = ((unsigned)(ee + 7) << 3) | mq;
  if (code > 0x7Eu) code = 0x7Eu;
  return (unsigned char)(sign | code);
}

__global__ void __launch_bounds__(256) to_e4m3_kernel(const float* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      const float* __restrict__ scale,
                                                      unsigned char* __restrict__ out,
                                                      int64_t ldo) {
  const int64_t total = m * n, stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
    const int64_t i = e / n, j = e - i * n;
    out[i * ldo + j] = e4m3_encode(A[i * lda + j] / scale[j]);
  }
}

// rows per column-max chunk: 256, more when the chunk count would pass the
// grid's y limit
static int64_t quant_chunk(int64_t m) { return 256 * ceil_div(ceil_div(m, 256), 65535); }

size_t quantize_work_bytes(int64_t m, int64_t n) {
  return (size_t)ceil_div(m, quant_chunk(m)) * (size_t)n * sizeof(float);
}

void launch_quantize(hipStream_t st, const float* A, int64_t lda, int64_t m, int64_t n, int dtype,
                     void* out, int64_t ldo, float* scale, float* work) {
  // grid-stride element kernels: at most 2^20 workgroups whatever m n is
  const int64_t gb = ceil_div(m * n, 256);
  const unsigned g = (unsigned)(gb < ((int64_t)1 << 20) ? gb : ((int64_t)1 << 20));
  if (dtype == 1) {
    hipLaunchKernelGGL(to_bf16_kernel, dim3(g), dim3(256), 0, st, A, lda, m, n,
                       static_cast<__bf16*>(out), ldo);
    return;
  }
  const unsigned gc = (unsigned)ceil_div(n, 256);
  const int64_t chunk = quant_chunk(m);
  const unsigned nchunk = (unsigned)ceil_div(m, chunk);
  hipLaunchKernelGGL(colabs_partial_kernel, dim3(gc, nchunk), dim3(256), 0, st, A, lda, m, n, chunk,
                     work);
  hipLaunchKernelGGL(colscale_kernel, dim3(gc), dim3(256), 0, st, work, (int)nchunk, n, scale);
  hipLaunchKernelGGL(to_e4m3_kernel, dim3(g), dim3(256), 0, st, A, lda, m, n, scale,
                     static_cast<unsigned char*>(out), ldo);
}

}  // namespace rpca
