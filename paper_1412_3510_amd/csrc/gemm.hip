// Passes over A: Y = A X and Z = A^T X with X tall and skinny (l <= 128).
//
// These are the products the paper identifies as the cost of the method
// (Section 2: A has far more entries than any other matrix; Section 5: A* is
// applied as (Q* A)* so that A is streamed in its own storage order).  Each
// pass streams A once from HBM in coalesced 128/512-byte row segments and
// feeds MFMA tiles through LDS.
//
// Arithmetic: float32 A and X are split into bfloat16 pairs (hi, lo) and
// multiplied as hi*hi' + hi*lo' + lo*hi' with float32 accumulation on
// v_mfma_f32_32x32x16_bf16; the dropped lo*lo' term and the split residuals
// are below 2^-16 relative per product.  The split keeps the pass bound by
// HBM bandwidth: three bf16 MFMAs cost less than one float32 FMA stream at
// the arithmetic intensity of l = 60..120 columns.
//
// Fragment order (the layout of LDS tiles and of packed X): for a K16 step s
// (16 consecutive K indices) and a 32-wide column block cb, a fragment is 64
// lanes x 8 bf16 = 1 KB in which lane L = c + 32 g holds the K indices
// 16 s + 8 g + j (j = 0..7) of column c.  This is the operand layout of
// v_mfma_f32_32x32x16_bf16 for both the A and the B operand; the
// accumulator of lane L, register r, is (row (r%4) + 4 g + 8 (r/4), col c).
#include <algorithm>
#include <cstdlib>

#include "common.h"
#include "dma.h"
#include "kernels.h"

namespace rpca {

// ------------------------------------------------------------------------
// pack: tall float32 X (rows x cols, ld ldx) -> fragment-ordered bf16 (hi, lo)
// ------------------------------------------------------------------------
__global__ void __launch_bounds__(256) pack_kernel(const float* __restrict__ X, int64_t ldx,
                                                   int64_t rows, int cols, int nb,
                                                   const float* __restrict__ mu,
                                                   const float* __restrict__ rscale,
                                                   __bf16* __restrict__ out, int64_t nsteps) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t total = nsteps * nb * RPCA_WAVE;
  if (t >= total) return;
  const int L = (int)(t % RPCA_WAVE);
  const int64_t rest = t / RPCA_WAVE;
  const int cb = (int)(rest % nb);
  const int64_t s = rest / nb;
  const int c = 32 * cb + (L & 31);
  const int g = L >> 5;
  bf16x8 hi, lo;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const int64_t r = 16 * s + 8 * g + j;
    float v = 0.f;
    if (r < rows && c < cols) {
      v = X[r * ldx + c];
      if (mu) v -= mu[c];
      if (rscale) v *= rscale[r];
    }
    __bf16 h, lw;
    split_bf16(v, h, lw);
    hi[j] = h;
    lo[j] = lw;
  }
  const int64_t base = ((s * nb + cb) * 2) * kFragElems + (int64_t)L * 8;
  *reinterpret_cast<bf16x8*>(out + base) = hi;
  *reinterpret_cast<bf16x8*>(out + base + kFragElems) = lo;
}

size_t packed_bytes(int64_t nsteps, int nb) { return (size_t)nsteps * nb * 2 * 1024; }

void launch_pack(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int cols, int nb,
                 const float* mu, const float* rscale, __bf16* out, int64_t nsteps) {
  const int64_t total = nsteps * nb * RPCA_WAVE;
  if (total == 0) return;
  hipLaunchKernelGGL(pack_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0, st, X, ldx,
                     rows, cols, nb, mu, rscale, out, nsteps);
}

// ------------------------------------------------------------------------
// float32 row loads with bounds
// ------------------------------------------------------------------------
__device__ __forceinline__ float4 load_row4(const float* __restrict__ A, int64_t lda, int64_t r,
                                            int64_t c, int64_t rmax, int64_t n, bool vec) {
  float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
  if (r >= rmax) return v;
  const float* p = A + r * lda + c;
  if (vec && c + 4 <= n) return *reinterpret_cast<const float4*>(p);
  if (c + 0 < n) v.x = p[0];
  if (c + 1 < n) v.y = p[1];
  if (c + 2 < n) v.z = p[2];
  if (c + 3 < n) v.w = p[3];
  return v;
}

// ------------------------------------------------------------------------
// Y = A X.  Workgroup: 4 waves on a 128-row tile, wave w owns rows
// 32w..32w+31 and all 32*NB columns.  K advances 32 columns per stage: each
// thread loads four float4 of A (row (q>>3), columns 4(q&7)..+3 of the stage,
// q = tid + 256 v: every wave instruction reads eight full 128-byte row
// segments) and NB 16-byte words of packed X; the next stage's loads are in
// flight while the current stage is multiplied out of LDS.
// ------------------------------------------------------------------------
template <int NB>
__global__ void __launch_bounds__(256) ax_f32_kernel(const float* __restrict__ A, int64_t lda,
                                                     int64_t m, int64_t n,
                                                     const __bf16* __restrict__ Xp,
                                                     float* __restrict__ Y, int64_t ldy,
                                                     int vec) {
  constexpr int BM = 128;
  constexpr int KC = 32;
  __shared__ __attribute__((aligned(16))) char lds_a[4 * 4 * 1024];   // [rb 4][s 2][part 2]
  __shared__ __attribute__((aligned(16))) char lds_x[NB * 4 * 1024];  // [s 2][cb NB][part 2]

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int64_t row0 = (int64_t)blockIdx.x * BM;
  const int64_t nstage = ceil_div(n, KC);
  const bool rows_in = (row0 + BM <= m) && vec;
  const int64_t nfast = rows_in ? n / KC : 0;  // stages loadable without masks

  const int lr = tid >> 3, lc = 4 * (tid & 7);
  const float* ap = A + (row0 + lr) * lda + lc;
  const int64_t rstride = 32 * lda;
  const uint4* xbase = reinterpret_cast<const uint4*>(Xp);

  float4 ra[4];
  uint4 rx[NB];
#define AX_LOAD(STG)                                                                     \
  do {                                                                                   \
    const int64_t stg_ = (STG);                                                          \
    if (stg_ < nfast) {                                                                  \
      _Pragma("unroll") for (int v = 0; v < 4; ++v) ra[v] =                              \
          *reinterpret_cast<const float4*>(ap + v * rstride + stg_ * KC);               \
    } else {                                                                             \
      _Pragma("unroll") for (int v = 0; v < 4; ++v) ra[v] =                              \
          load_row4(A, lda, row0 + lr + 32 * v, stg_ * KC + lc, m, n, vec != 0);         \
    }                                                                                    \
    _Pragma("unroll") for (int v = 0; v < NB; ++v) rx[v] =                               \
        xbase[stg_ * (NB * 256) + tid + 256 * v];                                        \
  } while (0)

  f32x16 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

  // LDS byte offset of this thread's four (row, 4-column) pieces
  const int c4 = tid & 7;
  const int s_t = c4 >> 2, g_t = (c4 & 3) >> 1, j0 = 4 * (c4 & 1);

  AX_LOAD(0);
  for (int64_t stg = 0; stg < nstage; ++stg) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = lr + 32 * v;
      const int off = ((v * 2 + s_t) * 2) * 1024 + 16 * ((row & 31) + 32 * g_t) + 2 * j0;
      bf16x4 h, lo;
      __bf16 th, tl;
      split_bf16(ra[v].x, th, tl); h[0] = th; lo[0] = tl;
      split_bf16(ra[v].y, th, tl); h[1] = th; lo[1] = tl;
      split_bf16(ra[v].z, th, tl); h[2] = th; lo[2] = tl;
      split_bf16(ra[v].w, th, tl); h[3] = th; lo[3] = tl;
      *reinterpret_cast<bf16x4*>(lds_a + off) = h;
      *reinterpret_cast<bf16x4*>(lds_a + off + 1024) = lo;
    }
#pragma unroll
    for (int v = 0; v < NB; ++v) reinterpret_cast<uint4*>(lds_x)[tid + 256 * v] = rx[v];
    __syncthreads();
    if (stg + 1 < nstage) AX_LOAD(stg + 1);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const bf16x8 ah = *reinterpret_cast<const bf16x8*>(lds_a + ((wave * 2 + s) * 2) * 1024 + 16 * lane);
      const bf16x8 al = *reinterpret_cast<const bf16x8*>(lds_a + ((wave * 2 + s) * 2 + 1) * 1024 + 16 * lane);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const bf16x8 xh = *reinterpret_cast<const bf16x8*>(lds_x + ((s * NB + cb) * 2) * 1024 + 16 * lane);
        const bf16x8 xl = *reinterpret_cast<const bf16x8*>(lds_x + ((s * NB + cb) * 2 + 1) * 1024 + 16 * lane);
        acc[cb] = mfma3(ah, al, xh, xl, acc[cb]);
      }
    }
    __syncthreads();
  }
#undef AX_LOAD
  const int g = lane >> 5;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb) {
    const int col = 32 * cb + (lane & 31);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t row = row0 + 32 * wave + (r & 3) + 4 * g + 8 * (r >> 2);
      if (row < m) Y[row * ldy + col] = acc[cb][r];
    }
  }
}

// ========================================================================
// LDS-DMA variants (row-major A with lda % 4 == 0, 16-byte aligned, n % 4 == 0
// for Y = A X).  A and packed X tiles are copied global -> LDS by
// global_load_lds_dwordx4 into a ring of S stages, so S - 1 stages stay in
// flight while one is multiplied; the float32 -> bf16 split happens on the
// LDS -> register read.  Every lane's source address is clamped to valid
// memory; the entries this brings in for rows or columns outside A are
// multiplied by zero rows of packed X or never stored.
// ========================================================================
// ---------------- Y = A X --------------------------------------------------
// NW waves on a 32 NW-row tile.  Stage: 32 columns of the tile (4 NW KB of A,
// rows 8b..8b+7 per 1 KB DMA block b; the 16-byte chunk c of row R sits at
// position c ^ ((R >> 1) & 7)) plus the matching 4 NB packed X fragments, XW
// per wave.  With NW = 8 one workgroup holds a CU's whole LDS, so a deeper
// ring keeps more bytes of A in flight per CU.  Each wave loads (and reads)
// only its own 32 rows of A, so in a short last tile a wave whose rows are
// all past the end issues only its X fragments (and waits for those alone)
// and skips its products: the tile then costs what its rows cost.
template <int NB, int S, int NW>
__global__ void __launch_bounds__(64 * NW) ax_dma_kernel(const float* __restrict__ A,
                                                         int64_t lda, int64_t m, int64_t n,
                                                         const __bf16* __restrict__ Xp,
                                                         float* __restrict__ Y, int64_t ldy,
                                                         int64_t rows_per_wg) {
  constexpr int KC = 32;
  constexpr int TR = 32 * NW;             // tile rows
  constexpr int ABYTES = TR * 128;
  constexpr int STAGE = ABYTES + NB * 4096;
  constexpr int XW = 4 * NB / NW;         // X fragments per wave per stage
  static_assert(XW * NW == 4 * NB, "X fragments per wave");
  constexpr int PER = 4 + XW;  // DMA instructions per wave per stage
  __shared__ __attribute__((aligned(1024))) char ring[S * STAGE];

  // scalar wave index: the per-wave choices (live rows) are scalar branches
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int64_t rbeg = (int64_t)blockIdx.x * rows_per_wg;
  const int64_t rend = min(m, rbeg + rows_per_wg);
  const int64_t nstage = ceil_div(n, KC);
  const char* xg = reinterpret_cast<const char*>(Xp);

  // this lane's chunk within its DMA row (swizzled), constant over stages
  const int lrow = lane >> 3;  // row within the 8-row block
  const int g = lane >> 5;

  for (int64_t row0 = rbeg; row0 < rend; row0 += TR) {
    const float* rowp[4];
    int cofs[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int R = 8 * (4 * wave + i) + lrow;  // tile row of this lane's DMA
      const int64_t grow = min(row0 + R, rend - 1);
      rowp[i] = A + grow * lda;
      cofs[i] = 4 * ((lane & 7) ^ ((R >> 1) & 7));
    }
    const bool live = row0 + 32 * wave < rend;  // this wave has rows in the tile
#define AX_ISSUE(STG)                                                                     \
  do {                                                                                    \
    const int64_t stg_ = (STG);                                                           \
    char* slot_ = ring + (int)(stg_ % S) * STAGE;                                         \
    if (live) {                                                                           \
      _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                     \
        const int64_t col_ = stg_ * KC + cofs[i];                                         \
        dma16(rowp[i] + (col_ < n ? col_ : 0), slot_ + (4 * wave + i) * 1024);            \
      }                                                                                   \
    }                                                                                     \
    _Pragma("unroll") for (int i = 0; i < XW; ++i) {                                      \
      const int blk_ = wave + NW * i;                                                     \
      dma16(xg + (stg_ * (NB * 4) + blk_) * 1024 + 16 * lane, slot_ + ABYTES + blk_ * 1024); \
    }                                                                                     \
  } while (0)

    f32x16 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

#pragma unroll
    for (int t = 0; t < S - 1; ++t)
      if (t < nstage) AX_ISSUE(t);
    const int R = 32 * wave + (lane & 31);
    const int sw = (R >> 1) & 7;
    for (int64_t stg = 0; stg < nstage; ++stg) {
      if (stg + S - 1 < nstage) AX_ISSUE(stg + S - 1);
      const int64_t last = min(nstage - 1, stg + S - 1);
      // (both waits end in the workgroup barrier; a wave without rows
      // still takes every barrier of the stage)
      if (live) wait_ahead<PER, S>((int)(last - stg));
      else wait_ahead<XW, S>((int)(last - stg));
      const char* As = ring + (int)(stg % S) * STAGE;
      const char* Xs = As + ABYTES;
      if (live) {
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const int c0 = 4 * s + 2 * g;
          const float4 a0 = *reinterpret_cast<const float4*>(As + R * 128 + 16 * (c0 ^ sw));
          const float4 a1 = *reinterpret_cast<const float4*>(As + R * 128 + 16 * ((c0 + 1) ^ sw));
          bf16x8 ah, al;
          split_bf16x8(a0, a1, ah, al);
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) {
            const bf16x8 xh = *reinterpret_cast<const bf16x8*>(Xs + ((s * NB + cb) * 2) * 1024 + 16 * lane);
            const bf16x8 xl = *reinterpret_cast<const bf16x8*>(Xs + ((s * NB + cb) * 2 + 1) * 1024 + 16 * lane);
            acc[cb] = mfma3(ah, al, xh, xl, acc[cb]);
          }
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
#undef AX_ISSUE
}

// ---------------- Z = A^T X (split-K partials) ------------------------------
// NW waves on a 32 NW-column tile (wave w: columns 32w..32w+31 of it).
// Stage: 32 rows of the tile (4 NW KB; RPB = 2 or 1 rows per 1 KB DMA block;
// the 16-byte chunk c of row r sits at position c ^ (8 ((r >> 3) & 1))) plus
// the matching 4 NB packed X fragments, XW per wave.  The workgroup index
// gives (split, tile) over gtiles tiles per split; partials are laid out by
// 32-column block, ntiles * 4 blocks per split (ntiles = ceil(n / 128)),
// whatever the tile width.
template <int NB, int S, int NW>
__global__ void __launch_bounds__(64 * NW) atx_dma_kernel(const float* __restrict__ A,
                                                          int64_t lda, int64_t m, int64_t n,
                                                          const __bf16* __restrict__ Xp,
                                                          float* __restrict__ P, int gtiles,
                                                          int ntiles, int64_t rows_per) {
  constexpr int KC = 32;
  constexpr int TC = 32 * NW;           // tile columns
  constexpr int ABYTES = KC * TC * 4;
  constexpr int STAGE = ABYTES + NB * 4096;
  constexpr int RPB = 1024 / (TC * 4);  // rows per DMA block
  constexpr int LPR = 64 / RPB;         // lanes per row
  constexpr int XW = 4 * NB / NW;       // X fragments per wave per stage
  static_assert(RPB >= 1 && XW * NW == 4 * NB, "tile shape");
  constexpr int PER = 4 + XW;
  __shared__ __attribute__((aligned(1024))) char ring[S * STAGE];

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int split = t / gtiles, tile = t % gtiles;
  const int64_t col0 = (int64_t)tile * TC;
  const int64_t rbeg = (int64_t)split * rows_per;
  const int64_t rend = (rbeg + rows_per < m) ? rbeg + rows_per : m;
  const int64_t nstage = (rend > rbeg) ? ceil_div(rend - rbeg, KC) : 0;
  const char* xg = reinterpret_cast<const char*>(Xp) + (rbeg / 16) * NB * 2 * 1024;

  // DMA: block b = 4 * wave + i covers stage rows RPB b + lane / LPR
  int64_t colc[4];
  int rr[4];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int b = 4 * wave + i;
    rr[i] = RPB * b + lane / LPR;
    const int chunk = (lane % LPR) ^ (8 * ((rr[i] >> 3) & 1));
    int64_t c = col0 + 4 * chunk;
    colc[i] = (c + 4 <= n) ? c : 0;
  }
#define ATX_ISSUE(STG)                                                                    \
  do {                                                                                    \
    const int64_t stg_ = (STG);                                                           \
    char* slot_ = ring + (int)(stg_ % S) * STAGE;                                         \
    _Pragma("unroll") for (int i = 0; i < 4; ++i) {                                       \
      const int64_t grow_ = min(rbeg + stg_ * KC + rr[i], rend - 1);                      \
      dma16(A + grow_ * lda + colc[i], slot_ + (4 * wave + i) * 1024);                    \
    }                                                                                     \
    _Pragma("unroll") for (int i = 0; i < XW; ++i) {                                      \
      const int blk_ = wave + NW * i;                                                     \
      dma16(xg + (stg_ * (NB * 4) + blk_) * 1024 + 16 * lane, slot_ + ABYTES + blk_ * 1024); \
    }                                                                                     \
  } while (0)

  f32x16 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

#pragma unroll
  for (int u = 0; u < S - 1; ++u)
    if (u < nstage) ATX_ISSUE(u);
  const int j = lane & 31, g = lane >> 5;
  // word offset of (row 8g + jj, column 32 wave + j) inside a 16-row half
  const int chunk_r = (8 * wave + (j >> 2)) ^ (8 * g);
  const int word = chunk_r * 4 + (j & 3);
  for (int64_t stg = 0; stg < nstage; ++stg) {
    if (stg + S - 1 < nstage) ATX_ISSUE(stg + S - 1);
    const int64_t last = min(nstage - 1, stg + S - 1);
    wait_ahead<PER, S>((int)(last - stg));
    const char* As = ring + (int)(stg % S) * STAGE;
    const char* Xs = As + ABYTES;
    const float* Af = reinterpret_cast<const float*>(As);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const float* col = Af + (16 * s + 8 * g) * TC + word;
      const float4 a0 = make_float4(col[0], col[TC], col[2 * TC], col[3 * TC]);
      const float4 a1 = make_float4(col[4 * TC], col[5 * TC], col[6 * TC], col[7 * TC]);
      bf16x8 bh, bl;
      split_bf16x8(a0, a1, bh, bl);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const bf16x8 xh = *reinterpret_cast<const bf16x8*>(Xs + ((s * NB + cb) * 2) * 1024 + 16 * lane);
        const bf16x8 xl = *reinterpret_cast<const bf16x8*>(Xs + ((s * NB + cb) * 2 + 1) * 1024 + 16 * lane);
        acc[cb] = mfma3(xh, xl, bh, bl, acc[cb]);
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
#undef ATX_ISSUE
}

// built-in LDS ring depth of the 4-wave float32 kernels
static int ring_depth(int nb) { return nb >= 4 ? 2 : 3; }

static int dma_stage_bytes(int nb) { return 16384 + nb * 4096; }

static bool dma_ok(const float* A, int64_t lda, int64_t n) {
  static int env = -1;
  if (env < 0) {
    const char* e = getenv("RPCA_NO_DMA");
    env = (e && atoi(e)) ? 1 : 0;
  }
  return !env && (lda % 4) == 0 && (reinterpret_cast<uintptr_t>(A) % 16) == 0 && (n % 4) == 0;
}

bool dma_ok_shape(const void* A, int64_t lda, int64_t n) {
  return dma_ok(static_cast<const float*>(A), lda, n);
}

// (waves, ring stages) of the float32 Y = A X kernel: the configuration when
// the kernel has it, else the built-in choice: 8 waves with a four-stage ring
// (one workgroup per CU) for nb = 2 on tall A, 4 waves otherwise.
struct PassChoice {
  int nw, S;
};
// 8 waves: a 256-row tile; the ring has 4 stages (40 KB each) for nb = 2 and
// 3 (48 KB each) for nb = 4
static int ring8(int nb) { return nb == 4 ? 3 : 4; }

// nw: 16 = the tall form (built in where every CU gets 256 rows or more), 8
// or 4 waves of 32 rows
static PassChoice ax_choice(int nb, int64_t m, int num_cus, const TuneCfg* cfg) {
  const bool can8 = (nb == 2 || nb == 4);
  PassChoice c{ax_tall_ok(m, num_cus) ? 16 : 4, 0};
  if (cfg && cfg->ax_waves == 16) c.nw = 16;
  if (cfg && cfg->ax_waves == 8 && can8) c.nw = 8;
  if (cfg && cfg->ax_waves == 4) c.nw = 4;
  c.S = c.nw == 16 ? 0 : c.nw == 8 ? ring8(nb) : ((cfg && cfg->ax_ring >= 2 && cfg->ax_ring <= 4) ? cfg->ax_ring : ring_depth(nb));
  return c;
}

int atx_candidates(int nb, int (*out)[2]) {
  int k = 0;
  out[k][0] = 16; out[k][1] = 0; ++k;  // the wide form (atx_wide.hip)
  if (nb == 2 || nb == 4) { out[k][0] = 8; out[k][1] = ring8(nb); ++k; }
  for (int S = 2; S <= 4; ++S) { out[k][0] = 4; out[k][1] = S; ++k; }
  return k;
}

int ax_candidates(int nb, int (*out)[2]) {
  int k = 0;
  out[k][0] = 16; out[k][1] = 0; ++k;  // the tall form (ax_tall.hip)
  if (nb == 2 || nb == 4) { out[k][0] = 8; out[k][1] = ring8(nb); ++k; }
  for (int S = 2; S <= 4; ++S) { out[k][0] = 4; out[k][1] = S; ++k; }
  return k;
}

template <int NB>
static void launch_ax_dma(hipStream_t st, const float* A, int64_t lda, int64_t m, int64_t n,
                          const __bf16* Xp, float* Y, int64_t ldy, int num_cus,
                          const TuneCfg* cfg) {
  const PassChoice c = ax_choice(NB, m, num_cus, cfg);
  if (c.nw == 16) {
    launch_ax_tall(st, A, 0, lda, m, n, Xp, Y, ldy, NB, num_cus);
    return;
  }
  const int stage = 32 * c.nw * 128 + NB * 4096;
  const int per_cu = std::max(1, (160 * 1024) / (c.S * stage));
  int64_t G = (int64_t)num_cus * per_cu;
  G = std::min<int64_t>(G, ceil_div(m, 32));
  const int64_t rows_per = ceil_div(m, G);
  G = ceil_div(m, rows_per);
  const dim3 grid((unsigned)G);
  if constexpr (NB == 2) {
    if (c.nw == 8) {
      hipLaunchKernelGGL((ax_dma_kernel<2, 4, 8>), grid, dim3(512), 0, st, A, lda, m, n, Xp, Y, ldy, rows_per);
      return;
    }
  }
  if constexpr (NB == 4) {
    if (c.nw == 8) {
      hipLaunchKernelGGL((ax_dma_kernel<4, 3, 8>), grid, dim3(512), 0, st, A, lda, m, n, Xp, Y, ldy, rows_per);
      return;
    }
  }
  switch (c.S) {
    case 2: hipLaunchKernelGGL((ax_dma_kernel<NB, 2, 4>), grid, dim3(256), 0, st, A, lda, m, n, Xp, Y, ldy, rows_per); break;
    case 4: hipLaunchKernelGGL((ax_dma_kernel<NB, 4, 4>), grid, dim3(256), 0, st, A, lda, m, n, Xp, Y, ldy, rows_per); break;
    default: hipLaunchKernelGGL((ax_dma_kernel<NB, 3, 4>), grid, dim3(256), 0, st, A, lda, m, n, Xp, Y, ldy, rows_per); break;
  }
}

void launch_ax(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
               const __bf16* Xp, float* Y, int64_t ldy, int nb, int num_cus,
               const TuneCfg* cfg) {
  (void)dtype;
  const float* Af = static_cast<const float*>(A);
  if (dma_ok(Af, lda, n)) {
    switch (nb) {
      case 1: launch_ax_dma<1>(st, Af, lda, m, n, Xp, Y, ldy, num_cus, cfg); return;
      case 2: launch_ax_dma<2>(st, Af, lda, m, n, Xp, Y, ldy, num_cus, cfg); return;
      case 4: launch_ax_dma<4>(st, Af, lda, m, n, Xp, Y, ldy, num_cus, cfg); return;
      default: return;
    }
  }
  const int vec = ((lda % 4) == 0 && (reinterpret_cast<uintptr_t>(Af) % 16) == 0) ? 1 : 0;
  const dim3 grid((unsigned)ceil_div(m, 128));
  switch (nb) {
    case 1: hipLaunchKernelGGL(ax_f32_kernel<1>, grid, dim3(256), 0, st, Af, lda, m, n, Xp, Y, ldy, vec); break;
    case 2: hipLaunchKernelGGL(ax_f32_kernel<2>, grid, dim3(256), 0, st, Af, lda, m, n, Xp, Y, ldy, vec); break;
    case 4: hipLaunchKernelGGL(ax_f32_kernel<4>, grid, dim3(256), 0, st, Af, lda, m, n, Xp, Y, ldy, vec); break;
    default: break;
  }
}

// ------------------------------------------------------------------------
// Z = A^T X, split over rows of A.  Workgroup: 4 waves on a 128-column tile
// of A (one 32-column block per wave) and all 32*NB columns of X.  Each
// thread loads 4 rows x 4 columns of a 32-row stage (coalesced 512-byte row
// segments) and scatters them into B-operand fragments.  Partials are
// written in accumulator order and summed by atx_reduce_kernel.
// ------------------------------------------------------------------------
template <int NB>
__global__ void __launch_bounds__(256) atx_f32_kernel(const float* __restrict__ A, int64_t lda,
                                                      int64_t m, int64_t n,
                                                      const __bf16* __restrict__ Xp,
                                                      float* __restrict__ P, int ntiles,
                                                      int64_t rows_per, int vec) {
  constexpr int KC = 32;
  __shared__ __attribute__((aligned(16))) char lds_a[16 * 1024];      // [s 2][jb 4][part 2]
  __shared__ __attribute__((aligned(16))) char lds_x[NB * 4 * 1024];  // [s 2][cb NB][part 2]

  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int split = t / ntiles, tile = t % ntiles;
  const int64_t col0 = (int64_t)tile * 128;
  const int64_t rbeg = (int64_t)split * rows_per;
  const int64_t rend = (rbeg + rows_per < m) ? rbeg + rows_per : m;
  const int64_t nstage = (rend > rbeg) ? ceil_div(rend - rbeg, KC) : 0;
  const bool cols_in = (col0 + 128 <= n) && vec;
  const int64_t nfast = cols_in ? (rend - rbeg) / KC : 0;

  const int cg = tid & 31, ro = tid >> 5;
  const float* ap = A + (rbeg + 4 * ro) * lda + col0 + 4 * cg;
  const uint4* xbase = reinterpret_cast<const uint4*>(Xp + (rbeg / 16) * NB * 2 * kFragElems);
  float4 ra[4];
  uint4 rx[NB];
#define ATX_LOAD(STG)                                                                    \
  do {                                                                                   \
    const int64_t stg_ = (STG);                                                          \
    if (stg_ < nfast) {                                                                  \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) ra[q] =                              \
          *reinterpret_cast<const float4*>(ap + (stg_ * KC + q) * lda);                  \
    } else {                                                                             \
      _Pragma("unroll") for (int q = 0; q < 4; ++q) ra[q] =                              \
          load_row4(A, lda, rbeg + stg_ * KC + 4 * ro + q, col0 + 4 * cg, rend, n,       \
                    vec != 0);                                                           \
    }                                                                                    \
    _Pragma("unroll") for (int v = 0; v < NB; ++v) rx[v] =                               \
        xbase[stg_ * (NB * 256) + tid + 256 * v];                                        \
  } while (0)

  f32x16 acc[NB];
#pragma unroll
  for (int i = 0; i < NB; ++i)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;

  const int s_w = ro >> 2, g_w = (ro & 3) >> 1, jj0 = 4 * (ro & 1);
  const int jb_w = cg >> 3;
  if (nstage > 0) ATX_LOAD(0);
  for (int64_t stg = 0; stg < nstage; ++stg) {
#pragma unroll
    for (int qc = 0; qc < 4; ++qc) {
      const int j = (4 * cg + qc) & 31;
      bf16x4 h, lo;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const float x = (qc == 0) ? ra[q].x : (qc == 1) ? ra[q].y : (qc == 2) ? ra[q].z : ra[q].w;
        __bf16 th, tl;
        split_bf16(x, th, tl);
        h[q] = th;
        lo[q] = tl;
      }
      const int off = ((s_w * 4 + jb_w) * 2) * 1024 + 16 * (j + 32 * g_w) + 2 * jj0;
      *reinterpret_cast<bf16x4*>(lds_a + off) = h;
      *reinterpret_cast<bf16x4*>(lds_a + off + 1024) = lo;
    }
#pragma unroll
    for (int v = 0; v < NB; ++v) reinterpret_cast<uint4*>(lds_x)[tid + 256 * v] = rx[v];
    __syncthreads();
    if (stg + 1 < nstage) ATX_LOAD(stg + 1);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const bf16x8 bh = *reinterpret_cast<const bf16x8*>(lds_a + ((s * 4 + wave) * 2) * 1024 + 16 * lane);
      const bf16x8 bl = *reinterpret_cast<const bf16x8*>(lds_a + ((s * 4 + wave) * 2 + 1) * 1024 + 16 * lane);
#pragma unroll
      for (int cb = 0; cb < NB; ++cb) {
        const bf16x8 xh = *reinterpret_cast<const bf16x8*>(lds_x + ((s * NB + cb) * 2) * 1024 + 16 * lane);
        const bf16x8 xl = *reinterpret_cast<const bf16x8*>(lds_x + ((s * NB + cb) * 2 + 1) * 1024 + 16 * lane);
        acc[cb] = mfma3(xh, xl, bh, bl, acc[cb]);
      }
    }
    __syncthreads();
  }
#undef ATX_LOAD
  float* out = P + ((int64_t)(split * ntiles + tile) * 4 + wave) * NB * 1024;
#pragma unroll
  for (int cb = 0; cb < NB; ++cb)
#pragma unroll
    for (int r = 0; r < 16; ++r) out[(cb * 16 + r) * 64 + lane] = acc[cb][r];
}

// (waves, ring stages) of the float32 A^T X DMA kernel, as for Y = A X: 8
// waves (256-column tiles, one workgroup per CU, a four-stage ring) for nb = 2
// on wide, tall A, else 4; the low-precision kernels have one configuration.
static PassChoice atx_choice(int64_t m, int64_t n, int nb, int num_cus, int dtype,
                             const TuneCfg* cfg) {
  // low precision: the wide form (512-column tiles) on wide, tall A, else
  // 256-column tiles where the kernel has the form (its ring depth is fixed
  // by the stage size), else 128; a loaded configuration may name 16 or 4
  if (dtype != 0) {
    const bool big = n >= 1024 && m >= (int64_t)num_cus * 128;
    int nw = big ? 16 : 4;
    if (cfg && cfg->atx_waves == 16) nw = 16;
    if (cfg && cfg->atx_waves == 4) nw = 4;
    if (cfg && cfg->atx_waves == 8) nw = lp_atx_can8(nb, dtype) ? 8 : 4;
    return PassChoice{nw, 0};
  }
  // built in: the wide form (512-column tiles, atx_wide.hip) on wide, tall
  // A -- 0.315 against 0.325 ms (8 waves) at 100000 x 4000, l = 60, and 1.49
  // against 1.62 ms (4 waves) at 200000 x 8000, l = 120 -- else 4 waves; the
  // autotuner may pick any form
  const bool can8 = (nb == 2 || nb == 4);
  PassChoice c{(n >= 1024 && m >= (int64_t)num_cus * 128) ? 16 : 4, 0};
  if (cfg && cfg->atx_waves == 16) c.nw = 16;
  if (cfg && cfg->atx_waves == 8 && can8) c.nw = 8;
  if (cfg && cfg->atx_waves == 4) c.nw = 4;
  c.S = c.nw == 16 ? 0 : c.nw == 8 ? ring8(nb) : ((cfg && cfg->atx_ring >= 2 && cfg->atx_ring <= 4) ? cfg->atx_ring : ring_depth(nb));
  return c;
}

AtxPlan plan_atx(int64_t m, int64_t n, int nb, int num_cus, int dtype, const TuneCfg* cfg) {
  AtxPlan p;
  const PassChoice c = atx_choice(m, n, nb, num_cus, dtype, cfg);
  p.ntiles = (int)ceil_div(n, 128);
  p.waves = c.nw;
  p.ring = c.S;
  p.gtiles = (int)ceil_div(n, p.waves == 16 ? 512 : 32 * p.waves);
  const int rs = p.waves == 16 ? atx_wide_rows_per_stage(dtype)
                 : dtype == 0 ? 32 : lp_rows_per_stage(dtype);  // rows per stage
  const int64_t stages = ceil_div(m, rs);
  // workgroups resident per CU for the LDS ring of the DMA kernel
  const int per_cu = p.waves >= 8 ? 1
                     : dtype == 0 ? std::max(1, (160 * 1024) / (p.ring * dma_stage_bytes(nb)))
                                  : lp_per_cu(nb, dtype);
  int64_t want = (int64_t)per_cu * num_cus / p.gtiles;
  if (want < 1) want = 1;
  int64_t maxs = stages / 4;
  if (maxs < 1) maxs = 1;
  if (want > maxs) want = maxs;
  int64_t per = ceil_div(stages, want);
  p.nsplit = (int)ceil_div(stages, per);
  p.rows_per = per * rs;
  p.partial_bytes = (size_t)p.nsplit * p.ntiles * 4 * nb * 1024 * sizeof(float);
  return p;
}

size_t atx_partial_bytes_max(int64_t m, int64_t n, int nb, int num_cus, int dtype) {
  size_t b = plan_atx(m, n, nb, num_cus, dtype, nullptr).partial_bytes;
  if (dtype != 0) {
    for (int w : {4, 8, 16}) {  // every form a loaded configuration may name
      TuneCfg c;
      c.atx_waves = w;
      b = std::max(b, plan_atx(m, n, nb, num_cus, dtype, &c).partial_bytes);
    }
    return b;
  }
  int cand[8][2];
  const int k = atx_candidates(nb, cand);
  for (int i = 0; i < k; ++i) {
    TuneCfg c;
    c.atx_waves = cand[i][0];
    c.atx_ring = cand[i][1];
    b = std::max(b, plan_atx(m, n, nb, num_cus, dtype, &c).partial_bytes);
  }
  return b;
}

void launch_atx(hipStream_t st, const void* A, int dtype, int64_t lda, int64_t m, int64_t n,
                const __bf16* Xp, float* P, const AtxPlan& plan, int nb) {
  (void)dtype;
  const float* Af = static_cast<const float*>(A);
  const dim3 grid((unsigned)(plan.ntiles * plan.nsplit));
  if (dma_ok(Af, lda, n) && plan.waves == 16) {
    launch_atx_wide(st, A, 0, lda, m, n, Xp, P, plan, nb);
    return;
  }
  if (dma_ok(Af, lda, n)) {
    const int S = plan.ring;
    if (plan.waves == 8 && nb == 2) {
      hipLaunchKernelGGL((atx_dma_kernel<2, 4, 8>), dim3((unsigned)(plan.gtiles * plan.nsplit)),
                         dim3(512), 0, st, Af, lda, m, n, Xp, P, plan.gtiles, plan.ntiles,
                         plan.rows_per);
      return;
    }
    if (plan.waves == 8 && nb == 4) {
      hipLaunchKernelGGL((atx_dma_kernel<4, 3, 8>), dim3((unsigned)(plan.gtiles * plan.nsplit)),
                         dim3(512), 0, st, Af, lda, m, n, Xp, P, plan.gtiles, plan.ntiles,
                         plan.rows_per);
      return;
    }
#define ATX_DMA(NB_)                                                                                 \
  switch (S) {                                                                                       \
    case 2: hipLaunchKernelGGL((atx_dma_kernel<NB_, 2, 4>), grid, dim3(256), 0, st, Af, lda, m, n, Xp, P, plan.ntiles, plan.ntiles, plan.rows_per); break; \
    case 4: hipLaunchKernelGGL((atx_dma_kernel<NB_, 4, 4>), grid, dim3(256), 0, st, Af, lda, m, n, Xp, P, plan.ntiles, plan.ntiles, plan.rows_per); break; \
    default: hipLaunchKernelGGL((atx_dma_kernel<NB_, 3, 4>), grid, dim3(256), 0, st, Af, lda, m, n, Xp, P, plan.ntiles, plan.ntiles, plan.rows_per); break; \
  }
    switch (nb) {
      case 1: ATX_DMA(1); return;
      case 2: ATX_DMA(2); return;
      case 4: ATX_DMA(4); return;
      default: return;
    }
#undef ATX_DMA
  }
  const int vec = ((lda % 4) == 0 && (reinterpret_cast<uintptr_t>(Af) % 16) == 0) ? 1 : 0;
  switch (nb) {
    case 1: hipLaunchKernelGGL(atx_f32_kernel<1>, grid, dim3(256), 0, st, Af, lda, m, n, Xp, P, plan.ntiles, plan.rows_per, vec); break;
    case 2: hipLaunchKernelGGL(atx_f32_kernel<2>, grid, dim3(256), 0, st, Af, lda, m, n, Xp, P, plan.ntiles, plan.rows_per, vec); break;
    case 4: hipLaunchKernelGGL(atx_f32_kernel<4>, grid, dim3(256), 0, st, Af, lda, m, n, Xp, P, plan.ntiles, plan.rows_per, vec); break;
    default: break;
  }
}

// Z[j][c] = sum over splits of the partial at (tile, wave, cb, r, lane).
__global__ void __launch_bounds__(256) atx_reduce_kernel(const float* __restrict__ P, int nsplit,
                                                         int ntiles, int nb, int64_t n,
                                                         const float* __restrict__ cscale,
                                                         float* __restrict__ Z, int64_t ldz) {
  const int64_t per_split = (int64_t)ntiles * 4 * nb * 1024;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= per_split) return;
  const int lane = (int)(e & 63);
  const int r = (int)((e >> 6) & 15);
  const int cb = (int)((e >> 10) % nb);
  const int64_t wt = (e >> 10) / nb;  // tile * 4 + wave
  const int64_t j = (wt >> 2) * 128 + 32 * (wt & 3) + (lane & 31);
  if (j >= n) return;
  const int c = 32 * cb + (r & 3) + 4 * (lane >> 5) + 8 * (r >> 2);
  float s = 0.f;
  for (int sp = 0; sp < nsplit; ++sp) s += P[sp * per_split + e];
  if (cscale) s *= cscale[j];
  Z[j * ldz + c] = s;
}

void launch_atx_reduce(hipStream_t st, const float* P, const AtxPlan& plan, int nb, int64_t n,
                       const float* cscale, float* Z, int64_t ldz) {
  const int64_t per_split = (int64_t)plan.ntiles * 4 * nb * 1024;
  hipLaunchKernelGGL(atx_reduce_kernel, dim3((unsigned)ceil_div(per_split, 256)), dim3(256), 0, st,
                     P, plan.nsplit, plan.ntiles, nb, n, cscale, Z, ldz);
}

}  // namespace rpca
