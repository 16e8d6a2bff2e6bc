// Pivot selection for the LU renormalization (Section 5: an LU decomposition
// with partial pivoting renormalizes Q after each application of A or A*,
// except the last).  The renormalized matrix is P L = Y U^-1, so only U and
// the pivot rows are needed; the solve itself is trsm_kernel (tall.hip).
//
// Tall Y (up to 10^6 rows) cannot be factored column by column with a
// grid-wide argmax per column, so pivots are chosen by tournament (Grigori,
// Demmel and Xiang's CALU): every block of NT rows (NT = 512 by default;
// one row per thread) runs Gaussian elimination with
// partial pivoting on its own rows and nominates its l pivot rows; the
// nominated original rows of F = NT/lp blocks are merged by the same
// elimination, level after level, until one set of l rows is left; its
// elimination gives U.  The levels run inside one launch: the last
// workgroup to finish a group (an atomic arrival counter) merges it, so no
// grid-wide barrier is needed and every workgroup exits after its own block.
// Counters are reset by the workgroup that consumed them.
//
// Zero pivots follow LAPACK's getrf: when the remaining column is exactly
// zero, the first unused row is taken as pivot, U[j][j] = 0, and nothing is
// eliminated; the solve then makes column j of P L the unit vector of that
// row, so span(P L) contains span(Y).
#include <cstdlib>

#include "common.h"
#include "kernels.h"

namespace rpca {

struct LuLevels {
  int levels;
  int nblk[16];
  int cand_off[16];
  int cnt_off[16];
};

template <int LP, int NT_>
struct LuCfg {
  static constexpr int NT = NT_;       // threads = rows per block
  static constexpr int NW = NT / 64;   // waves
  static constexpr int F = NT / LP;    // candidate sets merged per block
};

// row[c] <- row[c+1] - mult * prow[c+1] for c < W - 1 (the moving frame, see
// gepp_block), prow streamed from LDS four values at a time.
template <int W, int LP>
__device__ __forceinline__ void shift_update(float (&row)[LP], float mult, const float* prow) {
  static_assert(W <= LP && W % 4 == 0, "width");
  float4 cur = *reinterpret_cast<const float4*>(prow);
#pragma unroll
  for (int c = 0; c < W; c += 4) {
    const float4 nxt = (c + 4 < W) ? *reinterpret_cast<const float4*>(prow + c + 4)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
    row[c] = row[c + 1] - mult * cur.y;
    row[c + 1] = row[c + 2] - mult * cur.z;
    row[c + 2] = row[c + 3] - mult * cur.w;
    if (c + 4 < W) row[c + 3] = row[c + 4] - mult * nxt.x;
    else row[c + 3] = 0.f;
    cur = nxt;
  }
}

template <int LP>
__device__ __forceinline__ void shift_bucket(float (&row)[LP], float mult, const float* prow,
                                             int live) {
  if (LP >= 128 && live > 96) shift_update<(LP >= 128 ? 128 : 16), LP>(row, mult, prow);
  else if (LP >= 128 && live > 64) shift_update<(LP >= 128 ? 96 : 16), LP>(row, mult, prow);
  else if (LP >= 64 && live > 48) shift_update<(LP >= 64 ? 64 : 16), LP>(row, mult, prow);
  else if (LP >= 64 && live > 32) shift_update<(LP >= 64 ? 48 : 16), LP>(row, mult, prow);
  else if (live > 16) shift_update<(LP >= 32 ? 32 : 16), LP>(row, mult, prow);
  else shift_update<16, LP>(row, mult, prow);
}

// Gaussian elimination with partial pivoting over the rows held by the NT
// threads of a workgroup (one row per thread, in registers).  The row is kept
// in a moving frame: before step p, register c holds column p + c, and the
// elimination update writes the shifted row, so the current column is always
// row[0] and no register is addressed by a run-time index.
//
// The pivot search works on one 32-bit key per row: the top bits of |row[0]|
// (sign, exponent and 13 fraction bits) above NT - tid in the low KB bits,
// 0 for rows that are no longer candidates.  The largest key is the largest
// |value| up to 2^-13 relative (so |L| <= 1 + 2^-13), ties going to the lower
// thread slot; |values| below 2^-100 count as zero; every key is distinct, so a wave maximum (six DPP max steps)
// names its row.  Per step: the wave maximum, the wave winner's live row and
// global index to LDS, one barrier, the maximum of the NW wave keys, the pivot
// row streamed from LDS into the update of the live columns.  A key whose
// value bits are all zero is a zero pivot (LAPACK getrf: nothing is
// eliminated and U[p][p] = 0).  When ``U`` (LDS) is given the eliminated
// pivot rows (row p of U = pivot row in frame p) are written to it.
__device__ __forceinline__ unsigned dpp_max_u32(unsigned v, int sel) {
  unsigned o;
  switch (sel) {
    case 0: o = __builtin_amdgcn_update_dpp(0u, v, 0xB1, 0xF, 0xF, false); break;   // quad_perm [1,0,3,2]
    case 1: o = __builtin_amdgcn_update_dpp(0u, v, 0x4E, 0xF, 0xF, false); break;   // quad_perm [2,3,0,1]
    case 2: o = __builtin_amdgcn_update_dpp(0u, v, 0x141, 0xF, 0xF, false); break;  // row_half_mirror
    case 3: o = __builtin_amdgcn_update_dpp(0u, v, 0x140, 0xF, 0xF, false); break;  // row_mirror
    case 4: o = __builtin_amdgcn_update_dpp(0u, v, 0x142, 0xA, 0xF, false); break;  // row_bcast:15
    default: o = __builtin_amdgcn_update_dpp(0u, v, 0x143, 0xC, 0xF, false); break; // row_bcast:31
  }
  return max(v, o);
}

__device__ __forceinline__ unsigned wave_max_key(unsigned k) {
#pragma unroll
  for (int s = 0; s < 6; ++s) k = dpp_max_u32(k, s);
  return (unsigned)__builtin_amdgcn_readlane((int)k, 63);
}

template <int LP, int NT>
__device__ __forceinline__ void gepp_block(float (&row)[LP], bool cand, int gidx, int l,
                                           int* s_piv, unsigned* s_wkey, int* s_widx,
                                           float* s_wrow, float* U) {
  constexpr int NW = LuCfg<LP, NT>::NW;
  constexpr int KB = (NT <= 255) ? 8 : (NT <= 511 ? 9 : (NT <= 1023 ? 10 : 11));  // bits for NT - tid
  constexpr unsigned KMASK = (1u << KB) - 1u;
  static_assert(NT <= (int)KMASK, "slot bits");
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const unsigned slot = (unsigned)(NT - tid);  // 1 .. NT
  for (int p = 0; p < l; ++p) {
    const int buf = p & 1;
    const int live = l - p;
    // values below 2^-100 count as zero pivots (their reciprocal would overflow)
    const float a0 = fabsf(row[0]);
    const unsigned vbits = (a0 >= 7.8886091e-31f) ? (__float_as_uint(a0) & ~KMASK) : 0u;
    const unsigned key = cand ? (vbits | slot) : 0u;
    const unsigned wmax = wave_max_key(key);
    if (wmax != 0u && key == wmax) {  // this wave's candidate for the pivot
      s_wkey[buf * NW + wave] = wmax;
      s_widx[buf * NW + wave] = gidx;
      float4* dst = reinterpret_cast<float4*>(s_wrow + (buf * NW + wave) * LP);
#pragma unroll
      for (int c = 0; c < LP; c += 4)
        if (c < live) dst[c / 4] = make_float4(row[c], row[c + 1], row[c + 2], row[c + 3]);
    } else if (wmax == 0u && lane == 0) {
      s_wkey[buf * NW + wave] = 0u;
    }
    __syncthreads();
    unsigned gk = 0u;
#pragma unroll
    for (int w = 0; w < NW; w += 4) {
      const uint4 k4 = *reinterpret_cast<const uint4*>(s_wkey + buf * NW + w);
      gk = max(gk, max(max(k4.x, k4.y), max(k4.z, k4.w)));
    }
    const bool have = gk != 0u;  // some candidate row was left
    const int wt = NT - (int)(gk & KMASK);  // thread slot of the pivot row
    const int bw = have ? (wt >> 6) : 0;
    const float* prow = s_wrow + (buf * NW + bw) * LP;
    const bool nonzero = (gk & ~KMASK) != 0u;
    if (tid == 0) s_piv[p] = have ? s_widx[buf * NW + bw] : -1;
    if (U && tid < LP)  // LDS
      U[p * LP + tid] = (have && tid >= p && tid < l && (nonzero || tid > p)) ? prow[tid - p] : 0.f;
    const float inv = nonzero ? __builtin_amdgcn_rcpf(prow[0]) : 0.f;
    float mult = 0.f;
    if (cand && tid == wt) cand = false;
    else if (cand) mult = row[0] * inv;
    shift_bucket<LP>(row, mult, prow, live);
  }
  __syncthreads();
}

template <int LP, int NT_>
__global__ void __launch_bounds__(NT_) lu_tree_kernel(const float* __restrict__ X, int64_t ldx,
                                                      int64_t rows, int l, LuLevels lv,
                                                      int* __restrict__ cand,
                                                      unsigned* __restrict__ counters,
                                                      float* __restrict__ U,
                                                      int* __restrict__ piv) {
  constexpr int NT = LuCfg<LP, NT_>::NT, NW = LuCfg<LP, NT_>::NW, F = LuCfg<LP, NT_>::F;
  __shared__ int s_piv[LP];
  __shared__ __attribute__((aligned(16))) unsigned s_wkey[2 * NW];
  __shared__ __attribute__((aligned(16))) int s_widx[2 * NW];
  __shared__ __attribute__((aligned(16))) float s_wrow[2 * NW * LP];
  __shared__ float s_U[LP * LP];  // U of the root block (global stores stay out of the steps)
  __shared__ int s_last;
  const int tid = threadIdx.x;
  int level = 0, blk = blockIdx.x;
  while (true) {
    float row[LP];
    bool valid = false;
    int gidx = 0x7fffffff;
    if (level == 0) {
      const int64_t r = (int64_t)blk * NT + tid;
      valid = r < rows;
      gidx = (int)r;
    } else {
      const int child = blk * F + tid / LP, p = tid % LP;
      if (child < lv.nblk[level - 1] && p < l) {
        const int ci = __hip_atomic_load(&cand[lv.cand_off[level - 1] + child * LP + p],
                                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (ci >= 0) {
          valid = true;
          gidx = ci;
        }
      }
    }
    if (valid) {
      const float* src = X + (int64_t)gidx * ldx;
#pragma unroll
      for (int c = 0; c < LP; c += 4) {
        const float4 v = *reinterpret_cast<const float4*>(src + c);
        row[c] = v.x; row[c + 1] = v.y; row[c + 2] = v.z; row[c + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int c = 0; c < LP; ++c) row[c] = 0.f;
    }
    const bool root = (lv.nblk[level] == 1);
    gepp_block<LP, NT>(row, valid, gidx, l, s_piv, s_wkey, s_widx, s_wrow, root ? s_U : nullptr);
    if (root) {
      if (tid < LP) piv[tid] = (tid < l) ? s_piv[tid] : -1;
      for (int e = tid; e < LP * LP; e += NT) U[e] = (e < l * LP) ? s_U[e] : 0.f;
      return;
    }
    if (tid < LP) cand[lv.cand_off[level] + blk * LP + tid] = (tid < l) ? s_piv[tid] : -1;
    __threadfence();
    __syncthreads();
    const int parent = blk / F;
    if (tid == 0) {
      const int nchild = min(F, lv.nblk[level] - parent * F);
      unsigned* ctr = counters + lv.cnt_off[level + 1] + parent;
      const unsigned old = atomicAdd(ctr, 1u);
      const int last = (old == (unsigned)(nchild - 1));
      if (last) __hip_atomic_store(ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = last;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();
    ++level;
    blk = parent;
  }
}

// rows per block (= threads); RPCA_LU_NT overrides for tuning
static int lu_block_rows(int lp) {
  static int env = -1;
  if (env < 0) {
    const char* e = getenv("RPCA_LU_NT");
    env = e ? atoi(e) : 0;
  }
  int nt = 512;
  if (env == 256 || env == 512 || (env == 1024 && lp <= 64)) nt = env;
  if (nt < 2 * lp) nt = 2 * lp;
  return nt;
}

LuPlan plan_lu(int64_t rows, int lp) {
  LuPlan p{};
  p.lp = lp;
  const int NT = lu_block_rows(lp);
  const int F = NT / lp;
  int nb = (int)ceil_div(rows, NT);
  int64_t coff = 0, koff = 0;
  p.levels = 0;
  while (true) {
    p.nblk[p.levels] = nb;
    p.cand_off[p.levels] = coff;
    coff += (int64_t)nb * lp;
    ++p.levels;
    if (nb == 1) break;
    nb = (int)ceil_div(nb, F);
    koff += nb;
  }
  p.cand_total = coff;
  p.counter_total = koff + 1;
  return p;
}

void launch_lu_tree(hipStream_t st, const float* X, int64_t ldx, int64_t rows, int l,
                    const LuPlan& plan, int* cand, unsigned* counters, float* U, int* piv) {
  LuLevels lv{};
  lv.levels = plan.levels;
  // counters of level i >= 1 (one per block of that level, counting the
  // arrivals of its children) start at cnt_off[i]
  int acc = 0;
  for (int i = 0; i < plan.levels; ++i) {
    lv.nblk[i] = plan.nblk[i];
    lv.cand_off[i] = (int)plan.cand_off[i];
    lv.cnt_off[i] = acc;
    if (i >= 1) acc += plan.nblk[i];
  }
  const dim3 grid((unsigned)plan.nblk[0]);
  const int nt = lu_block_rows(plan.lp);
#define LU_LAUNCH(LP_, NT_)                                                                  \
  hipLaunchKernelGGL((lu_tree_kernel<LP_, NT_>), grid, dim3(NT_), 0, st, X, ldx, rows, l, lv, \
                     cand, counters, U, piv)
  if (plan.lp == 32) {
    if (nt == 1024) LU_LAUNCH(32, 1024);
    else if (nt == 512) LU_LAUNCH(32, 512);
    else LU_LAUNCH(32, 256);
  } else if (plan.lp == 64) {
    if (nt == 1024) LU_LAUNCH(64, 1024);
    else if (nt == 512) LU_LAUNCH(64, 512);
    else LU_LAUNCH(64, 256);
  } else if (plan.lp == 128) {
    LU_LAUNCH(128, 512);
  }
#undef LU_LAUNCH
}

}  // namespace rpca
