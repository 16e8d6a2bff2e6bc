// Pivot selection for the LU renormalization (Section 5: an LU decomposition
// with partial pivoting renormalizes Q after each application of A or A*,
// except the last).  The renormalized matrix is P L = Y U^-1, so only U and
// the pivot rows are needed; the solve itself is trsm_kernel (tall.hip).
//
// Tall Y (up to 10^6 rows) cannot be factored column by column with a
// grid-wide argmax per column, so pivots are chosen by tournament (Grigori,
// Demmel and Xiang's CALU): every 256-row block runs Gaussian elimination
// with partial pivoting on its own rows and nominates its l pivot rows; the
// nominated original rows of F = 256/lp blocks are merged by the same
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
#include "common.h"
#include "kernels.h"

namespace rpca {

struct LuLevels {
  int levels;
  int nblk[16];
  int cand_off[16];
  int cnt_off[16];
};

// Gaussian elimination with partial pivoting over the rows held by the 256
// threads of a workgroup (one row per thread, in registers).  Chooses up to
// l pivot rows; ties in |value| go to the smaller global row index.  When
// ``U`` is given the eliminated pivot rows are written to it.
// Gaussian elimination with partial pivoting over the rows held by the 256
// threads of a workgroup (one row per thread, in registers; the column loop
// is unrolled so every row access has a constant index).  Chooses up to l
// pivot rows; ties in |value| go to the smaller global row index.  When
// ``U`` is given the eliminated pivot rows are written to it.
template <int LP>
__device__ __forceinline__ void gepp_block(float (&row)[LP], bool cand, int gidx, int l, int* s_piv,
                           float* s_wkey, int* s_widx, float* s_wrow, float* U) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll
  for (int p = 0; p < LP; ++p) {
    if (p < l) {
      const int buf = p & 1;
      float key = cand ? fabsf(row[p]) : -1.f;
      int idx = cand ? gidx : 0x7fffffff;
      wave_argmax(key, idx);
      if (lane == 0) {
        s_wkey[buf * 4 + wave] = key;
        s_widx[buf * 4 + wave] = idx;
      }
      if (cand && gidx == idx) {
        float4* dst = reinterpret_cast<float4*>(s_wrow + (buf * 4 + wave) * LP);
#pragma unroll
        for (int c = 0; c < LP; c += 4)
          if (c + 3 >= p) dst[c / 4] = make_float4(row[c], row[c + 1], row[c + 2], row[c + 3]);
      }
      __syncthreads();
      float bk = s_wkey[buf * 4];
      int bi = s_widx[buf * 4], bw = 0;
#pragma unroll
      for (int w = 1; w < 4; ++w) {
        const float k2 = s_wkey[buf * 4 + w];
        const int i2 = s_widx[buf * 4 + w];
        if (k2 > bk || (k2 == bk && i2 < bi)) {
          bk = k2;
          bi = i2;
          bw = w;
        }
      }
      const float* prow = s_wrow + (buf * 4 + bw) * LP;
      const bool have = (bk >= 0.f);  // some candidate row was left
      if (tid == 0) s_piv[p] = have ? bi : -1;
      if (U && tid < LP) U[p * LP + tid] = (have && tid >= p && tid < l) ? prow[tid] : 0.f;
      if (cand && gidx == bi) {
        cand = false;
      } else if (cand && bk > 0.f) {
        const float mult = row[p] / prow[p];
#pragma unroll
        for (int c = 0; c < LP; ++c)
          if (c > p) row[c] -= mult * prow[c];
      }
    }
  }
  __syncthreads();
}

template <int LP>
__global__ void __launch_bounds__(256) lu_tree_kernel(const float* __restrict__ X, int64_t ldx,
                                                      int64_t rows, int l, LuLevels lv,
                                                      int* __restrict__ cand,
                                                      unsigned* __restrict__ counters,
                                                      float* __restrict__ U,
                                                      int* __restrict__ piv) {
  constexpr int F = 256 / LP;
  __shared__ int s_piv[LP];
  __shared__ float s_wkey[8];
  __shared__ int s_widx[8];
  __shared__ __attribute__((aligned(16))) float s_wrow[8 * LP];
  __shared__ int s_last;
  const int tid = threadIdx.x;
  int level = 0, blk = blockIdx.x;
  while (true) {
    float row[LP];
    bool valid = false;
    int gidx = 0x7fffffff;
    if (level == 0) {
      const int64_t r = (int64_t)blk * 256 + tid;
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
    gepp_block<LP>(row, valid, gidx, l, s_piv, s_wkey, s_widx, s_wrow, root ? U : nullptr);
    if (root) {
      if (tid < LP) piv[tid] = (tid < l) ? s_piv[tid] : -1;
      for (int e = l * LP + tid; e < LP * LP; e += 256) U[e] = 0.f;
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

LuPlan plan_lu(int64_t rows, int lp) {
  LuPlan p{};
  p.lp = lp;
  const int F = 256 / lp;
  int nb = (int)ceil_div(rows, 256);
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
  switch (plan.lp) {
    case 32: hipLaunchKernelGGL(lu_tree_kernel<32>, grid, dim3(256), 0, st, X, ldx, rows, l, lv, cand, counters, U, piv); break;
    case 64: hipLaunchKernelGGL(lu_tree_kernel<64>, grid, dim3(256), 0, st, X, ldx, rows, l, lv, cand, counters, U, piv); break;
    case 128: hipLaunchKernelGGL(lu_tree_kernel<128>, grid, dim3(256), 0, st, X, ldx, rows, l, lv, cand, counters, U, piv); break;
    default: break;
  }
}

}  // namespace rpca
