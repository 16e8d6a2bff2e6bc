// Pivot selection for the LU renormalization (Section 5: an LU decomposition
// with partial pivoting renormalizes Q after each application of A or A*,
// except the last).  The renormalized matrix is P L = Y U^-1, so only U and
// the pivot rows are needed; the solve itself is trsm_kernel (tall.hip).
//
// Tall Y (up to 10^6 rows) cannot be factored column by column with a
// grid-wide argmax per column, so pivots are chosen by tournament (Grigori,
// Demmel and Xiang's CALU): every block of R rows (R = 512 by default, 512
// threads) runs Gaussian elimination with partial pivoting on its own rows
// and nominates its l pivot rows; the nominated original rows of F = R/lp
// blocks are merged by the same elimination, level after level, until one
// set of l rows is left; its elimination gives U.  The levels run inside one
// launch: the last workgroup to finish a group (an atomic arrival counter)
// merges it, so no grid-wide barrier is needed and every workgroup exits
// after its own block.
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

template <int LP, int R_, int NT_>
struct LuCfg {
  static constexpr int R = R_;          // rows per block
  static constexpr int NT = NT_;        // threads
  static constexpr int NW = NT / 64;    // waves
  static constexpr int RPL = R / 64;    // rows per lane
  static constexpr int CPW = LP / NW;   // columns per wave (frame slots)
  static constexpr int F = R / LP;      // candidate sets merged per block
  static constexpr int KB = (R <= 255) ? 8 : (R <= 511 ? 9 : (R <= 1023 ? 10 : 11));
  static constexpr unsigned KMASK = (1u << KB) - 1u;  // bits for R - local row
  static constexpr int SROW = LP + 1;                 // staging row stride (floats)
  static constexpr int STAGE = 2 * 64 * SROW;         // two 64-row staging buffers
  static constexpr int SHARED = STAGE > LP * LP ? STAGE : LP * LP;  // staging, then U
  static constexpr int PF = 64 * LP / 4 / NT;         // float4 loads per thread per chunk
  static constexpr int PD = (LP >= 128) ? 2 : 3;      // chunks in flight
  static_assert(RPL % 4 == 0 && CPW >= 2 && PF >= 1 && R % LP == 0, "LU block shape");
};

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

__device__ __forceinline__ float lane_read(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// Gaussian elimination with partial pivoting over the R rows of a block,
// distributed by columns: lane `lane` of every wave holds rows lane + 64 s
// (s < RPL); wave w holds columns w + NW t in slots t < CPW.  The steps run in
// CPW super-steps of NW steps; in super-step B the pivot column j = NW B + wp
// is slot B of wave wp, and slots below B hold finished columns, so slot
// indices are compile-time constants (template recursion over B) and no
// register is addressed by a run-time index.
//
// A step: the wave that holds column j finds the pivot within the wave (one
// 32-bit key per row, six DPP max steps), forms the multipliers of its rows
// and writes them and the key to LDS (double buffered by step parity); after
// one barrier every wave reads them, takes the pivot row's entries of its own
// columns from the owning lane (readlane) and updates its columns.  Slots B
// and B + 1 (one of which holds column j + 1) are updated first, then the
// wave that holds column j + 1 publishes step j + 1, then the other slots are
// updated.  The update has no branches (a slot that is not live gets a zero
// pivot-row entry), so the row registers stay in place.
//
// Rows are never swapped.  A row leaves the candidate set (a bit per row) when
// it becomes a pivot; it is still updated with the rest, but never read again.
// Key: the top bits of |a| (exponent and 13 fraction bits) above R - local
// row in the low KB bits, 0 for a non-candidate.  The largest key is the
// largest |value| up to 2^-13 relative (|L| <= 1 + 2^-13 within a block), ties
// going to the lower row.  A pivot below 2^-100 (including 0) is a zero
// pivot, as in LAPACK getrf for an exactly zero column: nothing is eliminated
// and U[j][j] = 0.
template <int LP, int R, int NT>
struct Gepp {
  using C = LuCfg<LP, R, NT>;
  static constexpr int RPL = C::RPL, CPW = C::CPW, NW = C::NW;
  static constexpr unsigned KMASK = C::KMASK;
  static constexpr unsigned VMASK = 0x7fffffffu & ~KMASK;  // |value| bits of a key
  static constexpr unsigned TINY = 0x0d800000u;            // 2^-100

  struct Ctx {
    int lane, w, l;
    unsigned live;  // slots whose column is < l
    int* s_lr;
    float* s_mult;
    unsigned* s_key;
    float* sU;
  };

  // a[.][T] -= m * (slot T live ? u[T] : 0)
  template <int T>
  static __device__ __forceinline__ void update(float (&a)[RPL][CPW], const float (&m)[RPL],
                                                const float (&u)[CPW], unsigned lm) {
    const float ut = ((lm >> T) & 1u) ? u[T] : 0.f;
#pragma unroll
    for (int s = 0; s < RPL; ++s) a[s][T] -= m[s] * ut;
  }

  // Pivot search on slot T (the owner wave); multipliers and key to LDS.
  template <int T>
  static __device__ __forceinline__ void publish(const float (&a)[RPL][CPW], unsigned cm,
                                                 const Ctx& c, int j) {
    unsigned best = 0u;
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      const unsigned key = (__float_as_uint(a[s][T]) & VMASK) | (unsigned)(R - 64 * s - c.lane);
      best = max(best, ((cm >> s) & 1u) ? key : 0u);
    }
    const unsigned wmax = wave_max_key(best);
    const bool nonzero = (wmax & ~KMASK) >= TINY;
    const int lr = R - (int)(wmax & KMASK);  // local pivot row (R when there is none)
    const int ls = lr & 63, ss = lr >> 6;
    float pv = 0.f;
#pragma unroll
    for (int s = 0; s < RPL; ++s)
      if (s == ss) pv = lane_read(a[s][T], ls);
    const float inv = nonzero ? __builtin_amdgcn_rcpf(pv) : 0.f;
    float4* dst = reinterpret_cast<float4*>(c.s_mult + (j & 1) * R + c.lane * RPL);
#pragma unroll
    for (int s = 0; s < RPL; s += 4)
      dst[s / 4] = make_float4(a[s][T] * inv, a[s + 1][T] * inv, a[s + 2][T] * inv,
                               a[s + 3][T] * inv);
    if (c.lane == 0) {
      c.s_key[j & 1] = wmax;
      if (wmax != 0u) {
        c.s_lr[j] = lr;
        if (c.sU) c.sU[j * LP + j] = nonzero ? pv : 0.f;
      }
    }
  }

  template <int T>
  static __device__ __forceinline__ void update_from(float (&a)[RPL][CPW], const float (&m)[RPL],
                                                     const float (&u)[CPW], unsigned lm) {
    if constexpr (T < CPW) {
      update<T>(a, m, u, lm);
      update_from<T + 1>(a, m, u, lm);
    }
  }

  // The NW steps of super-step B, then the next super-step, up to column l.
  template <int B>
  static __device__ __forceinline__ void steps(float (&a)[RPL][CPW], unsigned& cm,
                                               const Ctx& c) {
    if constexpr (B < CPW) {
      for (int wp = 0; wp < NW; ++wp) {
        const int j = NW * B + wp;
        if (j >= c.l) return;
        __syncthreads();
        float m[RPL];
        const float4* src =
            reinterpret_cast<const float4*>(c.s_mult + (j & 1) * R + c.lane * RPL);
#pragma unroll
        for (int s = 0; s < RPL; s += 4) {
          const float4 v = src[s / 4];
          m[s] = v.x; m[s + 1] = v.y; m[s + 2] = v.z; m[s + 3] = v.w;
        }
        // key 0: no candidate row is left; the step then eliminates nothing
        // and records no pivot (no early exit, so the multiplier reads above
        // are issued together with this one)
        const unsigned key = (unsigned)__builtin_amdgcn_readfirstlane((int)c.s_key[j & 1]);
        const bool nz = (key & ~KMASK) >= TINY;
        const int lr = R - (int)(key & KMASK), ls = lr & 63, ss = lr >> 6;
        float u[CPW];
#pragma unroll
        for (int t = 0; t < CPW; ++t) u[t] = 0.f;
#pragma unroll
        for (int s = 0; s < RPL; ++s)
          if (s == ss) {
#pragma unroll
            for (int t = B; t < CPW; ++t) u[t] = lane_read(a[s][t], ls);
          }
        if (c.lane == ls) cm &= ~(1u << ss);
        // live slots: column w + NW t is right of j and left of l
        unsigned lm = c.live;
        if (c.w <= wp) lm &= ~(1u << B);
        if (c.sU && c.lane == 0) {
#pragma unroll
          for (int t = B; t < CPW; ++t)
            if ((lm >> t) & 1u) c.sU[j * LP + c.w + NW * t] = u[t];
        }
        if (!nz) lm = 0u;
        const int jn = j + 1;
        const bool next = jn < c.l && c.w == (wp + 1) % NW;
        // the wave that publishes column j + 1 is the critical path of the
        // step: it takes issue priority over the other wave on its SIMD until
        // it has published
        if (next) __builtin_amdgcn_s_setprio(2);
        update<B>(a, m, u, lm);
        if constexpr (B + 1 < CPW) update<B + 1>(a, m, u, lm);
        if (next) {
          // column j + 1: slot B, or slot B + 1 when it starts the next super-step
          if (wp != NW - 1) {
            publish<B>(a, cm, c, jn);
          } else {
            if constexpr (B + 1 < CPW) publish<B + 1>(a, cm, c, jn);
          }
          __builtin_amdgcn_s_setprio(0);
        }
        update_from<B + 2>(a, m, u, lm);
      }
      steps<B + 1>(a, cm, c);
    }
  }

  // a: the block's rows (see above, zero where a row does not exist); valid:
  // bit s = row lane + 64 s exists.  Writes s_lr[j] (local pivot row, left as
  // is when no candidate remains) and, when sU is given, U (LDS, zeroed by
  // the caller).
  static __device__ __forceinline__ void run(float (&a)[RPL][CPW], unsigned valid, int l,
                                             int* s_lr, float* s_mult, unsigned* s_key,
                                             float* sU) {
    Ctx c;
    c.lane = threadIdx.x & 63;
    c.w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    c.l = l;
    const int left = l - c.w;
    const int t1 = left <= 0 ? 0 : min(CPW, (left + NW - 1) / NW);
    c.live = (t1 >= 32) ? ~0u : ((1u << t1) - 1u);
    c.s_lr = s_lr;
    c.s_mult = s_mult;
    c.s_key = s_key;
    c.sU = sU;
    unsigned cm = valid;  // candidate rows (bit s: row lane + 64 s)
    if (c.w == 0 && l > 0) publish<0>(a, cm, c, 0);
    steps<0>(a, cm, c);
    __syncthreads();
  }
};

template <int LP, int R, int NT>
__global__ void __launch_bounds__(NT) lu_tree_kernel(const float* __restrict__ X, int64_t ldx,
                                                     int64_t rows, int l, LuLevels lv,
                                                     int* __restrict__ cand,
                                                     unsigned* __restrict__ counters,
                                                     float* __restrict__ U,
                                                     int* __restrict__ piv) {
  using C = LuCfg<LP, R, NT>;
  constexpr int NW = C::NW, RPL = C::RPL, CPW = C::CPW, F = C::F, SROW = C::SROW, PF = C::PF,
                PD = C::PD;
  __shared__ int s_lr[LP];  // local pivot rows
  __shared__ int s_gidx[R];
  __shared__ __attribute__((aligned(16))) float s_mult[2 * R];
  __shared__ unsigned s_key[2];
  __shared__ __attribute__((aligned(16))) float s_big[C::SHARED];  // staging, then U of the root
  __shared__ int s_last;
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  int level = 0, blk = blockIdx.x;
  while (true) {
    // global row of each local row (-1: none)
    for (int i = tid; i < R; i += NT) {
      int g = -1;
      if (level == 0) {
        const int64_t r = (int64_t)blk * R + i;
        if (r < rows) g = (int)r;
      } else {
        const int child = blk * F + i / LP, p = i % LP;
        if (child < lv.nblk[level - 1] && p < l) {
          const int ci = __hip_atomic_load(&cand[lv.cand_off[level - 1] + child * LP + p],
                                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (ci >= 0) g = ci;
        }
      }
      s_gidx[i] = g;
    }
    if (tid < LP) s_lr[tid] = -1;
    __syncthreads();
    unsigned valid = 0u;
#pragma unroll
    for (int s = 0; s < RPL; ++s)
      if (s_gidx[64 * s + lane] >= 0) valid |= 1u << s;
    // rows to registers through LDS, 64 rows at a time (coalesced float4 loads
    // PD chunks ahead, two staging buffers, one barrier per chunk)
    float a[RPL][CPW];
    float4 pre[RPL][PF];
    auto load = [&](int s) {
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int e = tid + NT * q, rr = e / (LP / 4), c4 = e % (LP / 4);
        const int g = s_gidx[64 * s + rr];
        pre[s][q] = (g >= 0) ? *reinterpret_cast<const float4*>(X + (int64_t)g * ldx + 4 * c4)
                             : make_float4(0.f, 0.f, 0.f, 0.f);
      }
    };
#pragma unroll
    for (int s = 0; s < PD && s < RPL; ++s) load(s);
#pragma unroll
    for (int s = 0; s < RPL; ++s) {
      float* st = s_big + (s & 1) * 64 * SROW;
#pragma unroll
      for (int q = 0; q < PF; ++q) {
        const int e = tid + NT * q, rr = e / (LP / 4), c = 4 * (e % (LP / 4));
        st[rr * SROW + c] = pre[s][q].x;
        st[rr * SROW + c + 1] = pre[s][q].y;
        st[rr * SROW + c + 2] = pre[s][q].z;
        st[rr * SROW + c + 3] = pre[s][q].w;
      }
      if (s + PD < RPL) load(s + PD);
      __syncthreads();
#pragma unroll
      for (int t = 0; t < CPW; ++t) a[s][t] = st[lane * SROW + w + NW * t];
    }
    const bool root = (lv.nblk[level] == 1);
    __syncthreads();  // staging reads are done before U overwrites it
    if (root)
      for (int e = tid; e < LP * LP; e += NT) s_big[e] = 0.f;
    __syncthreads();
    Gepp<LP, R, NT>::run(a, valid, l, s_lr, s_mult, s_key, root ? s_big : nullptr);
    int pg = -1;  // global index of pivot tid
    if (tid < l && s_lr[tid] >= 0) pg = s_gidx[s_lr[tid]];
    if (root) {
      if (tid < LP) piv[tid] = pg;
      for (int e = tid; e < LP * LP; e += NT) U[e] = s_big[e];
      return;
    }
    if (tid < LP) cand[lv.cand_off[level] + blk * LP + tid] = pg;
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

// rows per block (512 threads each): the requested count when the kernel
// has that instantiation, else 512; at least 2 lp
static int lu_block_rows(int lp, int want) {
  int r = 512;
  if (want == 256 || want == 512 || (want == 1024 && lp <= 64)) r = want;
  if (r < 2 * lp) r = 2 * lp;
  return r;
}

LuPlan plan_lu(int64_t rows, int lp, int block_rows) {
  LuPlan p{};
  p.lp = lp;
  const int NT = lu_block_rows(lp, block_rows);
  p.rows = NT;
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
  const int r = plan.rows;
#define LU_LAUNCH(LP_, R_)                                                                    \
  hipLaunchKernelGGL((lu_tree_kernel<LP_, R_, 512>), grid, dim3(512), 0, st, X, ldx, rows, l, \
                     lv, cand, counters, U, piv)
  if (plan.lp == 32) {
    if (r == 1024) LU_LAUNCH(32, 1024);
    else if (r == 512) LU_LAUNCH(32, 512);
    else LU_LAUNCH(32, 256);
  } else if (plan.lp == 64) {
    if (r == 1024) LU_LAUNCH(64, 1024);
    else if (r == 512) LU_LAUNCH(64, 512);
    else LU_LAUNCH(64, 256);
  } else if (plan.lp == 128) {
    if (r == 256) LU_LAUNCH(128, 256);
    else LU_LAUNCH(128, 512);
  }
#undef LU_LAUNCH
}

}  // namespace rpca
