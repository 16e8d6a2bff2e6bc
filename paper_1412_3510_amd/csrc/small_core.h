// Single-workgroup float64 building blocks shared by the small-matrix kernels
// and the persistent batched solver: Newton-refined reciprocal and square
// root, the register-blocked Cholesky factorization, and the one-sided Jacobi
// SVD.
#pragma once
#include "common.h"

namespace rpca {

// state[] layout (int):
//   0  the current orthonormalization shifted a Cholesky factorization
//   1  extra passes 3 and 4 are needed
//   2  dependent columns were replaced by random ones
//   5  non-finite values met (this orthonormalization)
//   6, 7  Jacobi SVD flags
//   8..11  bit mask of dependent columns (128 bits)
// Slots 0 .. 11 belong to one orthonormalization (its first pass clears
// them); slots 12 .. 15 belong to the whole solve (cleared when it starts):
//   12 Nystrom shift retries, 13 Nystrom: no positive definite shifted B2
//   found, 14 non-finite values met in any step, 15 a batched problem split
//   over several workgroups gave up waiting for the others (bounded wait).
static constexpr int kStRetries = 12;
static constexpr int kStNotPsd = 13;
static constexpr int kStNonFinite = 14;
static constexpr int kStTeam = 15;
// bits of a solve's status word (and of each batch problem's entry)
static constexpr int kErrNotPsd = 1;
static constexpr int kErrNonFinite = 2;
static constexpr int kErrTimeout = 4;
static constexpr double kTauRel = 1e-10;   // relative Cholesky pivot that marks dependence
static constexpr double kShiftRel = 1e-8;  // relative diagonal shift when dependence is met
static constexpr double kJunkNorm2 = 1e-2; // squared column norm after a shifted pass

// Cholesky G + shift = R^T R (R upper) of the leading l x l block by one
// workgroup of NTH threads (1024 unless given).  Thread (g, c) -- g = tid / LP,
// c = tid % LP -- keeps the entries (i, c) of the RPT = LP RG / NTH
// consecutive rows i = g RPT + q (RG = NTH / LP row groups) in registers.
// Step j: every thread reads the current row u = G[j][.] from a
// double-buffered LDS row (published by its owners at the end of step j - 1;
// zero at the columns already factored) and the pivot d = u[j]; row j of R,
// u[c] / sqrt(d), goes to the LDS factor Rs (float32, row-major stride LP);
// every entry takes G[i][c] -= u[i] u[c] / d (its rows' u[i] read as 16-byte
// pairs); the owners of row j + 1 publish it; one barrier.  1/sqrt(d) is
// v_rsq_f64 refined by two Newton steps, which keeps division and square
// root off the step's critical path.  Nothing in the loop touches global
// memory, so the barrier waits for LDS only.
// Returns false at the first pivot d <= tau * diag[j] (or not finite): all
// threads read the same d, so all agree.
static constexpr int kCholThreads = 1024;  // default workgroup size of chol_par

__device__ __forceinline__ double rsqrt_nr(double d) {
  double y = __builtin_amdgcn_rsq(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d * y, y, 1.0);
    y = fma(0.5 * y, e, y);
  }
  return y;
}

__device__ __forceinline__ double rcp_nr(double d) {
  double y = __builtin_amdgcn_rcp(d);
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-d, y, 1.0);
    y = fma(y, e, y);
  }
  return y;
}

template <int LP, int NTH = kCholThreads>
__device__ bool chol_par(const double* __restrict__ G, bool sym, int l, double srel, double sabs,
                         const double* diag, double tau, float* Rs, double* ubuf) {
  constexpr int RG = NTH / LP;   // row groups
  constexpr int RPT = LP / RG;   // rows per thread, contiguous: i = g RPT + q
  const int tid = threadIdx.x, g = tid / LP, c = tid % LP;
  double v[RPT];
#pragma unroll
  for (int q = 0; q < RPT; ++q) {
    const int i = g * RPT + q;
    double x = 0.0;
    if (i < l && c < l) x = sym ? 0.5 * (G[i * LP + c] + G[c * LP + i]) : G[i * LP + c];
    if (i == c && c < l) x += srel * diag[c] + sabs;
    v[q] = x;
  }
  if (g == 0) ubuf[c] = (c < l) ? v[0] : 0.0;  // row 0
  __syncthreads();
  for (int j = 0; j < l; ++j) {
    const double* u = ubuf + (j & 1) * LP;
    const double d = u[j];
    if (!(d > tau * diag[j]) || !(d > 0.0) || !(d < 1e300)) return false;
    const double uc = u[c];
    const double y = rsqrt_nr(d);
    const double f = uc * (y * y);
    if (g == 0) Rs[j * LP + c] = (c < l && c >= j) ? (float)((c == j) ? d * y : uc * y) : 0.f;
    // every entry is updated: the published row is zero at the finished
    // positions (c <= j), so rows above j and the lower triangle (never
    // published) take harmless updates, and no lane is masked
    double ui[RPT];
    if constexpr (RPT % 2 == 0) {  // (ubuf is 16-byte aligned)
#pragma unroll
      for (int q = 0; q < RPT; q += 2) {
        const double2 t = *reinterpret_cast<const double2*>(u + g * RPT + q);
        ui[q] = t.x;
        ui[q + 1] = t.y;
      }
    } else {
#pragma unroll
      for (int q = 0; q < RPT; ++q) ui[q] = u[g * RPT + q];
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) v[q] = fma(-ui[q], f, v[q]);
    const int jn = j + 1;
    if (g == jn / RPT) {  // the owners of row j + 1 publish it
      const int oq = jn % RPT;
      double nxt = 0.0;
#pragma unroll
      for (int q = 0; q < RPT; ++q) nxt = (q == oq) ? v[q] : nxt;
      ubuf[(jn & 1) * LP + c] = (c > j && c < l) ? nxt : 0.0;
    }
    __syncthreads();
  }
  return true;
}

// ------------------------------------------------------------------------
// One-sided (Hestenes) Jacobi SVD of M (or M^T), l <= LP, in float64.
// Columns are stored contiguously in LDS (Mc[j*CS + i] = column j, row i,
// CS = LP + 2 so columns of different pairs fall in different banks).
// Column pairs follow the round-robin (circle) ordering, lp2/2 disjoint
// pairs per round; each pair is handled by G = 16 lanes (one row block of
// RPT = LP/G consecutive rows each), whose partial inner products are
// combined with DPP lane permutations.  With M Wacc = Xn diag(s):
//   s    -- column norms, sorted descending
//   Wacc -- accumulated rotations (orthogonal), columns in the same order
//   Xn   -- normalized columns of M Wacc (zero where s = 0)
// For M = R (B^T = Q2 R) the left singular vectors of B are Wacc and the
// right ones Q2 Xn; for M = R^T (F = QF R) the left ones of F are QF Wacc.
// ------------------------------------------------------------------------
__device__ __forceinline__ double dpp_f64(double v, int ctrl_sel) {
  // ctrl_sel: 0 = quad_perm [1,0,3,2], 1 = quad_perm [2,3,0,1], 2 = row_half_mirror
  // every lane reads a valid source lane (full row and bank masks), so the
  // moves need no fill value
  int lo = __double2loint(v), hi = __double2hiint(v);
  int lo2, hi2;
  if (ctrl_sel == 0) {
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0xB1, 0xF, 0xF, false);
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0xB1, 0xF, 0xF, false);
  } else if (ctrl_sel == 1) {
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0x4E, 0xF, 0xF, false);
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0x4E, 0xF, 0xF, false);
  } else if (ctrl_sel == 2) {
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0x141, 0xF, 0xF, false);
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0x141, 0xF, 0xF, false);
  } else {  // row_mirror
    lo2 = __builtin_amdgcn_mov_dpp(lo, 0x140, 0xF, 0xF, false);
    hi2 = __builtin_amdgcn_mov_dpp(hi, 0x140, 0xF, 0xF, false);
  }
  return __hiloint2double(hi2, lo2);
}

// sum over the G (4, 8 or 16) aligned lanes of a group (all G get the sum)
template <int G>
__device__ __forceinline__ double sum_group(double v) {
  static_assert(G == 4 || G == 8 || G == 16, "sum_group: G must be 4, 8 or 16");
  v += dpp_f64(v, 0);
  v += dpp_f64(v, 1);
  if constexpr (G >= 8) v += dpp_f64(v, 2);
  if constexpr (G == 16) v += dpp_f64(v, 3);
  return v;
}

// The workgroup runs jacobi_body with at least NT = G LP / 2 threads (extra
// threads only join the barriers).  Mc and Vc hold LP * CS doubles each
// (CS = LP + 2 in LDS; LP in global memory for GLOBAL), sig LP doubles, perm
// LP ints; s_rot and s_big are two LDS ints.
template <int LP, bool GLOBAL>
constexpr int jacobi_cs() { return GLOBAL ? LP : LP + 2; }

// ACC = false: the rotations are not accumulated (Vc is not used).  With M0
// the starting matrix and M0 = X diag(s) W^T, the rotations are then
// recovered as W = M0^T X diag(s)^-1, column j from M0^T (M0 W)_j / s_j^2.
// The rounding of that product grows like c eps (s_1 / s_j)^2, with c about
// the square root of the rotations a column takes part in (~30: the rounding
// they leave in M0 W), so it is used only when the kneed largest s_j are all
// >= kJacobiRecover s_1, which keeps those columns of W within about 3e-7 of
// orthonormal, below the rounding of the float32 factors they multiply (the
// callers read only the first kneed columns of W); otherwise *flag is set to
// 1 (0 when the outputs are good) and the caller runs the accumulating form.
static constexpr double kJacobiRecover = 1e-4;

template <int LP, bool GLOBAL, int G, bool ACC = true>
__device__ __forceinline__ void jacobi_body(const double* __restrict__ M, int l, int transpose,
                                            double* __restrict__ s_out,
                                            double* __restrict__ Wacc, double* __restrict__ Xn,
                                            double* Mc, double* Vc, double* sig, int* perm,
                                            int& s_rot, int& s_big, int* flag = nullptr,
                                            int kneed = 0, int* sweeps_out = nullptr,
                                            double quiet = 1e-6) {
  constexpr int CS = jacobi_cs<LP, GLOBAL>();
  constexpr int RPT = LP / G;     // rows per lane
  constexpr int NT = G * LP / 2;  // G lanes for each of the LP/2 pair slots
  const int tid = threadIdx.x;
  for (int e = tid; tid < NT && e < LP * LP; e += NT) {
    const int j = e / LP, i = e % LP;
    double v = 0.0;
    if (i < l && j < l) v = transpose ? M[j * LP + i] : M[i * LP + j];
    Mc[j * CS + i] = v;
    if constexpr (ACC) Vc[j * CS + i] = (i == j) ? 1.0 : 0.0;
  }
  const int lp2 = l + (l & 1);
  const int npairs = lp2 / 2;
  const int k = tid / G, gl = tid % G;  // pair slot, lane in the group of G
  const bool active = (k < npairs);
  // rows of a lane: pairs (2 gl, 2 gl + 1) + 2 G v, v < RPT / 2, so that the
  // G lanes of a pair read consecutive 16-byte words (no LDS bank conflicts)
  const int i0 = 2 * gl;
  const double tol = 1e-13;
  // cyclic Jacobi converges quadratically: a sweep that starts with every
  // |cos of the pair angle| <= 1e-6 leaves them near 1e-12 or below, which
  // puts the column norms (the singular values) within about 1e-16 relative
  // and the accumulated rotations within about 1e-12 of the converged ones;
  // the sweeps after it only confirm that, and are skipped
  // round-robin pairs: slot k starts with (k, lp2 - 1 - k); every index but 0
  // advances by one per round, cyclically through 1 .. lp2 - 1
  const int P = lp2 - 1;
  int sweep = 0;
  for (; sweep < 60; ++sweep) {
    __syncthreads();
    if (tid == 0) {
      s_rot = 0;
      s_big = 0;
    }
    __syncthreads();
    int p = active ? k : 0, q = active ? P - k : 0;
    for (int r = 0; r < P; ++r, p = (p == 0) ? 0 : (p == P ? 1 : p + 1),
             q = (q == 0) ? 0 : (q == P ? 1 : q + 1)) {
      const bool go = active && p < l && q < l;
      double mp[RPT], mq[RPT];
      double al = 0.0, be = 0.0, ga = 0.0;
      if (go) {
#pragma unroll
        for (int u = 0; u < RPT; u += 2) {
          const double2 x = *reinterpret_cast<const double2*>(Mc + p * CS + i0 + u * G);
          const double2 y = *reinterpret_cast<const double2*>(Mc + q * CS + i0 + u * G);
          mp[u] = x.x; mp[u + 1] = x.y;
          mq[u] = y.x; mq[u + 1] = y.y;
        }
#pragma unroll
        for (int u = 0; u < RPT; ++u) {
          al += mp[u] * mp[u];
          be += mq[u] * mq[u];
          ga += mp[u] * mq[u];
        }
      }
      al = sum_group<G>(al);
      be = sum_group<G>(be);
      ga = sum_group<G>(ga);
      if (go && al > 0.0 && be > 0.0 && ga * ga > (quiet * quiet) * (al * be) && gl == 0)
        s_big = 1;
      if (go && al > 0.0 && be > 0.0 && ga * ga > (tol * tol) * (al * be)) {
        // Rutishauser's rotation, t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2))
        // with zeta = (be - al) / (2 ga), evaluated as
        // t = 2 ga sign(d) / (|d| + sqrt(d^2 + 4 ga^2)), d = be - al.  t needs
        // only the hardware reciprocal and square-root approximations (about
        // 22 bits: the rotation then removes all but ~1e-6 of ga, and the
        // next sweep the rest); c = 1/sqrt(1 + t^2) is refined by Newton
        // steps, so (c, s = c t) is orthogonal to rounding whatever t is and
        // the column norms are preserved
        const double d = be - al;
        double t;
        if (fabs(d) < 1e150 && fabs(ga) < 1e150) {
          const double h2 = fma(d, d, 4.0 * ga * ga);
          const double h = h2 * __builtin_amdgcn_rsq(h2);
          // sign(zeta) = sign(d) sign(ga), with d = +0 counting as positive
          t = copysign(2.0 * fabs(ga) * __builtin_amdgcn_rcp(fabs(d) + h), d >= 0.0 ? ga : -ga);
        } else {  // huge entries: the zeta form, which cannot overflow in h2
          const double zeta = d * (0.5 * rcp_nr(ga));
          t = (fabs(zeta) < 1e150)
                  ? copysign(rcp_nr(fabs(zeta) + fma(zeta, zeta, 1.0) * rsqrt_nr(fma(zeta, zeta, 1.0))), zeta)
                  : 0.5 * rcp_nr(zeta);
        }
        const double c = rsqrt_nr(fma(t, t, 1.0)), s = c * t;
#pragma unroll
        for (int u = 0; u < RPT; u += 2) {
          *reinterpret_cast<double2*>(Mc + p * CS + i0 + u * G) =
              make_double2(c * mp[u] - s * mq[u], c * mp[u + 1] - s * mq[u + 1]);
          *reinterpret_cast<double2*>(Mc + q * CS + i0 + u * G) =
              make_double2(s * mp[u] + c * mq[u], s * mp[u + 1] + c * mq[u + 1]);
          if constexpr (ACC) {
            const double2 vp = *reinterpret_cast<const double2*>(Vc + p * CS + i0 + u * G);
            const double2 vq = *reinterpret_cast<const double2*>(Vc + q * CS + i0 + u * G);
            *reinterpret_cast<double2*>(Vc + p * CS + i0 + u * G) =
                make_double2(c * vp.x - s * vq.x, c * vp.y - s * vq.y);
            *reinterpret_cast<double2*>(Vc + q * CS + i0 + u * G) =
                make_double2(s * vp.x + c * vq.x, s * vp.y + c * vq.y);
          }
        }
        if (gl == 0) s_rot = 1;
      }
      __syncthreads();
    }
    if (s_rot == 0 || s_big == 0) break;
  }
  if (sweeps_out && tid == 0) *sweeps_out = sweep;
  __syncthreads();
  if (tid < LP) {
    double s = 0.0;
    if (tid < l)
      for (int i = 0; i < l; ++i) s += Mc[tid * CS + i] * Mc[tid * CS + i];
    sig[tid] = sqrt(s);
  }
  __syncthreads();
  if (tid < l) {
    int rank = 0;
    for (int i = 0; i < l; ++i)
      if (sig[i] > sig[tid] || (sig[i] == sig[tid] && i < tid)) ++rank;
    perm[rank] = tid;
  }
  __syncthreads();
  if constexpr (!ACC) {
    if (tid == 0) {
      const int kk = (kneed > 0 && kneed < l) ? kneed : l;
      const double smax = sig[perm[0]], smin = sig[perm[kk - 1]];
      *flag = (smin >= kJacobiRecover * smax && smax < 1e300) ? 0 : 1;
    }
  }
  for (int e = tid; tid < NT && e < LP * LP; e += NT) {
    const int i = e / LP, rr = e % LP;  // output row i, column rr
    double w = 0.0, x = 0.0;
    if (i < l && rr < l) {
      const int j = perm[rr];
      if constexpr (ACC) {
        w = Vc[j * CS + i];
      } else {  // W[i][rr] = sum_t M0[t][i] (M0 W)[t][j] / s_j^2
        double acc = 0.0;
        for (int t = 0; t < l; ++t)
          acc += (transpose ? M[i * LP + t] : M[t * LP + i]) * Mc[j * CS + t];
        w = (sig[j] > 0.0) ? acc / (sig[j] * sig[j]) : 0.0;
      }
      x = (sig[j] > 0.0) ? Mc[j * CS + i] / sig[j] : 0.0;
    }
    Wacc[e] = w;
    Xn[e] = x;
  }
  if (tid < LP) s_out[tid] = (tid < l) ? sig[perm[tid]] : 0.0;
}

}  // namespace rpca
