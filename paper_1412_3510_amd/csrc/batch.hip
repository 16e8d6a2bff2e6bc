// Persistent batched solver: many small problems in one launch.
//
// A workgroup of 512 threads (8 waves) solves one whole problem at a time --
// the randomized SVD of Section 2 with the renormalized power iteration of
// Section 5 (optionally on the column-centered A), or the shifted Nystrom
// method of Section 3 for a PSD A -- with the workgroup-collective routines
// below, and then takes the next problem from a device counter until the
// list is exhausted.  The host orders the list by decreasing cost, so the
// largest problems start first and the small ones fill in behind them.  No
// workgroup ever waits for another, so the launch always drains.
//
// Per problem the steps are the ones of the multi-kernel path, restated for
// one workgroup:
//   * Omega from Philox4x32-10 (the same values as the single solve);
//   * Y = A X and Z = A^T X on MFMA (v_mfma_f32_32x32x16_bf16, float32
//     operands split into bfloat16 pairs, three products per tile): each wave
//     owns 32 rows of the output tile (32 columns of A for A^T X).  For A X a
//     wave reads its rows as whole 256-byte segments (lanes along k) and turns
//     them into the MFMA layout through its own LDS tile; for A^T X each half
//     wave reads 32 consecutive entries of a row.  A is read one chunk ahead
//     of the products, and the packed small operand is staged through a
//     two-buffer LDS ring shared by the 8 waves;
//   * centering (Section 2: A_c = A - 1 mu): Y minus its column means after
//     A X; the m-side operand minus its column means before A^T X;
//   * LU renormalization (Section 5): a right-looking partial-pivoting LU,
//     blocked by 8 columns, without physical row swaps.  Every thread keeps
//     16 rows of the 8-column panel in registers; a step finds the pivot with
//     one DPP wave argmax and one barrier (the winning lane of each wave
//     publishes its row), scales the multipliers and updates the panel; the
//     trailing columns get one rank-8 update per panel (whole rows).  The
//     result P L (rows in the original order) overwrites Y; a zero pivot
//     leaves the unit vector of its pivot row as that column of L;
//   * orthonormalization: Cholesky QR twice with a float64 Gram matrix (up to
//     four passes with a shifted factorization and completion of dependent
//     columns, exactly as in the multi-kernel path);
//   * the Rayleigh-Ritz step: B^T = A_c^T Q = Q2 R, the one-sided Jacobi SVD
//     of R^T (shared with the single-problem kernel), U = Q X, V = Q2 W;
//   * Nystrom: B1 = A Q, nu = sqrt(n) 2^-24 ||B1||_F, Cholesky of
//     Q^T B1 + nu I (nu times 10 while it fails), F = (B1 + nu Q) C^-1, its
//     SVD through Cholesky QR and Jacobi, lambda = max(s^2 - nu, 0);
//   * the sign convention: the largest-magnitude entry of each column of U
//     positive (ties to the smaller row), V's column follows.
// Results agree with the single solve up to rounding (the renormalizations
// choose other but equivalent bases; the final factors do not depend on
// them in exact arithmetic).
//
// Limits (checked by the host): float32 A, row-major, lda >= n; m, n <=
// 8192; l <= 64.  Working memory: one slot per workgroup (see pers_slot_floats).
#include "common.h"
#include "kernels.h"
#include "philox.h"
#include "small_core.h"

namespace rpca {

namespace {

// Pointers passed into the (non-inlined) routines are generic; the routines
// re-qualify them as global so that their accesses are global_* rather than
// flat_* instructions (flat accesses also count against the LDS wait
// counter, which would serialize the LDS reads with the A loads in flight).
#define GAS __attribute__((address_space(1)))
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));
template <class T>
__device__ __forceinline__ GAS T* as_global(T* p) { return (GAS T*)p; }

// Arguments of the routines are the same in every lane; reading them from the
// first lane puts them in scalar registers (uniform branches and addresses).
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni(int64_t v) {
  const int lo = __builtin_amdgcn_readfirstlane((int)(uint64_t)v);
  const int hi = __builtin_amdgcn_readfirstlane((int)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)(unsigned)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ uint64_t uni(uint64_t v) { return (uint64_t)uni((int64_t)v); }
template <class T>
__device__ __forceinline__ T* uni(T* p) { return (T*)(uintptr_t)uni((int64_t)(uintptr_t)p); }

constexpr int NT = 512;                  // threads per workgroup
constexpr int NWAVE = NT / 64;           // waves per workgroup
constexpr int RPT = kPersMaxDim / NT;    // rows per thread in the LU (16)
constexpr int PB = 8;                    // LU panel width

// LDS of one workgroup.  The union holds the buffers of one step at a time.
struct PLds {
  union {
    u32x4 xs[2][4 * 2 * 2 * 64];  // A-pass operand ring: 2 x (4 steps x 2 blocks x hi/lo x 64 lanes)
    double gr[4096];              // Gram: row slices, then the group partials
    struct {
      double M[64 * 66];
      double V[64 * 66];
      double sig[64];
      int perm[64];
      int rot, big;
    } jac;
    struct {
      float key[2][NWAVE];
      int kidx[2][NWAVE];
      float row[2][NWAVE][PB];
      float U12[PB][64] __attribute__((aligned(16)));
      int piv[64];
    } lu;
    struct {
      float R[64 * 64];   // float32 factor (row-major), written by the Cholesky
      float Rt[64 * 64];  // its transpose (column j contiguous)
      float rd[64];       // reciprocals of the diagonal (0 for a zero pivot)
    } tri;
    double red[16 * 64];
    unsigned long long kred[NWAVE * 64];
    float W[64 * 64];
  } u;
  float at[NWAVE][32 * 68] __attribute__((aligned(16)));  // A-pass row tiles (pitch 68)
  double ubuf[2 * 64] __attribute__((aligned(16)));
  double diag[64];
  double zero[64];
  float mu[64];
  float sgn[64];
  int state[16];
  int idx;
};

__shared__ PLds g_S;

// Working memory of one problem, carved from the workgroup's slot.
struct Buf {
  float* Y;     // R x 64
  float* Z;     // R x 64
  float* T;     // R x 64
  __bf16* P;    // packed operand, R x 64 x 2 bf16
  double* G;    // 64 x 64
  double* Wacc; // 64 x 64
  double* Xn;   // 64 x 64
  double* sv;   // 64
};

__device__ __forceinline__ Buf carve(float* slot, int64_t R) {
  Buf b;
  b.Y = slot;
  b.Z = slot + R * 64;
  b.T = slot + 2 * R * 64;
  b.P = reinterpret_cast<__bf16*>(slot + 3 * R * 64);
  double* d = reinterpret_cast<double*>(slot + 4 * R * 64);
  b.G = d;
  b.Wacc = d + 4096;
  b.Xn = d + 2 * 4096;
  b.sv = d + 3 * 4096;
  return b;
}

__device__ __forceinline__ f32x16 mfma3s(const bf16x8& ah, const bf16x8& al, const bf16x8& bh,
                                         const bf16x8& bl, f32x16 acc) {
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al, bh, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bl, acc, 0, 0, 0);
  acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah, bh, acc, 0, 0, 0);
  return acc;
}

__device__ __forceinline__ void split8(const float (&a)[8], bf16x8& hi, bf16x8& lo) {
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    __bf16 h, l;
    split_bf16(a[j], h, l);
    hi[j] = h;
    lo[j] = l;
  }
}

// |v| in the high word (larger wins), the complement of the index in the low
// word (ties go to the smaller index); never 0 for a valid index.
__device__ __forceinline__ unsigned long long abs_key(float v, int i) {
  return ((unsigned long long)(__float_as_uint(v) & 0x7fffffffu) << 32) | (unsigned)(~(unsigned)i);
}

// ---- Omega: X (n x LP), X[i][c] = Omega[i][c] for c < l, 0 beyond ------------
// (rows r0 .. r1 - 1 only: a workgroup of a team writes its own rows)
template <int LP>
__device__ __attribute__((noinline)) void p_omega(uint64_t seed, int n, int l, float* X_,
                                                  int uniform, int r0, int r1) {
  seed = uni(seed);
  n = uni(n);
  l = uni(l);
  uniform = uni(uniform);
  r0 = uni(r0);
  r1 = uni(r1);
  auto X = as_global(uni(X_));
  const int tid = threadIdx.x;
  for (int e = r0 * LP + tid; e < r1 * LP; e += NT)
    if ((e % LP) >= l) X[e] = 0.f;
  // element e = 4 t + q of the stream is Omega[e % n][e / n]
  const int64_t total = (int64_t)n * l, nb = (total + 3) / 4;
  for (int64_t t = tid; t < nb; t += NT) {
    uint32_t c[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u, 0u};
    philox_block(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    float z[4];
    if (uniform) {
#pragma unroll
      for (int q = 0; q < 4; ++q) z[q] = word_uniform(c[q]);
    } else {
      box_muller(c[0], c[1], z[0], z[1]);
      box_muller(c[2], c[3], z[2], z[3]);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int64_t e = 4 * t + q;
      if (e < total) {
        const int64_t j = e / n, i = e - j * n;
        if (i >= r0 && i < r1) X[i * LP + j] = z[q];
      }
    }
  }
  __syncthreads();
}

// ---- packed operand: src (rows x LP) minus mu -> bfloat16 (hi, lo) fragments,
// rows padded with zeros to a multiple of 64.  Fragment (s, cb, h) holds, for
// lane L = c + 32 g, the entries (16 s + 8 g + j, 32 cb + c), j = 0..7.
template <int LP>
__device__ __attribute__((noinline)) void p_pack(const float* src_, int rows, int l, bool use_mu, __bf16* out_) {
  rows = uni(rows);
  l = uni(l);
  auto src = as_global(uni(src_));
  auto out = as_global(uni(out_));
  constexpr int NB = LP / 32;
  const int nsteps = ((rows + 63) / 64) * 4;
  const int total = nsteps * NB * 64;
  GAS bf16x8* o = reinterpret_cast<GAS bf16x8*>(out);
  for (int t = threadIdx.x; t < total; t += NT) {
    const int L = t & 63, rest = t >> 6;
    const int cb = rest % NB, s = rest / NB;
    const int c = 32 * cb + (L & 31), g = L >> 5;
    const float m = (use_mu && c < l) ? g_S.mu[c] : 0.f;
    float a[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int r = 16 * s + 8 * g + j;
      a[j] = (r < rows && c < l) ? src[(int64_t)r * LP + c] - m : 0.f;
    }
    bf16x8 hi, lo;
    split8(a, hi, lo);
    o[((s * NB + cb) * 2) * 64 + L] = hi;
    o[((s * NB + cb) * 2 + 1) * 64 + L] = lo;
  }
  __syncthreads();
}

// Chunk ch (4 steps) of the packed operand: loaded into registers one chunk
// ahead, written to ring buffer buf after the current chunk's products.
template <int LP>
struct Stage {
  static constexpr int CH = 4 * (LP / 32) * 2 * 64;  // 16-byte pieces per chunk
  static constexpr int PER = CH / NT;                 // per thread (1 or 2)
  u32x4 v[PER];
  __device__ __forceinline__ void load(const GAS __bf16* Pk, int ch) {
    const GAS u32x4* src = reinterpret_cast<const GAS u32x4*>(Pk) + (int64_t)ch * CH;
#pragma unroll
    for (int i = 0; i < PER; ++i) v[i] = src[threadIdx.x + NT * i];
  }
  __device__ __forceinline__ void store(int buf) {
#pragma unroll
    for (int i = 0; i < PER; ++i) g_S.u.xs[buf][threadIdx.x + NT * i] = v[i];
  }
};

// ---- Y (m x LP) = A X, X packed (n side, >= ceil(n/64)*4 steps) -----------
template <int LP>
__device__ __attribute__((noinline)) void p_ax(const float* __restrict__ A_, int64_t lda, int m, int n, const __bf16* Xp_,
                     float* Y_) {
  lda = uni(lda);
  m = uni(m);
  n = uni(n);
  auto A = as_global(uni(A_));
  auto Xp = as_global(uni(Xp_));
  auto Y = as_global(uni(Y_));
  PLds& S = g_S;
  constexpr int NB = LP / 32;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, c = lane & 31, g = lane >> 5;
  const int nchunk = (n + 63) / 64;
  constexpr int AP = 68;  // pitch of the per-wave LDS tile (floats)
  float* tile = S.at[wave];
  for (int r0 = 0; r0 < m; r0 += 32 * NWAVE) {
    const int rbase = r0 + 32 * wave;
    const bool live = rbase < m;
    f32x16 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
    // A arrives row by row with the lanes along k (each load is one 256-byte
    // segment of a row), one chunk ahead, and is turned into the MFMA layout
    // through the wave's LDS tile; rows past m and columns past n read the
    // last row or column and are zeroed on the way into the tile
    float v[32];
    auto load_a = [&](int ch) {
      const int col = min(64 * ch + lane, n - 1);
#pragma unroll
      for (int r = 0; r < 32; ++r) {
        const int rr = min(rbase + r, m - 1);
        v[r] = A[(int64_t)rr * lda + col];
      }
    };
    auto put_a = [&](int ch) {
      if (64 * ch + 64 <= n && rbase + 32 <= m) {  // an interior chunk: no masking
#pragma unroll
        for (int r = 0; r < 32; ++r) tile[r * AP + lane] = v[r];
      } else {
        const bool colok = 64 * ch + lane < n;
#pragma unroll
        for (int r = 0; r < 32; ++r) tile[r * AP + lane] = (colok && rbase + r < m) ? v[r] : 0.f;
      }
    };
    Stage<LP> stg;
    stg.load(Xp, 0);
    stg.store(0);
    if (nchunk > 1) stg.load(Xp, 1);
    if (live) {
      load_a(0);
      put_a(0);
      if (nchunk > 1) load_a(1);
    }
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
      const int buf = ch & 1;
      if (live) {
        bf16x8 ah[4], al[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          float a8[8];
          const f32x4 t0 = *reinterpret_cast<const f32x4*>(tile + c * AP + 16 * s + 8 * g);
          const f32x4 t1 = *reinterpret_cast<const f32x4*>(tile + c * AP + 16 * s + 8 * g + 4);
          a8[0] = t0.x; a8[1] = t0.y; a8[2] = t0.z; a8[3] = t0.w;
          a8[4] = t1.x; a8[5] = t1.y; a8[6] = t1.z; a8[7] = t1.w;
          split8(a8, ah[s], al[s]);
        }
        if (ch + 1 < nchunk) {  // the next chunk into the tile (after this one's reads), and one more ahead
          put_a(ch + 1);
          if (ch + 2 < nchunk) load_a(ch + 2);
        }
        const bf16x8* xs = reinterpret_cast<const bf16x8*>(S.u.xs[buf]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) {
            const bf16x8 xh = xs[((s * NB + cb) * 2) * 64 + lane];
            const bf16x8 xl = xs[((s * NB + cb) * 2 + 1) * 64 + lane];
            acc[cb] = mfma3s(ah[s], al[s], xh, xl, acc[cb]);
          }
      }
      if (ch + 1 < nchunk) {  // chunk ch + 1 into the other buffer, chunk ch + 2 into registers
        stg.store(buf ^ 1);
        if (ch + 2 < nchunk) stg.load(Xp, ch + 2);
      }
      __syncthreads();
    }
    if (live) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int ro = rbase + (r & 3) + 4 * g + 8 * (r >> 2);
          if (ro < m) Y[(int64_t)ro * LP + 32 * cb + c] = acc[cb][r];
        }
    }
  }
  __syncthreads();
}

// ---- Z (n x LP) = A^T Q, Q packed (m side, >= ceil(m/64)*4 steps) ---------
template <int LP>
__device__ __attribute__((noinline)) void p_atx(const float* __restrict__ A_, int64_t lda, int m, int n, const __bf16* Qp_,
                      float* Z_) {
  lda = uni(lda);
  m = uni(m);
  n = uni(n);
  auto A = as_global(uni(A_));
  auto Qp = as_global(uni(Qp_));
  auto Z = as_global(uni(Z_));
  PLds& S = g_S;
  constexpr int NB = LP / 32;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, c = lane & 31, g = lane >> 5;
  const int nchunk = (m + 63) / 64;
  for (int j0 = 0; j0 < n; j0 += 32 * NWAVE) {
    const int cbase = j0 + 32 * wave;
    const bool live = cbase < n;
    const int col = cbase + c;
    const bool cok = col < n;
    const GAS float* acol = A + (cok ? col : 0);
    f32x16 acc[NB];
#pragma unroll
    for (int i = 0; i < NB; ++i)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[i][r] = 0.f;
    // raw loads (clamped rows) one chunk ahead, masked when split
    float a[4][8];
    auto load_a = [&](int ch) {
      if (64 * ch + 64 <= m) {  // every row of the chunk exists: offsets from one base
        const GAS float* p0 = acol + (int64_t)(64 * ch + 8 * g) * lda;
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int j = 0; j < 8; ++j) a[s][j] = p0[(int64_t)(16 * s + j) * lda];
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int j = 0; j < 8; ++j)
            a[s][j] = acol[(int64_t)min(64 * ch + 16 * s + 8 * g + j, m - 1) * lda];
      }
    };
    auto mask_a = [&](int ch) {
      if (64 * ch + 64 <= m && cbase + 32 <= n) return;  // an interior chunk
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          if (!(cok && 64 * ch + 16 * s + 8 * g + j < m)) a[s][j] = 0.f;
    };
    Stage<LP> stg;
    stg.load(Qp, 0);
    stg.store(0);
    if (nchunk > 1) stg.load(Qp, 1);
    if (live) load_a(0);
    __syncthreads();
    for (int ch = 0; ch < nchunk; ++ch) {
      const int buf = ch & 1;
      if (live) {
        bf16x8 ah[4], al[4];
        mask_a(ch);
#pragma unroll
        for (int s = 0; s < 4; ++s) split8(a[s], ah[s], al[s]);
        if (ch + 1 < nchunk) load_a(ch + 1);
        const bf16x8* xs = reinterpret_cast<const bf16x8*>(S.u.xs[buf]);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
          for (int cb = 0; cb < NB; ++cb) {
            const bf16x8 xh = xs[((s * NB + cb) * 2) * 64 + lane];
            const bf16x8 xl = xs[((s * NB + cb) * 2 + 1) * 64 + lane];
            acc[cb] = mfma3s(ah[s], al[s], xh, xl, acc[cb]);
          }
      }
      if (ch + 1 < nchunk) {  // chunk ch + 1 into the other buffer, chunk ch + 2 into registers
        stg.store(buf ^ 1);
        if (ch + 2 < nchunk) stg.load(Qp, ch + 2);
      }
      __syncthreads();
    }
    if (live) {
#pragma unroll
      for (int cb = 0; cb < NB; ++cb)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int jo = cbase + (r & 3) + 4 * g + 8 * (r >> 2);
          if (jo < n) Z[(int64_t)jo * LP + 32 * cb + c] = acc[cb][r];
        }
    }
  }
  __syncthreads();
}

// ---- column means of X (rows x LP) in float64 -> S.mu (0 beyond l) --------
template <int LP>
__device__ __attribute__((noinline)) void p_colmean(const float* X_, int rows, int l) {
  rows = uni(rows);
  l = uni(l);
  auto X = as_global(uni(X_));
  PLds& S = g_S;
  constexpr int NG = NT / LP;
  const int tid = threadIdx.x, c = tid % LP, gi = tid / LP;
  double s = 0.0;
  if (c < l)
    for (int r0 = gi; r0 < rows; r0 += 8 * NG) {  // eight loads in flight
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = X[(int64_t)min(r0 + j * NG, rows - 1) * LP + c];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (r0 + j * NG < rows) s += (double)v[j];
    }
  S.u.red[gi * LP + c] = s;
  __syncthreads();
  if (tid < LP) {
    double t = 0.0;
    for (int h = 0; h < NG; ++h) t += S.u.red[h * LP + tid];
    S.mu[tid] = (tid < l && rows > 0) ? (float)(t / rows) : 0.f;
  }
  __syncthreads();
}

template <int LP>
__device__ __attribute__((noinline)) void p_sub_mu(float* X_, int rows, int l) {
  rows = uni(rows);
  l = uni(l);
  auto X = as_global(uni(X_));
  PLds& S = g_S;
  for (int e = threadIdx.x; e < rows * LP; e += NT) {
    const int c = e % LP;
    if (c < l) X[e] -= S.mu[c];
  }
  __syncthreads();
}

// ---- LU renormalization: Y (rows x LP) <- P L in place (rows <= 8192) -----
template <int LP>
__device__ __attribute__((noinline)) void p_lu(float* Y_, int rows, int l) {
  rows = uni(rows);
  l = uni(l);
  auto Y = as_global(uni(Y_));
  PLds& S = g_S;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  unsigned done = 0u;  // bit r: row tid + NT r is a pivot row
  int ph = 0;
  for (int c0 = 0; c0 < l; c0 += PB) {
    const int pw = min(PB, l - c0);
    const unsigned done0 = done;
    // the panel of this thread's remaining rows (others read as zero)
    float pan[RPT][PB];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + NT * r;
      const bool own = i < rows && !((done >> r) & 1u);
#pragma unroll
      for (int q = 0; q < PB; ++q)
        pan[r][q] = (own && q < pw) ? Y[(int64_t)i * LP + c0 + q] : 0.f;
    }
#pragma unroll
    for (int jj = 0; jj < PB; ++jj) {
      if (jj < pw) {
        const int j = c0 + jj;
        // this thread's candidate: largest |entry| of column j over its
        // remaining rows (rows ascend with r, so ties keep the smaller row)
        float best = -1.f;
        int bi = 0x7fffffff;
        float bv[PB];
#pragma unroll
        for (int q = 0; q < PB; ++q) bv[q] = 0.f;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {  // selects only: no branch per row
          const int i = tid + NT * r;
          float a = fabsf(pan[r][jj]);
          a = (a == a) ? a : 3.0e38f;  // a NaN entry is still a candidate (never none)
          const bool take = (i < rows) && !((done >> r) & 1u) && (a > best);
          best = take ? a : best;
          bi = take ? i : bi;
#pragma unroll
          for (int q = 0; q < PB; ++q) bv[q] = take ? pan[r][q] : bv[q];
        }
        // the wave's (DPP), then the workgroup's: larger |entry|, ties to the smaller row
        float wk = best;
        int wi = bi;
        wave_argmax_fast(wk, wi);
        if (bi == wi && best == wk && best >= 0.f) {
          S.u.lu.key[ph][wave] = wk;
          S.u.lu.kidx[ph][wave] = wi;
#pragma unroll
          for (int q = 0; q < PB; ++q) S.u.lu.row[ph][wave][q] = bv[q];
        }
        if (lane == 0 && !(wk >= 0.f)) {
          S.u.lu.key[ph][wave] = -1.f;
          S.u.lu.kidx[ph][wave] = 0x7fffffff;
        }
        __syncthreads();
        float kb = -1.f;
        int p = 0x7fffffff, wb = 0;
#pragma unroll
        for (int w = 0; w < NWAVE; ++w) {
          const float k = S.u.lu.key[ph][w];
          const int ki = S.u.lu.kidx[ph][w];
          if (k > kb || (k == kb && ki < p)) {
            kb = k;
            p = ki;
            wb = w;
          }
        }
        p = min(max(p, 0), rows - 1);  // always a valid row (j < l <= rows leaves one)
        float pr[PB];
#pragma unroll
        for (int q = 0; q < PB; ++q) pr[q] = S.u.lu.row[ph][wb][q];
        const float pv = pr[jj];
        const float rp = (pv != 0.f) ? 1.0f / pv : 0.f;  // a zero pivot: multipliers 0
        if (tid == 0) S.u.lu.piv[j] = p;
#pragma unroll
        for (int r = 0; r < RPT; ++r)
          if (tid + NT * r == p) done |= 1u << r;
#pragma unroll
        for (int r = 0; r < RPT; ++r) {  // selects only: no branch per row
          const int i = tid + NT * r;
          const bool upd = (i < rows) && !((done >> r) & 1u);
          const float f = pan[r][jj] * rp;
          pan[r][jj] = upd ? f : pan[r][jj];
#pragma unroll
          for (int q = jj + 1; q < PB; ++q) pan[r][q] = upd ? fmaf(-f, pr[q], pan[r][q]) : pan[r][q];
        }
        ph ^= 1;
      }
    }
    // multipliers (and the U part of this panel's pivot rows) back to Y
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
      const int i = tid + NT * r;
      if (i < rows && !((done0 >> r) & 1u))
#pragma unroll
        for (int q = 0; q < PB; ++q)
          if (q < pw) Y[(int64_t)i * LP + c0 + q] = pan[r][q];
    }
    __syncthreads();
    const int cs = c0 + pw;  // first trailing column
    if (cs < l) {
      // U12: the pivot rows' trailing entries after this panel's eliminations
      // (zero outside the trailing columns, so the update below can run over
      // whole rows)
      if (tid < LP) {
        const int col = tid;
        const bool trail = col >= cs && col < l;
        float u[PB];
#pragma unroll
        for (int t = 0; t < PB; ++t) {
          u[t] = 0.f;
          if (t < pw && trail) {
            const int pt = S.u.lu.piv[c0 + t];
            float v = Y[(int64_t)pt * LP + col];
#pragma unroll
            for (int s2 = 0; s2 < t; ++s2) v = fmaf(-Y[(int64_t)pt * LP + c0 + s2], u[s2], v);
            u[t] = v;
            Y[(int64_t)pt * LP + col] = v;
          }
          S.u.lu.U12[t][col] = u[t];
        }
      }
      __syncthreads();
      // the remaining rows: one vector load and store of the whole row each
#pragma unroll
      for (int r = 0; r < RPT; ++r) {
        const int i = tid + NT * r;
        if (i < rows && !((done >> r) & 1u)) {
          asm volatile("" ::: "memory");  // read U12 from LDS per row (no hoisting)
          auto yr = Y + (int64_t)i * LP;
          float mlt[PB];
#pragma unroll
          for (int t = 0; t < PB; ++t) mlt[t] = pan[r][t];
          float x[LP];
#pragma unroll
          for (int c = 0; c < LP; c += 4) {
            const f32x4 v = *reinterpret_cast<const GAS f32x4*>(yr + c);
            x[c] = v.x; x[c + 1] = v.y; x[c + 2] = v.z; x[c + 3] = v.w;
          }
#pragma unroll
          for (int c = 0; c < LP; c += 4) {
            f32x4 uu[PB];
#pragma unroll
            for (int t = 0; t < PB; ++t) uu[t] = *reinterpret_cast<const f32x4*>(&S.u.lu.U12[t][c]);
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              float v = x[c + e];
#pragma unroll
              for (int t = 0; t < PB; ++t) v = fmaf(-mlt[t], uu[t][e], v);
              x[c + e] = v;
            }
          }
#pragma unroll
          for (int c = 0; c < LP; c += 4)
            *reinterpret_cast<GAS f32x4*>(yr + c) = f32x4{x[c], x[c + 1], x[c + 2], x[c + 3]};
        }
      }
    }
  }
  __syncthreads();
  // pivot rows of L: 1 at their own step, 0 after it
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    const int i = tid + NT * r;
    if (i < rows && ((done >> r) & 1u)) {
      int st = 0;
      for (int j = 0; j < l; ++j)
        if (S.u.lu.piv[j] == i) st = j;
      auto yr = Y + (int64_t)i * LP;
      yr[st] = 1.f;
      for (int c = st + 1; c < l; ++c) yr[c] = 0.f;
    }
  }
  __syncthreads();
}

// ---- G (LP x LP, float64) = X^T X2 (X2 = X when null) ---------------------
// On the float64 matrix cores: v_mfma_f64_16x16x4f64 takes a 16 x 4 block of
// X^T and a 4 x 16 block of X2, lane L holding the entry (row r + L / 16,
// column 16 t + L % 16) of X or X2 in both, and lane L's register q of the
// 16 x 16 result is entry (L / 16 + 4 q, L % 16).  Wave w accumulates the
// tiles (ti <= tj only when X2 = X; the rest by symmetry) over the 4-row
// groups w, w + 8, w + 16, ... of the rows; the waves add their tiles in LDS
// in wave order.  Products of float32 values are exact in float64.
template <int LP, bool SAME>
__device__ __forceinline__ void gram_body(const GAS float* X, const GAS float* X2, int rows,
                                          GAS double* G) {
  PLds& S = g_S;
  typedef double d4 __attribute__((ext_vector_type(4)));
  constexpr int T = LP / 16, NT2 = SAME ? T * (T + 1) / 2 : T * T;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, lr = lane >> 4, lc = lane & 15;
  double* sh = S.u.gr;  // LP x LP
  d4 acc[NT2];
#pragma unroll
  for (int t = 0; t < NT2; ++t) acc[t] = d4{0.0, 0.0, 0.0, 0.0};
  constexpr int U = 2;  // 4-row groups per step and wave (loads in flight)
  for (int g0 = 4 * wave; g0 < rows; g0 += 4 * NWAVE * U) {
    double a[U][T], b[U][T];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int r = g0 + 4 * NWAVE * u + lr;
      const bool ok = r < rows;
      const int rc = ok ? r : 0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const float va = X[(int64_t)rc * LP + 16 * t + lc];
        a[u][t] = ok ? (double)va : 0.0;
        if constexpr (!SAME) {
          const float vb = X2[(int64_t)rc * LP + 16 * t + lc];
          b[u][t] = ok ? (double)vb : 0.0;
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < T; ++ti)
#pragma unroll
        for (int tj = SAME ? ti : 0; tj < T; ++tj) {
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][ti], SAME ? a[u][tj] : b[u][tj],
                                                        acc[t], 0, 0, 0);
          ++t;
        }
    }
  }
  for (int w = 0; w < NWAVE; ++w) {
    if (wave == w) {
      int t = 0;
#pragma unroll
      for (int ti = 0; ti < T; ++ti)
#pragma unroll
        for (int tj = SAME ? ti : 0; tj < T; ++tj) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int i = 16 * ti + lr + 4 * q, j = 16 * tj + lc;
            const double v = (w == 0) ? acc[t][q] : sh[i * LP + j] + acc[t][q];
            sh[i * LP + j] = v;
            if (SAME && ti != tj) sh[j * LP + i] = v;
          }
          ++t;
        }
    }
    __syncthreads();
  }
  for (int e = threadIdx.x; e < LP * LP; e += NT) G[e] = sh[e];
  __syncthreads();
}

template <int LP>
__device__ __attribute__((noinline)) void p_gram(const float* X_, const float* X2_, int rows, double* G_) {
  rows = uni(rows);
  auto X = as_global(uni(X_));
  auto X2 = as_global(uni(X2_));
  auto G = as_global(uni(G_));
  if (X2_ == nullptr) gram_body<LP, true>(X, X, rows, G);
  else gram_body<LP, false>(X, X2, rows, G);
}

// transpose and reciprocal diagonal of the float32 factor in S.u.tri.R (rows < l)
template <int LP>
__device__ __attribute__((noinline)) void p_tri_finish(int l) {
  PLds& S = g_S;
  for (int e = threadIdx.x; e < LP * LP; e += NT) {
    const int i = e / LP, j = e % LP;
    S.u.tri.Rt[j * LP + i] = (i < l && j < l) ? S.u.tri.R[e] : 0.f;
  }
  if (threadIdx.x < LP) {
    const int j = threadIdx.x;
    const float d = (j < l) ? S.u.tri.R[j * LP + j] : 0.f;
    S.u.tri.rd[j] = (d != 0.f) ? 1.0f / d : 0.f;
  }
  __syncthreads();
}

// One Cholesky-QR pass on the Gram matrix G: the factor (shifted when G is
// numerically singular) in S.u.tri, the pass bookkeeping in S.state (the
// layout of the multi-kernel path).
template <int LP>
__device__ __attribute__((noinline)) void p_chol_qr(const double* G_, int l, int pass) {
  l = uni(l);
  pass = uni(pass);
  auto G = as_global(uni(G_));
  PLds& S = g_S;
  const int tid = threadIdx.x;
  if (pass == 1 && tid < 12) S.state[tid] = 0;
  if (tid < LP) S.diag[tid] = (tid < l) ? G[tid * LP + tid] : 0.0;
  __syncthreads();
  double maxd = 0.0;
  for (int j = 0; j < l; ++j) maxd = fmax(maxd, S.diag[j]);
  bool shifted = false;
  for (int attempt = 0; attempt < 2; ++attempt) {
    __syncthreads();
    const double srel = attempt ? kShiftRel : 0.0;
    const double sabs = attempt ? (1e-30 * maxd + 1e-300) : 0.0;
    const bool ok = chol_par<LP, NT>(G_, false, l, srel, sabs, S.diag, attempt ? 0.0 : kTauRel,
                                     S.u.tri.R, S.ubuf);
    if (ok) break;
    if (attempt == 1 && tid == 0) {
      S.state[5] = 1;
      S.state[kStNonFinite] = 1;  // kept for the rest of the problem
    }
    shifted = true;
  }
  __syncthreads();
  if (tid == 0) {
    if (shifted) S.state[0] = 1;
    if (pass == 2) {
      unsigned mask[4] = {0u, 0u, 0u, 0u};
      int any = 0;
      if (S.state[0]) {
        for (int j = 0; j < l; ++j)
          if (!(S.diag[j] >= kJunkNorm2)) {
            mask[j >> 5] |= 1u << (j & 31);
            any = 1;
          }
      }
      for (int w = 0; w < 4; ++w) S.state[8 + w] = (int)mask[w];
      S.state[2] = any;
      S.state[1] = S.state[0] | any;
    }
  }
  p_tri_finish<LP>(l);
}

// X (rows x LP) <- (X + nu addX) R^-1 with the factor in S.u.tri
template <int LP>
__device__ __attribute__((noinline)) void p_trsm(float* X_, int rows, int l, const float* addX_, float nu) {
  rows = uni(rows);
  l = uni(l);
  auto X = as_global(uni(X_));
  auto addX = as_global(uni(addX_));
  PLds& S = g_S;
  for (int row = threadIdx.x; row < rows; row += NT) {
    asm volatile("" ::: "memory");  // read the factor from LDS inside the loop
    float x[LP];
    auto src = X + (int64_t)row * LP;
#pragma unroll
    for (int c = 0; c < LP; c += 4) {
      const f32x4 v = *reinterpret_cast<const GAS f32x4*>(src + c);
      x[c] = v.x; x[c + 1] = v.y; x[c + 2] = v.z; x[c + 3] = v.w;
    }
    if (addX) {
      auto a = addX + (int64_t)row * LP;
#pragma unroll
      for (int c = 0; c < LP; c += 4) {
        const f32x4 v = *reinterpret_cast<const GAS f32x4*>(a + c);
        x[c] += nu * v.x; x[c + 1] += nu * v.y; x[c + 2] += nu * v.z; x[c + 3] += nu * v.w;
      }
    }
#pragma unroll
    for (int j = 0; j < LP; ++j) {
      if (j < l) {
        float s = x[j];
        const float* col = S.u.tri.Rt + j * LP;
#pragma unroll
        for (int i = 0; i < j; ++i) s -= x[i] * col[i];
        x[j] = s * S.u.tri.rd[j];
      } else {
        x[j] = 0.f;
      }
    }
#pragma unroll
    for (int c = 0; c < LP; c += 4)
      *reinterpret_cast<GAS f32x4*>(src + c) = f32x4{x[c], x[c + 1], x[c + 2], x[c + 3]};
  }
  __syncthreads();
}

// Q (rows x LP): dependent columns (S.state mask) replaced by Gaussian ones;
// row r of Q is row r0 + r of the whole matrix (the counter of its entries)
template <int LP>
__device__ __attribute__((noinline)) void p_complete(float* Q_, int rows, int l, uint64_t seed,
                                                     int r0 = 0) {
  rows = uni(rows);
  l = uni(l);
  seed = uni(seed);
  r0 = uni(r0);
  auto Q = as_global(uni(Q_));
  PLds& S = g_S;
  if (S.state[2] == 0) return;
  for (int e = threadIdx.x; e < rows * l; e += NT) {
    const int r = e / l, j = e % l;
    if ((((unsigned)S.state[8 + (j >> 5)]) >> (j & 31)) & 1u)
      Q[(int64_t)r * LP + j] = philox_normal(seed, 3u, (uint64_t)(r0 + r) * 128u + (uint64_t)j);
  }
  __syncthreads();
}

// Cholesky QR, twice (and twice more when a pass was shifted or columns were
// completed); with want_r, G = Q^T X_in afterwards (X_in kept in Bk).
template <int LP>
// single: one Cholesky QR pass unless it had to shift (then the repair passes)
__device__ __attribute__((noinline)) void p_orth(float* X, int rows, int l, bool want_r, float* Bk, double* G,
                       uint64_t seed, bool single = false) {
  rows = uni(rows);
  l = uni(l);
  seed = uni(seed);
  X = uni(X);
  Bk = uni(Bk);
  G = uni(G);
  want_r = uni((int)want_r) != 0;
  single = uni((int)single) != 0;
  PLds& S = g_S;
  if (want_r) {
    auto src = as_global(X);
    auto dst = as_global(Bk);
    for (int e = threadIdx.x; e < rows * LP; e += NT) dst[e] = src[e];
    __syncthreads();
  }
  for (int pass = 1; pass <= 4; ++pass) {
    if (pass >= 3 && S.state[1] == 0) break;
    if (pass == 2 && single && S.state[0] == 0) break;
    p_gram<LP>(X, nullptr, rows, G);
    p_chol_qr<LP>(G, l, pass);
    p_trsm<LP>(X, rows, l, nullptr, 0.f);
    if (pass == 2) p_complete<LP>(X, rows, l, seed ^ 0x5bd1e995u);
  }
  if (want_r) p_gram<LP>(X, Bk, rows, G);
}

// out (rows x k, ld ldo) = X (rows x l) W (l x k), W float64 (stride LP) rounded to float32
template <int LP>
__device__ __attribute__((noinline)) void p_small_gemm(const float* X_, int rows, int l, const double* W_, int k, float* out_,
                             int64_t ldo) {
  rows = uni(rows);
  l = uni(l);
  k = uni(k);
  ldo = uni(ldo);
  auto X = as_global(uni(X_));
  auto W = as_global(uni(W_));
  auto out = as_global(uni(out_));
  PLds& S = g_S;
  for (int e = threadIdx.x; e < LP * LP; e += NT) {
    const int c = e / LP, i = e % LP;  // column c of W stored contiguously
    S.u.W[e] = (i < l && c < k) ? (float)W[i * LP + c] : 0.f;
  }
  __syncthreads();
  for (int row = threadIdx.x; row < rows; row += NT) {
    asm volatile("" ::: "memory");  // read the factor from LDS inside the loop
    float x[LP];
    auto src = X + (int64_t)row * LP;
#pragma unroll
    for (int c = 0; c < LP; c += 4) {
      const f32x4 v = *reinterpret_cast<const GAS f32x4*>(src + c);
      x[c] = v.x; x[c + 1] = v.y; x[c + 2] = v.z; x[c + 3] = v.w;
    }
    for (int c = 0; c < k; ++c) {
      const float* w = S.u.W + c * LP;
      float s = 0.f;
#pragma unroll
      for (int i = 0; i < LP; ++i) s += x[i] * w[i];
      out[(int64_t)row * ldo + c] = s;
    }
  }
  __syncthreads();
}

// sign convention on U (m x k) and V (n x k, nullable)
__device__ __attribute__((noinline)) void p_sign(float* U_, int64_t ldu, int m, int k, float* V_,
                                                 int64_t ldv, int n) {
  ldu = uni(ldu);
  m = uni(m);
  k = uni(k);
  ldv = uni(ldv);
  n = uni(n);
  auto U = as_global(uni(U_));
  auto V = as_global(uni(V_));
  PLds& S = g_S;
  const int tid = threadIdx.x, q = tid & 63, gi = tid >> 6;
  unsigned long long best = 0ull;
  if (q < k)
    for (int r0 = gi; r0 < m; r0 += 8 * NWAVE) {  // eight loads in flight
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = U[(int64_t)min(r0 + j * NWAVE, m - 1) * ldu + q];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int r = r0 + j * NWAVE;
        const unsigned long long key = (r < m) ? abs_key(v[j], r) : 0ull;
        best = key > best ? key : best;
      }
    }
  S.u.kred[gi * 64 + q] = best;
  __syncthreads();
  if (tid < k) {
    unsigned long long b = 0ull;
    for (int h = 0; h < NWAVE; ++h) b = S.u.kred[h * 64 + tid] > b ? S.u.kred[h * 64 + tid] : b;
    const int r = (int)(~(unsigned)b);
    S.sgn[tid] = (U[(int64_t)r * ldu + tid] < 0.f) ? -1.f : 1.f;
  }
  __syncthreads();
  for (int e = tid; e < m * k; e += NT) {
    const int r = e / k, c = e % k;
    if (S.sgn[c] < 0.f) U[(int64_t)r * ldu + c] = -U[(int64_t)r * ldu + c];
  }
  if (V)
    for (int e = tid; e < n * k; e += NT) {
      const int r = e / k, c = e % k;
      if (S.sgn[c] < 0.f) V[(int64_t)r * ldv + c] = -V[(int64_t)r * ldv + c];
    }
  __syncthreads();
}

// ||X||_F^2 over the first l columns, float64 (every thread gets the value)
template <int LP>
__device__ __attribute__((noinline)) double p_fro2(const float* X_, int rows, int l) {
  rows = uni(rows);
  l = uni(l);
  auto X = as_global(uni(X_));
  PLds& S = g_S;
  double s = 0.0;
  const int total = rows * LP;
  for (int e0 = threadIdx.x; e0 < total; e0 += 8 * NT) {  // eight loads in flight
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = X[min(e0 + j * NT, total - 1)];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int e = e0 + j * NT;
      if (e < total && (e % LP) < l) s += (double)v[j] * (double)v[j];
    }
  }
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) S.u.red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < NWAVE; ++w) t += S.u.red[w];
  __syncthreads();
  return t;
}

// Nystrom: Cholesky of (G + G^T)/2 + nu I with nu multiplied by 10 while it
// fails (at most max_retries times); the identity if it never succeeds.
template <int LP>
__device__ __attribute__((noinline)) double p_chol_nystrom(const double* G_, int l, double fro2, double n_sqrt_u,
                                 int max_retries) {
  l = uni(l);
  max_retries = uni(max_retries);
  const double* G = uni(G_);
  PLds& S = g_S;
  double nu = n_sqrt_u * sqrt(fro2);
  if (!(nu > 0.0)) nu = 1e-300;
  bool ok = false;
  int used = 0;
  for (int retry = 0; retry <= max_retries; ++retry) {
    __syncthreads();
    ok = chol_par<LP, NT>(G, true, l, 0.0, nu, S.zero, 0.0, S.u.tri.R, S.ubuf);
    used = retry;
    if (ok) break;
    if (retry < max_retries) nu *= 10.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    S.state[kStRetries] = used;
    S.state[kStNotPsd] = ok ? 0 : 1;
  }
  if (!ok)
    for (int e = threadIdx.x; e < LP * LP; e += NT) {
      const int i = e / LP, c = e % LP;
      S.u.tri.R[e] = (i == c && i < l) ? 1.f : 0.f;
    }
  __syncthreads();
  p_tri_finish<LP>(l);
  return nu;
}

template <int LP>
__device__ __attribute__((noinline)) void jacobi_wg(const double* G, int l, int transpose, Buf& b) {
  l = uni(l);
  transpose = uni(transpose);
  PLds& S = g_S;
  jacobi_body<LP, false, 16>((const double*)as_global(uni(G)), l, transpose,
                             (double*)as_global(uni(b.sv)), (double*)as_global(uni(b.Wacc)),
                             (double*)as_global(uni(b.Xn)), S.u.jac.M, S.u.jac.V,
                             S.u.jac.sig, S.u.jac.perm, S.u.jac.rot, S.u.jac.big);
  __syncthreads();
}

// The problem's status bits (small_core.h): non-finite returned values or
// Cholesky input, and for Nystrom a shifted factor never found; OR-ed into
// the caller's status word and stored in the problem's entry.
__device__ __attribute__((noinline)) void p_status(const PersProblem& p, const double* sv_,
                                                   double nu) {
  PLds& S = g_S;
  const double* sv = uni(sv_);
  __syncthreads();
  if (threadIdx.x == 0) {
    int bits = S.state[kStNonFinite] ? kErrNonFinite : 0;
    if (S.state[kStTeam]) bits |= kErrTimeout;
    if (!isfinite(nu)) bits |= kErrNonFinite;
    for (int j = 0; j < p.k; ++j)
      if (!isfinite(sv[j])) bits |= kErrNonFinite;
    if (p.kind == 1) {
      if (S.state[kStNotPsd]) bits |= kErrNotPsd;
      if (p.gstatus && p.part == 0) p.gstatus[1] = S.state[kStRetries];
    }
    if (bits && p.gstatus) atomicOr(p.gstatus, bits);
    // the entry is zero when the batch starts; every workgroup of a team adds its bits
    if (bits && p.status) atomicOr(p.status, bits);
  }
  __syncthreads();
}

template <int LP>
__device__ __attribute__((noinline)) void solve_svd(const PersProblem& p, Buf& b) {
  const float* A = p.A;
  const int m = p.m, n = p.n, l = p.l;
  const bool center = p.center != 0;
  auto mid = [&](float* T, int rows) {
    if (p.mid == 1) p_lu<LP>(T, rows, l);
    else p_orth<LP>(T, rows, l, false, b.T, b.G, p.seed, p.mid == 0);
  };
  auto apply_a = [&](const float* X) {  // Y = A X (centered when asked)
    p_pack<LP>(X, n, l, false, b.P);
    p_ax<LP>(A, p.lda, m, n, b.P, b.Y);
    if (center) {
      p_colmean<LP>(b.Y, m, l);
      p_sub_mu<LP>(b.Y, m, l);
    }
  };
  auto apply_at = [&]() {  // Z = A_c^T Y
    if (center) p_colmean<LP>(b.Y, m, l);
    p_pack<LP>(b.Y, m, l, center, b.P);
    p_atx<LP>(A, p.lda, m, n, b.P, b.Z);
  };
  p_omega<LP>(p.seed, n, l, b.Z, p.uniform, 0, n);
  apply_a(b.Z);
  if (p.its == 0) p_orth<LP>(b.Y, m, l, false, b.T, b.G, p.seed);
  else mid(b.Y, m);
  for (int it = 1; it <= p.its; ++it) {
    apply_at();
    mid(b.Z, n);
    apply_a(b.Z);
    if (it < p.its) mid(b.Y, m);
    else p_orth<LP>(b.Y, m, l, false, b.T, b.G, p.seed);
  }
  // Rayleigh-Ritz: A_c^T Q = Q2 R; the Jacobi SVD of R^T (graded rows of R:
  // fewer sweeps) gives R^T = X S W^T, so U = Q X, V = Q2 W
  apply_at();
  p_orth<LP>(b.Z, n, l, true, b.T, b.G, p.seed + 1);
  jacobi_wg<LP>(b.G, l, 1, b);
  p_small_gemm<LP>(b.Y, m, l, b.Xn, p.k, p.U, p.ldu);
  p_small_gemm<LP>(b.Z, n, l, b.Wacc, p.k, p.V, p.ldv);
  if (threadIdx.x < p.k) p.S[threadIdx.x] = b.sv[threadIdx.x];
  p_status(p, b.sv, 0.0);
  p_sign(p.U, p.ldu, m, p.k, p.V, p.ldv, n);
}

template <int LP>
__device__ __attribute__((noinline)) void solve_psd(const PersProblem& p, Buf& b,
                                                    int max_retries) {
  const float* A = p.A;
  const int n = p.n, l = p.l;
  float* Q = b.Y;
  float* Q2 = b.Z;
  p_omega<LP>(p.seed, n, l, Q, p.uniform, 0, n);
  if (p.its == 0) p_orth<LP>(Q, n, l, false, b.T, b.G, p.seed);
  for (int it = 1; it <= p.its; ++it) {
    p_pack<LP>(Q, n, l, false, b.P);
    p_ax<LP>(A, p.lda, n, n, b.P, Q2);
    float* t = Q;
    Q = Q2;
    Q2 = t;
    if (it < p.its && p.mid == 1) p_lu<LP>(Q, n, l);
    else p_orth<LP>(Q, n, l, false, b.T, b.G, p.seed, it < p.its && p.mid == 0);
  }
  // B1 = A Q (start); B2 = Q^T B1 (second), shifted; C = chol (Cholesky)
  p_pack<LP>(Q, n, l, false, b.P);
  p_ax<LP>(A, p.lda, n, n, b.P, Q2);
  const double fro2 = p_fro2<LP>(Q2, n, l);
  p_gram<LP>(Q, Q2, n, b.G);
  // u = 2^-16: B1 is formed by three bfloat16 products of split operands
  const double nu = p_chol_nystrom<LP>(b.G, l, fro2, sqrt((double)n) * 0x1p-16, max_retries);
  // F = (B1 + nu Q) C^-1 (pseudo); F = QF R, and the Jacobi SVD of R^T gives
  // F = QF W diag(s) X^T, so U = QF W
  p_trsm<LP>(Q2, n, l, Q, (float)nu);
  p_orth<LP>(Q2, n, l, true, b.T, b.G, p.seed + 1);
  jacobi_wg<LP>(b.G, l, 1, b);
  p_small_gemm<LP>(Q2, n, l, b.Wacc, p.k, p.U, p.ldu);
  if (threadIdx.x < p.k) {
    const double s = b.sv[threadIdx.x];
    p.S[threadIdx.x] = fmax(s * s - nu, 0.0);
  }
  p_status(p, b.sv, nu);
  p_sign(p.U, p.ldu, n, p.k, nullptr, 0, 0);
}

// ---- one problem over several workgroups (a team) ---------------------------
// A problem that costs more than the batch's average share of a workgroup is
// split by the host over ``parts`` workgroups.  Every team's entries come
// first in the table and the grid holds all of them, so the workgroups of a
// team are on the device together.  Each workgroup takes a range of rows (a
// multiple of 64, never empty) on the m side and on the n side: its share of
// Omega and of the packed operands, of the passes over A (A X over its m
// rows; A^T X over its m rows into a partial that the team then sums by n
// rows, in a fixed order), of the Gram matrices, the triangular solves,
// U = Q W, V = Q2 X and the sign convention.  The l x l steps (Cholesky,
// Jacobi) run in every workgroup of the team on the same summed Gram matrix,
// so every workgroup takes the same branches.  The workgroups meet at an
// arrival counter (team_sync); a wait is bounded, and a workgroup that gives
// up marks the problem kErrTimeout and waits no more.

struct TeamBufs {
  float* Y;
  float* Z;
  float* T;
  __bf16* P;
  float* zpart;               // parts x np x 64
  double* gpart;              // 2 x parts x 4096
  double* vpart;              // 2 x parts x 64
  unsigned long long* kpart;  // parts x 128 (keys, then signs)
};

// the layout team_floats (kernels.h) sizes
__device__ __forceinline__ TeamBufs team_carve(float* sh, int parts, int64_t R, int64_t np) {
  TeamBufs t;
  t.Y = sh;
  t.Z = sh + R * 64;
  t.T = sh + 2 * R * 64;
  t.P = reinterpret_cast<__bf16*>(sh + 3 * R * 64);
  t.zpart = sh + 4 * R * 64;
  double* d = reinterpret_cast<double*>(t.zpart + (int64_t)parts * np * 64);
  t.gpart = d;
  t.vpart = d + 2 * (int64_t)parts * 4096;
  t.kpart = reinterpret_cast<unsigned long long*>(t.vpart + 2 * (int64_t)parts * 64);
  return t;
}

// first row of part g of ``rows`` rows over ``parts`` (multiples of 64; with
// parts <= rows / 64 every part is non-empty)
__device__ __forceinline__ int part_row(int rows, int parts, int g) {
  const int64_t r = ((int64_t)rows * g + parts - 1) / parts;
  const int64_t a = (r + 63) / 64 * 64;
  return (int)(a < rows ? a : rows);
}

__device__ __attribute__((noinline)) int p_state(int i) { return g_S.state[uni(i)]; }

// Every workgroup of the team arrives (the k-th call of a solve waits for
// k * parts arrivals); the writes of every workgroup before it are visible to
// all after it.  At most spin_limit polls.
__device__ __attribute__((noinline)) void team_sync(int* bar_, int target, int spin_limit) {
  int* bar = uni(bar_);
  target = uni(target);
  spin_limit = uni(spin_limit);
  PLds& S = g_S;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    atomicAdd(bar, 1);
    if (S.state[kStTeam] == 0) {
      int spins = 0;
      while (__hip_atomic_load(bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
        __builtin_amdgcn_s_sleep(8);
        if (++spins >= spin_limit) {
          S.state[kStTeam] = 1;
          break;
        }
      }
    }
  }
  __syncthreads();
  __threadfence();
}

// column sums (float64) of X (rows x LP) -> out[0 .. LP)
template <int LP>
__device__ __attribute__((noinline)) void p_colsum_part(const float* X_, int rows, int l,
                                                        double* out_) {
  rows = uni(rows);
  l = uni(l);
  auto X = as_global(uni(X_));
  auto out = as_global(uni(out_));
  PLds& S = g_S;
  constexpr int NG = NT / LP;
  const int tid = threadIdx.x, c = tid % LP, gi = tid / LP;
  double s = 0.0;
  if (c < l)
    for (int r0 = gi; r0 < rows; r0 += 8 * NG) {  // eight loads in flight
      float v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = X[(int64_t)min(r0 + j * NG, rows - 1) * LP + c];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (r0 + j * NG < rows) s += (double)v[j];
    }
  S.u.red[gi * LP + c] = s;
  __syncthreads();
  if (tid < LP) {
    double t = 0.0;
    for (int h = 0; h < NG; ++h) t += S.u.red[h * LP + tid];
    out[tid] = t;
  }
  __syncthreads();
}

// S.mu = (the column sums of the parts, added in order) / rows
template <int LP>
__device__ __attribute__((noinline)) void p_mu_parts(const double* vp_, int parts, int rows,
                                                     int l) {
  auto vp = as_global(uni(vp_));
  parts = uni(parts);
  rows = uni(rows);
  l = uni(l);
  PLds& S = g_S;
  if (threadIdx.x < LP) {
    double t = 0.0;
    for (int q = 0; q < parts; ++q) t += vp[q * 64 + threadIdx.x];
    S.mu[threadIdx.x] = ((int)threadIdx.x < l && rows > 0) ? (float)(t / rows) : 0.f;
  }
  __syncthreads();
}

// G (LP x LP) = the partial Gram matrices of the parts (stride 4096), added in order
template <int LP>
__device__ __attribute__((noinline)) void p_sum_parts(const double* gp_, int parts, double* G_) {
  auto gp = as_global(uni(gp_));
  auto G = as_global(uni(G_));
  parts = uni(parts);
  for (int e = threadIdx.x; e < LP * LP; e += NT) {
    double t = 0.0;
    for (int q = 0; q < parts; ++q) t += gp[(int64_t)q * 4096 + e];
    G[e] = t;
  }
  __syncthreads();
}

// one float64 value per part: write this part's (thread 0), or add all in order
__device__ __attribute__((noinline)) void p_put_scalar(double* dst_, double v) {
  auto dst = as_global(uni(dst_));
  if (threadIdx.x == 0) *dst = v;
  __syncthreads();
}
__device__ __attribute__((noinline)) double p_sum_scalars(const double* vp_, int parts) {
  auto vp = as_global(uni(vp_));
  parts = uni(parts);
  double t = 0.0;
  for (int q = 0; q < parts; ++q) t += vp[q * 64];
  return t;
}

// Z rows r0 .. r1 - 1 = the A^T X partials of the parts (slot stride ``slot``
// floats, row stride LP) added in order
template <int LP>
__device__ __attribute__((noinline)) void p_reduce_parts(const float* zp_, int parts, int64_t slot,
                                                         int r0, int r1, float* Z_) {
  auto zp = as_global(uni(zp_));
  auto Z = as_global(uni(Z_));
  parts = uni(parts);
  slot = uni(slot);
  r0 = uni(r0);
  r1 = uni(r1);
  const int64_t e1 = (int64_t)r1 * LP;
  for (int64_t e = (int64_t)r0 * LP + 4 * threadIdx.x; e < e1; e += 4 * NT) {
    f32x4 a = *reinterpret_cast<const GAS f32x4*>(zp + e);
    for (int q = 1; q < parts; ++q) {
      const f32x4 v = *reinterpret_cast<const GAS f32x4*>(zp + (int64_t)q * slot + e);
      a.x += v.x;
      a.y += v.y;
      a.z += v.z;
      a.w += v.w;
    }
    *reinterpret_cast<GAS f32x4*>(Z + e) = a;
  }
  __syncthreads();
}

// rows (x LP) of X copied to Y
template <int LP>
__device__ __attribute__((noinline)) void p_copy_rows(const float* X_, float* Y_, int rows) {
  auto X = as_global(uni(X_));
  auto Y = as_global(uni(Y_));
  rows = uni(rows);
  for (int e = threadIdx.x; e < rows * LP; e += NT) Y[e] = X[e];
  __syncthreads();
}

// Sign convention over a team, first half: per column q < k the key of the
// largest-magnitude entry among rows r0 .. r1 - 1 of U (ties to the smaller
// row) -> kp[q], and that entry's sign -> kp[64 + q] (1 when negative)
__device__ __attribute__((noinline)) void p_sign_key(const float* U_, int64_t ldu, int r0, int r1,
                                                     int k, unsigned long long* kp_) {
  auto U = as_global(uni(U_));
  auto kp = as_global(uni(kp_));
  ldu = uni(ldu);
  r0 = uni(r0);
  r1 = uni(r1);
  k = uni(k);
  PLds& S = g_S;
  const int tid = threadIdx.x, q = tid & 63, gi = tid >> 6;
  unsigned long long best = 0ull;
  if (q < k)
    for (int r = r0 + gi; r < r1; r += NWAVE) {
      const unsigned long long key = abs_key(U[(int64_t)r * ldu + q], r);
      best = key > best ? key : best;
    }
  S.u.kred[gi * 64 + q] = best;
  __syncthreads();
  if (tid < 64) {
    unsigned long long bb = 0ull;
    for (int h = 0; h < NWAVE; ++h) bb = S.u.kred[h * 64 + tid] > bb ? S.u.kred[h * 64 + tid] : bb;
    kp[tid] = bb;
    kp[64 + tid] = (tid < k && bb != 0ull && U[(int64_t)(int)(~(unsigned)bb) * ldu + tid] < 0.f)
                       ? 1ull : 0ull;
  }
  __syncthreads();
}

// second half: the winning part's sign per column; this part's rows of U and V flipped
__device__ __attribute__((noinline)) void p_sign_apply(const unsigned long long* kp_, int parts,
                                                       float* U_, int64_t ldu, int k, int ur0,
                                                       int ur1, float* V_, int64_t ldv, int vr0,
                                                       int vr1) {
  auto kp = as_global(uni(kp_));
  auto U = as_global(uni(U_));
  auto V = as_global(uni(V_));
  parts = uni(parts);
  ldu = uni(ldu);
  k = uni(k);
  ur0 = uni(ur0);
  ur1 = uni(ur1);
  ldv = uni(ldv);
  vr0 = uni(vr0);
  vr1 = uni(vr1);
  PLds& S = g_S;
  const int tid = threadIdx.x;
  if (tid < k) {
    unsigned long long bb = 0ull, neg = 0ull;
    for (int q = 0; q < parts; ++q) {
      const unsigned long long key = kp[q * 128 + tid];
      if (key > bb) {
        bb = key;
        neg = kp[q * 128 + 64 + tid];
      }
    }
    S.sgn[tid] = neg ? -1.f : 1.f;
  }
  __syncthreads();
  for (int e = tid; e < (ur1 - ur0) * k; e += NT) {
    const int r = ur0 + e / k, c = e % k;
    if (S.sgn[c] < 0.f) U[(int64_t)r * ldu + c] = -U[(int64_t)r * ldu + c];
  }
  if (V)
    for (int e = tid; e < (vr1 - vr0) * k; e += NT) {
      const int r = vr0 + e / k, c = e % k;
      if (S.sgn[c] < 0.f) V[(int64_t)r * ldv + c] = -V[(int64_t)r * ldv + c];
    }
  __syncthreads();
}

// The steps a team shares: the row ranges, the synchronization and the
// partial sums of one solve.
template <int LP>
struct TeamRun {
  const PersProblem& p;
  Buf& b;
  TeamBufs t;
  int parts, g, spin, target, gsel, vsel;
  int64_t np;
  __device__ TeamRun(const PersProblem& p_, Buf& b_, int spin_limit) : p(p_), b(b_) {
    parts = p.parts;
    g = p.part;
    spin = spin_limit;
    target = gsel = vsel = 0;
    np = round_up(p.n, 64);
    t = team_carve(p.sh, parts, round_up(max(p.m, p.n), 64), np);
  }
  __device__ void sync() {
    target += parts;
    team_sync(p.bar, target, spin);
  }
  __device__ __bf16* packed(int r0) { return t.P + (int64_t)(r0 / 16) * (LP / 32) * 2 * 512; }
  // S.mu = the column means of X (``rows`` rows; this part holds r0 .. r1 - 1)
  __device__ void colmean(const float* X, int rows, int r0, int r1) {
    double* vp = t.vpart + (int64_t)vsel * parts * 64;
    vsel ^= 1;
    p_colsum_part<LP>(X + (int64_t)r0 * LP, r1 - r0, p.l, vp + (int64_t)g * 64);
    sync();
    p_mu_parts<LP>(vp, parts, rows, p.l);
  }
  // a sum over all rows of a per-part float64 value
  __device__ double scalar_sum(double v) {
    double* vp = t.vpart + (int64_t)vsel * parts * 64;
    vsel ^= 1;
    p_put_scalar(vp + (int64_t)g * 64, v);
    sync();
    return p_sum_scalars(vp, parts);
  }
  // b.G = X^T X2 (X^T X when X2 is null) over all rows
  __device__ void gram(const float* X, const float* X2, int r0, int r1) {
    double* gp = t.gpart + (int64_t)gsel * parts * 4096;
    gsel ^= 1;
    p_gram<LP>(X + (int64_t)r0 * LP, X2 ? X2 + (int64_t)r0 * LP : nullptr, r1 - r0,
               gp + (int64_t)g * 4096);
    sync();
    p_sum_parts<LP>(gp, parts, b.G);
  }
  // p_orth over the team (Cholesky QR; with want_r, b.G = Q^T X_in after)
  __device__ void orth(float* X, int r0, int r1, bool want_r, uint64_t seed, bool single) {
    if (want_r) p_copy_rows<LP>(X + (int64_t)r0 * LP, t.T + (int64_t)r0 * LP, r1 - r0);
    for (int pass = 1; pass <= 4; ++pass) {
      if (pass >= 3 && p_state(1) == 0) break;
      if (pass == 2 && single && p_state(0) == 0) break;
      gram(X, nullptr, r0, r1);
      p_chol_qr<LP>(b.G, p.l, pass);
      p_trsm<LP>(X + (int64_t)r0 * LP, r1 - r0, p.l, nullptr, 0.f);
      if (pass == 2) p_complete<LP>(X + (int64_t)r0 * LP, r1 - r0, p.l, seed ^ 0x5bd1e995u, r0);
    }
    if (want_r) gram(X, t.T, r0, r1);
  }
  // out = A X for this part's rows r0 .. r1 of A, X (the n side, this part
  // holding rows x0 .. x1) packed first
  __device__ void ax(const float* X, int x0, int x1, float* out, int r0, int r1) {
    p_pack<LP>(X + (int64_t)x0 * LP, x1 - x0, p.l, false, packed(x0));
    sync();
    p_ax<LP>(p.A + (int64_t)r0 * p.lda, p.lda, r1 - r0, p.n, t.P, out + (int64_t)r0 * LP);
  }
  // sign convention for U (rows ur0 .. ur1 of this part) and V
  __device__ void sign(int ur0, int ur1, float* V, int vr0, int vr1) {
    p_sign_key(p.U, p.ldu, ur0, ur1, p.k, t.kpart + (int64_t)g * 128);
    sync();
    p_sign_apply(t.kpart, parts, p.U, p.ldu, p.k, ur0, ur1, V, p.ldv, vr0, vr1);
  }
};

template <int LP>
__device__ __attribute__((noinline)) void team_svd(const PersProblem& p, Buf& b, int spin_limit) {
  TeamRun<LP> T(p, b, spin_limit);
  const int m = p.m, n = p.n, l = p.l, parts = p.parts, g = p.part;
  const bool center = p.center != 0;
  const int mr0 = part_row(m, parts, g), mr1 = part_row(m, parts, g + 1);
  const int nr0 = part_row(n, parts, g), nr1 = part_row(n, parts, g + 1);
  float* Y = T.t.Y;
  float* Z = T.t.Z;
  auto apply_a = [&]() {  // Y = A_c Z
    T.ax(Z, nr0, nr1, Y, mr0, mr1);
    if (center) {
      T.colmean(Y, m, mr0, mr1);
      p_sub_mu<LP>(Y + (int64_t)mr0 * LP, mr1 - mr0, l);
    }
  };
  auto apply_at = [&]() {  // Z = A_c^T Y: partials over this part's m rows, summed by n rows
    if (center) T.colmean(Y, m, mr0, mr1);
    p_pack<LP>(Y + (int64_t)mr0 * LP, mr1 - mr0, l, center, T.packed(mr0));
    T.sync();
    float* zp = T.t.zpart + (int64_t)g * T.np * 64;
    p_atx<LP>(p.A + (int64_t)mr0 * p.lda, p.lda, mr1 - mr0, n, T.packed(mr0), zp);
    T.sync();
    p_reduce_parts<LP>(T.t.zpart, parts, T.np * 64, nr0, nr1, Z);
  };
  // LU problems are not split: the renormalization is Cholesky QR
  auto mid = [&](float* X, int r0, int r1) { T.orth(X, r0, r1, false, p.seed, p.mid == 0); };
  p_omega<LP>(p.seed, n, l, Z, p.uniform, nr0, nr1);
  apply_a();
  if (p.its == 0) T.orth(Y, mr0, mr1, false, p.seed, false);
  else mid(Y, mr0, mr1);
  for (int it = 1; it <= p.its; ++it) {
    apply_at();
    mid(Z, nr0, nr1);
    apply_a();
    if (it < p.its) mid(Y, mr0, mr1);
    else T.orth(Y, mr0, mr1, false, p.seed, false);
  }
  apply_at();
  T.orth(Z, nr0, nr1, true, p.seed + 1, false);
  jacobi_wg<LP>(b.G, l, 1, b);
  p_small_gemm<LP>(Y + (int64_t)mr0 * LP, mr1 - mr0, l, b.Xn, p.k, p.U + (int64_t)mr0 * p.ldu,
                   p.ldu);
  p_small_gemm<LP>(Z + (int64_t)nr0 * LP, nr1 - nr0, l, b.Wacc, p.k, p.V + (int64_t)nr0 * p.ldv,
                   p.ldv);
  if (g == 0 && threadIdx.x < p.k) p.S[threadIdx.x] = b.sv[threadIdx.x];
  T.sign(mr0, mr1, p.V, nr0, nr1);
  p_status(p, b.sv, 0.0);
}

template <int LP>
__device__ __attribute__((noinline)) void team_psd(const PersProblem& p, Buf& b, int max_retries,
                                                   int spin_limit) {
  TeamRun<LP> T(p, b, spin_limit);
  const int n = p.n, l = p.l, parts = p.parts, g = p.part;
  const int r0 = part_row(n, parts, g), r1 = part_row(n, parts, g + 1);
  float* Q = T.t.Y;
  float* Q2 = T.t.Z;
  p_omega<LP>(p.seed, n, l, Q, p.uniform, r0, r1);
  if (p.its == 0) T.orth(Q, r0, r1, false, p.seed, false);
  for (int it = 1; it <= p.its; ++it) {
    T.ax(Q, r0, r1, Q2, r0, r1);
    float* t = Q;
    Q = Q2;
    Q2 = t;
    T.orth(Q, r0, r1, false, p.seed, it < p.its && p.mid == 0);
  }
  // B1 = A Q (start); B2 = Q^T B1 (second), shifted; C = chol (Cholesky)
  T.ax(Q, r0, r1, Q2, r0, r1);
  const double fro2 = T.scalar_sum(p_fro2<LP>(Q2 + (int64_t)r0 * LP, r1 - r0, l));
  T.gram(Q, Q2, r0, r1);
  const double nu = p_chol_nystrom<LP>(b.G, l, fro2, sqrt((double)n) * 0x1p-16, max_retries);
  // F = (B1 + nu Q) C^-1 (pseudo); U from the Jacobi SVD of F's R factor
  p_trsm<LP>(Q2 + (int64_t)r0 * LP, r1 - r0, l, Q + (int64_t)r0 * LP, (float)nu);
  T.orth(Q2, r0, r1, true, p.seed + 1, false);
  jacobi_wg<LP>(b.G, l, 1, b);
  p_small_gemm<LP>(Q2 + (int64_t)r0 * LP, r1 - r0, l, b.Wacc, p.k, p.U + (int64_t)r0 * p.ldu,
                   p.ldu);
  if (g == 0 && threadIdx.x < p.k) {
    const double s = b.sv[threadIdx.x];
    p.S[threadIdx.x] = fmax(s * s - nu, 0.0);
  }
  T.sign(r0, r1, nullptr, 0, 0);
  p_status(p, b.sv, nu);
}

// The next problem index for the workgroup (the LDS block is only touched from
// non-inlined routines: LDS used both by a kernel and by the functions it
// calls would be allocated twice).
__device__ __attribute__((noinline)) int next_problem(int* counter) {
  PLds& S = g_S;
  if (threadIdx.x < 64) S.zero[threadIdx.x] = 0.0;
  if (threadIdx.x < 16) S.state[threadIdx.x] = 0;
  __syncthreads();
  if (threadIdx.x == 0) S.idx = atomicAdd(counter, 1);
  __syncthreads();
  return S.idx;
}

__global__ void __launch_bounds__(NT) persistent_kernel(const PersProblem* __restrict__ probs,
                                                        int count, int* counter, float* ws,
                                                        int64_t slot_floats, int64_t R,
                                                        int max_retries, int spin_limit) {
  Buf b = carve(ws + (int64_t)blockIdx.x * slot_floats, R);
  for (;;) {
    const int idx = next_problem(counter);
    if (idx >= count) break;
    const PersProblem p = probs[idx];
    if (p.parts > 1) {
      if (p.l <= 32) {
        if (p.kind == 0) team_svd<32>(p, b, spin_limit);
        else team_psd<32>(p, b, max_retries, spin_limit);
      } else {
        if (p.kind == 0) team_svd<64>(p, b, spin_limit);
        else team_psd<64>(p, b, max_retries, spin_limit);
      }
    } else if (p.l <= 32) {
      if (p.kind == 0) solve_svd<32>(p, b);
      else solve_psd<32>(p, b, max_retries);
    } else {
      if (p.kind == 0) solve_svd<64>(p, b);
      else solve_psd<64>(p, b, max_retries);
    }
  }
}

// The problem table travels in kernel arguments (16 entries per launch, well
// inside the 4 KiB argument block) and is written on the stream, so a
// captured graph replays its own table.
constexpr int kTabChunk = 16;
static_assert(sizeof(PersProblem) * kTabChunk + 16 <= 4096, "problem table chunk too large");
struct TabChunk {
  PersProblem p[kTabChunk];
};

__global__ void __launch_bounds__(kTabChunk) table_kernel(TabChunk c, int cnt, PersProblem* dst) {
  if ((int)threadIdx.x < cnt) dst[threadIdx.x] = c.p[threadIdx.x];
}

}  // namespace

void launch_pers_table(hipStream_t st, const PersProblem* host, int count, PersProblem* dev) {
  for (int c0 = 0; c0 < count; c0 += kTabChunk) {
    TabChunk c;
    const int cnt = count - c0 < kTabChunk ? count - c0 : kTabChunk;
    for (int i = 0; i < cnt; ++i) c.p[i] = host[c0 + i];
    hipLaunchKernelGGL(table_kernel, dim3(1), dim3(kTabChunk), 0, st, c, cnt, dev + c0);
  }
}

int64_t pers_rows(int64_t maxdim) { return round_up(maxdim > 0 ? maxdim : 1, 64); }

int64_t pers_slot_floats(int64_t maxdim) {
  return 4 * pers_rows(maxdim) * 64 + 2 * (3 * 4096 + 64);
}

void launch_persistent(hipStream_t st, const PersProblem* probs, int count, int* counter,
                       float* ws, int64_t maxdim, int grid, int max_retries, int spin_limit) {
  if (count <= 0 || grid <= 0) return;
  hipLaunchKernelGGL(persistent_kernel, dim3(grid), dim3(NT), 0, st, probs, count, counter, ws,
                     pers_slot_floats(maxdim), pers_rows(maxdim), max_retries, spin_limit);
}

}  // namespace rpca
