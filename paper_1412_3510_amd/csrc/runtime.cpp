// Host runtime and C ABI: context, workspace, argument checks, and the
// stream-ordered launch sequences of the randomized SVD (Sections 2 and 5),
// the Nystrom method (Section 3) and the step-level test entry points.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <list>
#include <map>
#include <queue>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/rpca.h"
#include "common.h"
#include "internal.h"
#include "kernels.h"
#include "small_core.h"

using namespace rpca;

namespace {

struct TimedLaunch {
  hipEvent_t a, b;
  int kind;  // 0 = A X, 1 = A^T X (float32 A); 2, 3 the same on a low-precision copy
  double bytes;
};

}  // namespace

// One stream of a batch: its own workspace and LU arrival counters.
struct BatchSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  unsigned* counters = nullptr;
  size_t counters_n = 0;
};

struct rpca_ctx_s {
  hipStream_t stream = nullptr;
  int device = 0;
  int num_cus = 256;
  char* ws = nullptr;
  size_t ws_bytes = 0;
  size_t ws_limit = 0;
  unsigned* counters = nullptr;  // LU arrival counters; zero between launches
  size_t counters_n = 0;
  std::string err;
  bool timing = false;
  std::vector<TimedLaunch> pending;
  std::vector<hipEvent_t> event_pool;
  rpca_stats stats{};
  int* host_state = nullptr;  // pinned
  // device status: [0] OR of the error bits (small_core.h) of the solves since
  // the last synchronizing call, [1] Nystrom shift retries of the last solve
  int* dstat = nullptr;
  int nys_retries = 10;  // Nystrom shift retries before RPCA_ERR_NOT_PSD
  // per-problem status of the last rpca_svd_batched call (device), its size
  int* bstat = nullptr;
  int bstat_cap = 0;
  int bstat_count = 0;
  std::vector<BatchSlot> slots;
  hipEvent_t fork = nullptr;
  // autotuned configurations by shape class (ceil log2 m, ceil log2 n, lp, dtype)
  std::map<std::array<int, 4>, TuneCfg> tune;
  int batch_streams = 8;  // streams rpca_svd_batched spreads a batch over
  int batch_mode = 0;     // 0: persistent launch for the problems it takes; 1: streams only
  // persistent batched launch: the device problem table (rewritten by every
  // call, on the stream, so a captured graph carries its own table), the work
  // counter, the working memory, and memory superseded by larger buffers
  // (graphs captured earlier still use it, so it is kept until rpca_destroy)
  rpca::PersProblem* pers_tab = nullptr;
  int pers_tab_cap = 0;
  int* pers_counter = nullptr;
  float* pers_ws = nullptr;
  int64_t pers_ws_floats = 0;
  // shared buffers and arrival counters of the problems split over workgroups
  float* pers_sh = nullptr;
  int64_t pers_sh_floats = 0;
  int* pers_bar = nullptr;
  int pers_bar_cap = 0;
  int split_max_parts = 8;
  int split_min_parts = 1;
  int team_spins = 1 << 22;
  std::vector<void*> pers_retired;
};

namespace {

rpca_status fail(rpca_ctx c, rpca_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

#define HIP_OK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, RPCA_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

int lp_of(int l) { return l <= 32 ? 32 : (l <= 64 ? 64 : 128); }

// Bump allocator over the context workspace.  plan() sizes, then carve().
struct Arena {
  size_t off = 0;
  char* base = nullptr;
  template <typename T>
  T* take(size_t count) {
    off = round_up(off, 256);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

rpca_status ensure_ws(rpca_ctx ctx, size_t bytes) {
  if (ctx->ws_limit && bytes > ctx->ws_limit)
    return fail(ctx, RPCA_ERR_NO_MEMORY,
                "workspace of " + std::to_string(bytes) + " bytes exceeds the limit of " +
                    std::to_string(ctx->ws_limit));
  if (bytes <= ctx->ws_bytes) return RPCA_OK;
  if (ctx->ws) {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    HIP_OK(hipFree(ctx->ws));
    ctx->ws = nullptr;
    ctx->ws_bytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RPCA_ERR_NO_MEMORY, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
  }
  ctx->ws = static_cast<char*>(p);
  ctx->ws_bytes = bytes;
  return RPCA_OK;
}

rpca_status ensure_counters(rpca_ctx ctx, size_t n) {
  if (n <= ctx->counters_n) return RPCA_OK;
  if (ctx->counters) {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    HIP_OK(hipFree(ctx->counters));
    ctx->counters = nullptr;
    ctx->counters_n = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, n * sizeof(unsigned)) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RPCA_ERR_NO_MEMORY, "hipMalloc of LU counters failed");
  }
  HIP_OK(hipMemset(p, 0, n * sizeof(unsigned)));
  ctx->counters = static_cast<unsigned*>(p);
  ctx->counters_n = n;
  return RPCA_OK;
}

// Synchronize the stream and report the device-side failures of the solves
// issued since the last such call (then forgotten).
rpca_status sync_status(rpca_ctx ctx) {
  HIP_OK(hipStreamSynchronize(ctx->stream));
  HIP_OK(hipMemcpyAsync(ctx->host_state, ctx->dstat, 2 * sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  const int bits = ctx->host_state[0];
  ctx->stats.shift_retries = ctx->host_state[1];
  if (!bits) return RPCA_OK;
  launch_fill_zero(ctx->stream, reinterpret_cast<float*>(ctx->dstat), 4);
  HIP_OK(hipStreamSynchronize(ctx->stream));
  // non-finite values are the cause when both are set (a NaN also defeats
  // every shifted Cholesky factorization)
  // a share that stopped waiting computed from incomplete data: that is the cause
  if (bits & kErrTimeout)
    return fail(ctx, RPCA_ERR_TIMEOUT,
                "a batched problem split over workgroups gave up waiting for its other shares");
  if (bits & kErrNonFinite)
    return fail(ctx, RPCA_ERR_NUMERICAL, "non-finite values met on the device (is A finite?)");
  return fail(ctx, RPCA_ERR_NOT_PSD,
              "shifted B2 = Q*(A + nu I)Q not positive definite after the shift retries");
}

hipEvent_t take_event(rpca_ctx ctx) {
  if (!ctx->event_pool.empty()) {
    hipEvent_t e = ctx->event_pool.back();
    ctx->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Scratch shared by the steps of one solve.
struct Work {
  int l = 0, lp = 0, nb = 0;
  int64_t rows_max = 0;
  // tall buffers
  float* Y = nullptr;     // m x lp
  float* Z = nullptr;     // n x lp
  float* Y2 = nullptr;    // m x lp (second tall buffer, Nystrom)
  float* Bk = nullptr;    // copy of the matrix being orthonormalized, for R = Q^T B
  __bf16* Xp = nullptr;   // packed operand (max of both sides)
  float* P = nullptr;     // A^T X partials
  float* mu = nullptr;    // lp
  double* colpart = nullptr;
  double* colpart2 = nullptr;
  double* gpart = nullptr;
  double* G = nullptr;
  float* Rf = nullptr;
  int* cand = nullptr;
  int* piv = nullptr;
  float* Ulu = nullptr;
  int* state = nullptr;
  double* sv = nullptr;
  double* Wacc = nullptr;
  double* Xn = nullptr;
  double* jwork = nullptr;
  int* signwork = nullptr;
  double* scal = nullptr;  // [0] fro2, [1] nu
  float* nu_f = nullptr;
  TuneCfg cfg{};     // tile configuration of this shape class
  int64_t lu_ctr = 0;  // LU arrival counters the largest tournament plan needs
  AtxPlan atx{};     // plan for the copy of A the range finder reads
  AtxPlan atx_rr{};  // plan for the float32 copy of the Rayleigh-Ritz pass
  LuPlan lu_m{}, lu_n{};
};

// The copy of A one pass reads: float32, bfloat16 or E4M3 with column scales.
struct AView {
  const void* data;
  int dtype;
  int64_t ld, m, n;
  const float* scale;  // E4M3: A = data diag(scale)
};

AView native_view(const rpca_matrix* A) {
  return {A->data, (int)A->dtype, A->ld, A->m, A->n,
          A->dtype == RPCA_FP8_E4M3 ? A->col_scale : nullptr};
}

// The Rayleigh-Ritz product (and the Nystrom B1 = A Q) read the float32 A of
// a low-precision matrix when one is given.
AView rr_view(const rpca_matrix* A) {
  if (A->dtype != RPCA_F32 && A->data_f32)
    return {A->data_f32, (int)RPCA_F32, A->ld_f32, A->m, A->n, nullptr};
  return native_view(A);
}

int elem_bytes(int dtype) { return dtype == RPCA_F32 ? 4 : (dtype == RPCA_BF16 ? 2 : 1); }

// packed-operand steps for ``rows`` rows: K16 steps rounded up to whole
// stages of every pass kernel (8 steps = 128 rows)
int64_t pack_steps(int64_t rows) { return round_up(ceil_div(rows, 16), 8); }

// Buffer sizes do not depend on the tile configuration: the partials and the
// tournament buffers are sized for every configuration the autotuner tries.
void layout(Arena& ar, Work& w, int64_t m, int64_t n, int l, int num_cus, bool need_y2,
            int dtype, const TuneCfg* cfg = nullptr) {
  w.cfg = cfg ? *cfg : TuneCfg{};
  w.l = l;
  w.lp = lp_of(l);
  w.nb = w.lp / 32;
  const int lp = w.lp;
  const int64_t rmax = std::max(m, n);
  w.rows_max = rmax;
  w.Y = ar.take<float>((size_t)round_up(m, 32) * lp);
  w.Z = ar.take<float>((size_t)round_up(n, 32) * lp);
  if (need_y2) w.Y2 = ar.take<float>((size_t)round_up(m, 32) * lp);
  w.Bk = ar.take<float>((size_t)round_up(rmax, 32) * lp);
  if (dtype >= 0) {  // dense A: packed operand and split partials of A^T X
    w.Xp = ar.take<__bf16>(packed_bytes(pack_steps(rmax), w.nb) / sizeof(__bf16));
    w.atx = plan_atx(m, n, w.nb, num_cus, dtype, &w.cfg);
    w.atx_rr = plan_atx(m, n, w.nb, num_cus, RPCA_F32, &w.cfg);
    w.P = ar.take<float>(std::max(atx_partial_bytes_max(m, n, w.nb, num_cus, dtype),
                                  atx_partial_bytes_max(m, n, w.nb, num_cus, RPCA_F32)) /
                         sizeof(float));
  }
  w.mu = ar.take<float>(128);
  w.colpart = ar.take<double>((size_t)colmean_blocks(rmax) * 128);
  w.colpart2 = ar.take<double>((size_t)colmean_blocks(rmax) * 128);
  w.gpart = ar.take<double>((size_t)gram_blocks(rmax) * lp * lp);
  w.G = ar.take<double>((size_t)lp * lp);
  w.Rf = ar.take<float>((size_t)lp * lp);
  w.lu_m = plan_lu(m, lp, w.cfg.lu_rows);
  w.lu_n = plan_lu(n, lp, w.cfg.lu_rows);
  int64_t cand = 0;
  w.lu_ctr = 0;
  for (int r : {256, 512, 1024}) {
    const LuPlan a = plan_lu(m, lp, r), b = plan_lu(n, lp, r);
    cand = std::max({cand, a.cand_total, b.cand_total});
    w.lu_ctr = std::max({w.lu_ctr, a.counter_total, b.counter_total});
  }
  w.cand = ar.take<int>((size_t)cand);
  w.piv = ar.take<int>(128);
  w.Ulu = ar.take<float>((size_t)lp * lp);
  w.state = ar.take<int>(16);
  w.sv = ar.take<double>(128);
  w.Wacc = ar.take<double>((size_t)lp * lp);
  w.Xn = ar.take<double>((size_t)lp * lp);
  w.jwork = ar.take<double>((size_t)2 * lp * lp);
  w.signwork = ar.take<int>(sign_work_bytes(rmax) / sizeof(int) + 4);
  w.scal = ar.take<double>(4);
  w.nu_f = ar.take<float>(4);
}

int ceil_log2(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}

std::array<int, 4> tune_key(int64_t m, int64_t n, int lp, int dtype) {
  return {ceil_log2(m), ceil_log2(n), lp, dtype};
}

const TuneCfg* tune_lookup(rpca_ctx ctx, int64_t m, int64_t n, int l, int dtype) {
  auto it = ctx->tune.find(tune_key(m, n, lp_of(l), dtype));
  return it == ctx->tune.end() ? nullptr : &it->second;
}

// RPCA_DETERMINISTIC: the built-in tile configurations, whatever the autotuner
// has stored (they fix every summation order and pivot tournament).
const TuneCfg kBuiltin{};

rpca_status prepare(rpca_ctx ctx, Work& w, int64_t m, int64_t n, int l, bool need_y2,
                    int dtype = RPCA_F32, const TuneCfg* force = nullptr) {
  const TuneCfg* cfg = force ? force : tune_lookup(ctx, m, n, l, dtype);
  Arena probe;
  layout(probe, w, m, n, l, ctx->num_cus, need_y2, dtype, cfg);
  rpca_status s = ensure_ws(ctx, probe.off + 256);
  if (s != RPCA_OK) return s;
  s = ensure_counters(ctx, (size_t)w.lu_ctr + 16);
  if (s != RPCA_OK) return s;
  Arena real;
  real.base = ctx->ws;
  layout(real, w, m, n, l, ctx->num_cus, need_y2, dtype, cfg);
  return RPCA_OK;
}

bool is_sparse(const rpca_matrix* A) { return A->format == RPCA_SPARSE_CSR; }

// layout argument: the dense copy's dtype, or -1 for a sparse A
int layout_kind(const rpca_matrix* A) { return is_sparse(A) ? -1 : (int)A->dtype; }

// need_t: the call applies A^T, so the CSC arrays must be there
rpca_status check_sparse(rpca_ctx ctx, const rpca_matrix* A, bool need_t) {
  if (A->dtype != RPCA_F32 && A->dtype != RPCA_BF16)
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "sparse values must be float32 or bfloat16");
  if (A->nnz < 0 || A->nnz > INT32_MAX) return fail(ctx, RPCA_ERR_INVALID_ARG, "nnz out of range");
  if (A->m > INT32_MAX || A->n > INT32_MAX)
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "sparse dimensions above 2^31 - 1");
  if (!A->row_ptr || (A->nnz > 0 && (!A->col_idx || !A->val)))
    return fail(ctx, RPCA_ERR_INVALID_ARG, "CSR arrays missing");
  if (need_t && (!A->col_ptr || (A->nnz > 0 && (!A->row_idx || !A->val_t))))
    return fail(ctx, RPCA_ERR_INVALID_ARG, "CSC arrays (A^T) missing");
  return RPCA_OK;
}

rpca_status check_matrix(rpca_ctx ctx, const rpca_matrix* A, bool need_t = true) {
  if (!A) return fail(ctx, RPCA_ERR_INVALID_ARG, "A is null");
  if (A->m <= 0 || A->n <= 0) return fail(ctx, RPCA_ERR_INVALID_ARG, "A must have m, n >= 1");
  if (is_sparse(A)) return check_sparse(ctx, A, need_t);
  if (A->format != RPCA_DENSE_ROWMAJOR)
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "unknown matrix format");
  if (!A->data) return fail(ctx, RPCA_ERR_INVALID_ARG, "A->data is null");
  if (A->ld < A->n) return fail(ctx, RPCA_ERR_INVALID_ARG, "A->ld < n");
  if (A->dtype == RPCA_BF16 || A->dtype == RPCA_FP8_E4M3) {
    if (!lp_shape_ok(A->data, A->dtype, A->ld, A->n))
      return fail(ctx, RPCA_ERR_UNSUPPORTED,
                  "low-precision A needs n and ld multiples of 16 bytes and 16-byte alignment");
    if (A->dtype == RPCA_FP8_E4M3 && !A->col_scale)
      return fail(ctx, RPCA_ERR_INVALID_ARG, "E4M3 A needs col_scale");
    if (A->data_f32 && A->ld_f32 < A->n) return fail(ctx, RPCA_ERR_INVALID_ARG, "A->ld_f32 < n");
  } else if (A->dtype != RPCA_F32) {
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "unknown dtype");
  }
  if (A->m > (int64_t)1 << 30 || A->n > (int64_t)1 << 30)
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "dimensions above 2^30");
  return RPCA_OK;
}

// ---- timed A-pass launches -------------------------------------------------
void begin_timed(rpca_ctx ctx, TimedLaunch& t, int kind, double bytes) {
  t.a = t.b = nullptr;
  t.kind = kind;
  t.bytes = bytes;
  if (!ctx->timing) return;
  t.a = take_event(ctx);
  t.b = take_event(ctx);
  if (t.a) (void)hipEventRecord(t.a, ctx->stream);
}
void end_timed(rpca_ctx ctx, TimedLaunch& t) {
  if (!ctx->timing || !t.a || !t.b) return;
  (void)hipEventRecord(t.b, ctx->stream);
  ctx->pending.push_back(t);
}

// Algorithmic bytes of one pass: A once, the packed operand once (4 bytes a
// value for the float32 kernels' hi/lo pairs, 2 for the high part alone),
// the output once.
void run_ax(rpca_ctx ctx, const AView& A, const Work& w, const __bf16* Xp, float* Y) {
  TimedLaunch t;
  const double xb = (A.dtype == RPCA_F32) ? 4.0 : 2.0;
  const double bytes = (double)A.m * A.n * elem_bytes(A.dtype) + (double)A.n * w.lp * xb +
                       (double)A.m * w.lp * 4.0;
  begin_timed(ctx, t, A.dtype == RPCA_F32 ? 0 : 2, bytes);
  if (A.dtype == RPCA_F32)
    launch_ax(ctx->stream, A.data, A.dtype, A.ld, A.m, A.n, Xp, Y, w.lp, w.nb, ctx->num_cus,
              &w.cfg);
  else
    launch_ax_lp(ctx->stream, A.data, A.dtype, A.ld, A.m, A.n, Xp, Y, w.lp, w.nb, ctx->num_cus,
                 &w.cfg);
  end_timed(ctx, t);
  ctx->stats.a_passes++;
}

void run_atx(rpca_ctx ctx, const AView& A, const Work& w, const __bf16* Qp) {
  TimedLaunch t;
  const AtxPlan& plan = (A.dtype == RPCA_F32) ? w.atx_rr : w.atx;
  const double xb = (A.dtype == RPCA_F32) ? 4.0 : 2.0;
  const double bytes = (double)A.m * A.n * elem_bytes(A.dtype) + (double)A.m * w.lp * xb +
                       (double)plan.partial_bytes;
  begin_timed(ctx, t, A.dtype == RPCA_F32 ? 1 : 3, bytes);
  if (A.dtype == RPCA_F32)
    launch_atx(ctx->stream, A.data, A.dtype, A.ld, A.m, A.n, Qp, w.P, plan, w.nb);
  else
    launch_atx_lp(ctx->stream, A.data, A.dtype, A.ld, A.m, A.n, Qp, w.P, plan, w.nb);
  end_timed(ctx, t);
  ctx->stats.a_passes++;
}

// Y (rows x lp) <- P L with Y = P L U (tournament-pivoted LU), in place.
void lu_renorm(rpca_ctx ctx, Work& w, float* Y, int64_t rows) {
  const LuPlan plan = plan_lu(rows, w.lp, w.cfg.lu_rows);
  launch_lu_tree(ctx->stream, Y, w.lp, rows, w.l, plan, w.cand, ctx->counters, w.Ulu, w.piv);
  launch_trsm(ctx->stream, Y, w.lp, rows, w.l, w.lp, w.Ulu, w.piv, nullptr, nullptr, nullptr, 0,
              ctx->num_cus);
}

// Y (rows x lp) <- Q with Y = Q R, Q orthonormal (Cholesky QR, float64 Gram,
// shifted and completed when Y is numerically rank deficient).  With
// ``want_r`` the l x l factor R = Q^T Y_in is formed in float64 into w.G
// (the exact projection of the input onto the final basis; upper triangular
// up to rounding).  ``single``: one Cholesky QR pass when its factorization
// needs no shift (the renormalization between applications of A, where only
// the span and a well-conditioned basis matter); the repair passes run, as
// in the orthonormalizing form, when it does.
void orth_renorm(rpca_ctx ctx, Work& w, float* Y, int64_t rows, bool want_r, uint64_t seed,
                 bool single = false) {
  hipStream_t st = ctx->stream;
  if (want_r)
    launch_copy(st, w.Bk, Y, rows * w.lp);
  for (int pass = 1; pass <= 4; ++pass) {
    const int* skip = (pass >= 3) ? (w.state + 1) : ((pass == 2 && single) ? w.state : nullptr);
    launch_gram(st, Y, w.lp, rows, w.lp, nullptr, 0, w.gpart, w.G, skip);
    launch_chol_qr_step(st, w.G, w.l, w.lp, pass, w.Rf, w.state, single);
    launch_trsm(st, Y, w.lp, rows, w.l, w.lp, w.Rf, nullptr, skip, nullptr, nullptr, 0, ctx->num_cus);
    if (pass == 2) launch_complete(st, Y, w.lp, rows, w.l, w.state, seed ^ 0x5bd1e995u);
  }
  if (want_r) launch_gram(st, Y, w.lp, rows, w.lp, w.Bk, w.lp, w.gpart, w.G, nullptr);
}

// The renormalization between applications of A and A* selected by the flags.
void renorm_mid(rpca_ctx ctx, Work& w, float* T, int64_t rows, unsigned kind, uint64_t seed) {
  if (kind & RPCA_RENORM_LU) lu_renorm(ctx, w, T, rows);
  else if (kind & RPCA_RENORM_ORTH) orth_renorm(ctx, w, T, rows, false, seed);
  else orth_renorm(ctx, w, T, rows, false, seed, true);
}

void center_rows(rpca_ctx ctx, Work& w, float* Y, int64_t rows) {
  launch_colmean(ctx->stream, Y, w.lp, rows, w.l, w.colpart, 0, w.mu);
  launch_sub_rowvec(ctx->stream, Y, w.lp, rows, w.l, w.mu);
}

// Q (m side) -> packed operand for A^T Q; centered when asked (A_c^T Q = A^T (Q - 1 qbar)).
void pack_m_side(rpca_ctx ctx, Work& w, const float* Q, int64_t m, bool center) {
  const float* mu = nullptr;
  if (center) {
    launch_colmean(ctx->stream, Q, w.lp, m, w.l, w.colpart, 0, w.mu);
    mu = w.mu;
  }
  launch_pack(ctx->stream, Q, w.lp, m, w.l, w.nb, mu, nullptr, w.Xp, pack_steps(m));
}

// X (n side) -> packed operand for A X; E4M3 column scales fold into X's rows.
void pack_n_side(rpca_ctx ctx, Work& w, const float* X, int64_t n, const AView& A) {
  launch_pack(ctx->stream, X, w.lp, n, w.l, w.nb, nullptr, A.scale, w.Xp, pack_steps(n));
}

void apply_at(rpca_ctx ctx, const AView& A, Work& w, float* Z) {
  run_atx(ctx, A, w, w.Xp);
  const AtxPlan& plan = (A.dtype == RPCA_F32) ? w.atx_rr : w.atx;
  launch_atx_reduce(ctx->stream, w.P, plan, w.nb, A.n, A.scale, Z, w.lp);
}

// Sparse passes: compulsory bytes are the index and value arrays, the
// operand and the output once each.
void run_spmm(rpca_ctx ctx, const rpca_matrix* A, bool trans, const Work& w, const float* X,
              float* Y) {
  TimedLaunch t;
  const int64_t nrows = trans ? A->n : A->m, ncols = trans ? A->m : A->n;
  const double vb = (A->dtype == RPCA_BF16) ? 2.0 : 4.0;
  const double bytes = (double)(nrows + 1) * 4.0 + (double)A->nnz * (4.0 + vb) +
                       (double)ncols * w.lp * 4.0 + (double)nrows * w.lp * 4.0;
  begin_timed(ctx, t, trans ? 1 : 0, bytes);
  if (trans)
    launch_spmm(ctx->stream, A->col_ptr, A->row_idx, A->val_t, A->dtype, nrows, A->nnz,
                (int)ncols, X, w.lp, Y, w.lp, w.lp);
  else
    launch_spmm(ctx->stream, A->row_ptr, A->col_idx, A->val, A->dtype, nrows, A->nnz, (int)ncols,
                X, w.lp, Y, w.lp, w.lp);
  end_timed(ctx, t);
  ctx->stats.a_passes++;
}

// Y (m x lp) = A X for X (n x lp, float32, zero beyond column l)
void apply_A(rpca_ctx ctx, const rpca_matrix* A, const AView& Av, Work& w, const float* X,
             float* Y) {
  if (is_sparse(A)) {
    run_spmm(ctx, A, false, w, X, Y);
    return;
  }
  pack_n_side(ctx, w, X, A->n, Av);
  run_ax(ctx, Av, w, w.Xp, Y);
}

// Z (n x lp) = A^T Q, or A_c^T Q = A^T (Q - 1 mean(Q)) with centering
void apply_At(rpca_ctx ctx, const rpca_matrix* A, const AView& Av, Work& w, const float* Q,
              float* Z, bool center) {
  if (is_sparse(A)) {
    const float* src = Q;
    if (center) {
      launch_colmean(ctx->stream, Q, w.lp, A->m, w.l, w.colpart, 0, w.mu);
      launch_copy(ctx->stream, w.Bk, Q, A->m * w.lp);
      launch_sub_rowvec(ctx->stream, w.Bk, w.lp, A->m, w.l, w.mu);
      src = w.Bk;
    }
    run_spmm(ctx, A, true, w, src, Z);
    return;
  }
  pack_m_side(ctx, w, Q, A->m, center);
  apply_at(ctx, Av, w, Z);
}

// Z (n x lp) <- A_c^T A_c Z: both products of a power step, with no
// renormalization between them (RPCA_FUSED_ATA); w.Y holds A_c Z
void apply_AtA(rpca_ctx ctx, const rpca_matrix* A, const AView& Av, Work& w, bool center) {
  apply_A(ctx, A, Av, w, w.Z, w.Y);
  if (center) center_rows(ctx, w, w.Y, A->m);
  apply_At(ctx, A, Av, w, w.Y, w.Z, center);
}

rpca_status check_kl(rpca_ctx ctx, int k, int& l, int64_t m, int64_t n) {
  if (l <= 0) l = k + 2;
  if (k < 1) return fail(ctx, RPCA_ERR_INVALID_ARG, "k must be >= 1");
  if (k > l) return fail(ctx, RPCA_ERR_INVALID_ARG, "k must be <= l");
  if (l > std::min(m, n)) return fail(ctx, RPCA_ERR_INVALID_ARG, "l must be <= min(m, n)");
  if (l > 128) return fail(ctx, RPCA_ERR_UNSUPPORTED, "l above 128 is not supported");
  return RPCA_OK;
}

// slot (nullable, device): the problem's status entry in a batch
rpca_status svd_impl(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its, uint64_t seed,
                     unsigned flags, float* U, int64_t ldu, double* S, float* V, int64_t ldv,
                     int* slot) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_status s = check_matrix(ctx, A);
  if (s != RPCA_OK) return s;
  s = check_kl(ctx, k, l, A->m, A->n);
  if (s != RPCA_OK) return s;
  if (its < 0) return fail(ctx, RPCA_ERR_INVALID_ARG, "its must be >= 0");
  if (!U || !S || !V) return fail(ctx, RPCA_ERR_INVALID_ARG, "null output");
  if (ldu < k || ldv < k) return fail(ctx, RPCA_ERR_INVALID_ARG, "ldu/ldv must be >= k");
  const int64_t m = A->m, n = A->n;
  const bool center = (flags & RPCA_CENTER) != 0;
  const unsigned mid_kind = flags & (RPCA_RENORM_ORTH | RPCA_RENORM_LU);
  Work w;
  s = prepare(ctx, w, m, n, l, false, layout_kind(A),
              (flags & RPCA_DETERMINISTIC) ? &kBuiltin : nullptr);
  if (s != RPCA_OK) return s;
  hipStream_t st = ctx->stream;
  ctx->stats.calls++;
  // the solve's own status slots start clear
  launch_fill_zero(st, reinterpret_cast<float*>(w.state + kStRetries), 4);
  const AView Av = native_view(A);  // range finder
  const AView Ar = rr_view(A);      // Rayleigh-Ritz product
  // renormalization between applications (Section 5: LU or QR both keep the
  // span): one Cholesky QR pass by default, pivoted LU or the two-pass
  // orthonormalization on request
  auto mid_renorm = [&](float* T, int64_t rows) { renorm_mid(ctx, w, T, rows, mid_kind, seed); };

  // Omega (n x l, zero padded to lp) -> packed right operand
  launch_fill_zero(st, w.Z, n * w.lp);
  launch_gaussian(st, seed, 0u, n, l, w.Z, w.lp, nullptr, (flags & RPCA_OMEGA_UNIFORM) != 0);
  if ((flags & RPCA_FUSED_ATA) && its > 0) {
    // Z = A_c^T A_c Z its times, renormalized after each; then Y = A_c Z,
    // orthonormalized (Section 5, renormalizing every second application)
    for (int it = 1; it <= its; ++it) {
      apply_AtA(ctx, A, Av, w, center);
      mid_renorm(w.Z, n);
    }
    apply_A(ctx, A, Av, w, w.Z, w.Y);
    if (center) center_rows(ctx, w, w.Y, m);
    orth_renorm(ctx, w, w.Y, m, false, seed);
  } else {
    // Y = A Omega
    apply_A(ctx, A, Av, w, w.Z, w.Y);
    if (center) center_rows(ctx, w, w.Y, m);
    if (its == 0) orth_renorm(ctx, w, w.Y, m, false, seed);
    else mid_renorm(w.Y, m);
    for (int it = 1; it <= its; ++it) {
      // Z = A^T Q, renormalized
      apply_At(ctx, A, Av, w, w.Y, w.Z, center);
      mid_renorm(w.Z, n);
      // Y = A Q; renormalized except after the last application, which is
      // orthonormalized
      apply_A(ctx, A, Av, w, w.Z, w.Y);
      if (center) center_rows(ctx, w, w.Y, m);
      if (it < its) mid_renorm(w.Y, m);
      else orth_renorm(ctx, w, w.Y, m, false, seed);
    }
  }
  // Rayleigh-Ritz: B^T = A^T Q (n x l) = Q2 R; the one-sided Jacobi SVD
  // rotates the columns of R^T (the rows of R, which the Cholesky QR leaves
  // graded, so fewer sweeps are needed than for the columns of R):
  // R^T W = X diag(s), i.e. R = W diag(s) X^T... with the roles of the two
  // factors exchanged: R^T = X diag(s) W^T, B = R^T Q2^T = X diag(s) (Q2 W)^T
  apply_At(ctx, A, Ar, w, w.Y, w.Z, center);
  orth_renorm(ctx, w, w.Z, n, true, seed + 1);
  launch_jacobi_svd(st, w.G, l, w.lp, 1, w.sv, w.Wacc, w.Xn, w.jwork, w.state + 6, k);
  // U = Q X, V = Q2 W, S = top k
  launch_small_gemm(st, w.Y, w.lp, m, l, w.Xn, w.lp, k, U, ldu, ctx->num_cus);
  launch_small_gemm(st, w.Z, w.lp, n, l, w.Wacc, w.lp, k, V, ldv, ctx->num_cus);
  launch_finish_values(st, w.sv, k, nullptr, S, w.state, ctx->dstat, slot);
  launch_sign_fix(st, U, ldu, m, k, V, ldv, n, w.signwork);
  HIP_OK(hipGetLastError());
  if (flags & RPCA_SYNC) return sync_status(ctx);
  return RPCA_OK;
}


}  // namespace

namespace rpca {

int ctx_device(rpca_ctx ctx) { return ctx->device; }

rpca_status ctx_fail(rpca_ctx ctx, rpca_status s, const char* msg) { return fail(ctx, s, msg); }

rpca_status svd_on_workspace(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                             uint64_t seed, unsigned flags, float* U, int64_t ldu, double* S,
                             float* V, int64_t ldv, char* ws, size_t ws_bytes,
                             unsigned* counters, size_t counters_n) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_status s = check_matrix(ctx, A);
  if (s != RPCA_OK) return s;
  s = check_kl(ctx, k, l, A->m, A->n);
  if (s != RPCA_OK) return s;
  // the sizes svd_impl's prepare() will ask for (independent of the tiles)
  Work w;
  Arena probe;
  layout(probe, w, A->m, A->n, l, ctx->num_cus, false, layout_kind(A));
  const size_t need = probe.off + 256, need_ctr = (size_t)w.lu_ctr + 16;
  if (need > ws_bytes || need_ctr > counters_n)
    return fail(ctx, RPCA_ERR_NO_MEMORY,
                "rpca_svd_noalloc: this problem needs " + std::to_string(need) +
                    " bytes of scratch and " + std::to_string(need_ctr) +
                    " counters; the static scratch holds " + std::to_string(ws_bytes) +
                    " bytes and " + std::to_string(counters_n) + " counters");
  // the tournament's arrival counters start at zero (a kernel node, not a memset)
  launch_fill_zero(ctx->stream, reinterpret_cast<float*>(counters),
                   round_up((int64_t)need_ctr, 4));
  char* const ws0 = ctx->ws;
  const size_t wsb0 = ctx->ws_bytes;
  unsigned* const ctr0 = ctx->counters;
  const size_t ctrn0 = ctx->counters_n;
  const bool timing0 = ctx->timing;
  ctx->ws = ws;
  ctx->ws_bytes = ws_bytes;
  ctx->counters = counters;
  ctx->counters_n = counters_n;
  ctx->timing = false;  // event pairs could need creating
  s = svd_impl(ctx, A, k, l, its, seed, flags, U, ldu, S, V, ldv, nullptr);
  ctx->ws = ws0;
  ctx->ws_bytes = wsb0;
  ctx->counters = ctr0;
  ctx->counters_n = ctrn0;
  ctx->timing = timing0;
  return s;
}

}  // namespace rpca

// ============================================================================
// C ABI
// ============================================================================
extern "C" {

const char* rpca_status_str(rpca_status s) {
  switch (s) {
    case RPCA_OK: return "ok";
    case RPCA_ERR_INVALID_ARG: return "invalid argument";
    case RPCA_ERR_UNSUPPORTED: return "unsupported";
    case RPCA_ERR_NO_MEMORY: return "out of memory";
    case RPCA_ERR_HIP: return "HIP error";
    case RPCA_ERR_NOT_PSD: return "matrix not positive semidefinite";
    case RPCA_ERR_NUMERICAL: return "non-finite values";
    case RPCA_ERR_TIMEOUT: return "device wait timed out";
  }
  return "unknown status";
}

const char* rpca_last_error(rpca_ctx ctx) { return ctx ? ctx->err.c_str() : "null context"; }

rpca_status rpca_create(rpca_ctx* out, void* hip_stream) {
  if (!out) return RPCA_ERR_INVALID_ARG;
  *out = nullptr;
  rpca_ctx ctx = new (std::nothrow) rpca_ctx_s();
  if (!ctx) return RPCA_ERR_NO_MEMORY;
  ctx->stream = static_cast<hipStream_t>(hip_stream);
  if (hipGetDevice(&ctx->device) != hipSuccess) {
    delete ctx;
    return RPCA_ERR_HIP;
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, ctx->device) == hipSuccess && prop.multiProcessorCount > 0)
    ctx->num_cus = prop.multiProcessorCount;
  void* hs = nullptr;
  if (hipHostMalloc(&hs, 64 * sizeof(int), hipHostMallocDefault) != hipSuccess) {
    delete ctx;
    return RPCA_ERR_HIP;
  }
  ctx->host_state = static_cast<int*>(hs);
  void* ds = nullptr;
  if (hipMalloc(&ds, 64 * sizeof(int)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipHostFree(hs);
    delete ctx;
    return RPCA_ERR_NO_MEMORY;
  }
  if (hipMemset(ds, 0, 64 * sizeof(int)) != hipSuccess) {
    (void)hipFree(ds);
    (void)hipHostFree(hs);
    delete ctx;
    return RPCA_ERR_HIP;
  }
  ctx->dstat = static_cast<int*>(ds);
  *out = ctx;
  return RPCA_OK;
}

rpca_status rpca_destroy(rpca_ctx ctx) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  (void)hipStreamSynchronize(ctx->stream);
  for (auto& t : ctx->pending) {
    (void)hipEventDestroy(t.a);
    (void)hipEventDestroy(t.b);
  }
  for (auto e : ctx->event_pool) (void)hipEventDestroy(e);
  if (ctx->ws) (void)hipFree(ctx->ws);
  if (ctx->counters) (void)hipFree(ctx->counters);
  if (ctx->host_state) (void)hipHostFree(ctx->host_state);
  if (ctx->dstat) (void)hipFree(ctx->dstat);
  if (ctx->bstat) (void)hipFree(ctx->bstat);
  for (auto& b : ctx->slots) {
    if (b.stream) (void)hipStreamSynchronize(b.stream);
    if (b.ws) (void)hipFree(b.ws);
    if (b.counters) (void)hipFree(b.counters);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.stream) (void)hipStreamDestroy(b.stream);
  }
  if (ctx->fork) (void)hipEventDestroy(ctx->fork);
  if (ctx->pers_tab) (void)hipFree(ctx->pers_tab);
  if (ctx->pers_counter) (void)hipFree(ctx->pers_counter);
  if (ctx->pers_ws) (void)hipFree(ctx->pers_ws);
  if (ctx->pers_sh) (void)hipFree(ctx->pers_sh);
  if (ctx->pers_bar) (void)hipFree(ctx->pers_bar);
  for (void* q : ctx->pers_retired) (void)hipFree(q);
  delete ctx;
  return RPCA_OK;
}

rpca_status rpca_set_stream(rpca_ctx ctx, void* hip_stream) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (ctx->stream != static_cast<hipStream_t>(hip_stream)) {
    HIP_OK(hipStreamSynchronize(ctx->stream));
    ctx->stream = static_cast<hipStream_t>(hip_stream);
  }
  return RPCA_OK;
}

rpca_status rpca_set_workspace_limit(rpca_ctx ctx, size_t bytes) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  ctx->ws_limit = bytes;
  return RPCA_OK;
}

rpca_status rpca_workspace_size(rpca_ctx ctx, const rpca_matrix* A, int k, int l, size_t* bytes) {
  if (!ctx || !bytes) return fail(ctx, RPCA_ERR_INVALID_ARG, "null argument");
  rpca_status s = check_matrix(ctx, A);
  if (s != RPCA_OK) return s;
  s = check_kl(ctx, k, l, A->m, A->n);
  if (s != RPCA_OK) return s;
  Work w;
  Arena probe;
  layout(probe, w, A->m, A->n, l, ctx->num_cus, true, layout_kind(A));
  *bytes = probe.off + 256;
  return RPCA_OK;
}

rpca_status rpca_quantize(rpca_ctx ctx, const float* A, int64_t m, int64_t n, int64_t lda,
                          rpca_dtype dtype, void* out, int64_t ldo, float* col_scale) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (!A || !out || m < 1 || n < 1 || lda < n || ldo < n)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "bad quantize arguments");
  if (dtype != RPCA_BF16 && dtype != RPCA_FP8_E4M3)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "quantize: dtype must be RPCA_BF16 or RPCA_FP8_E4M3");
  if (dtype == RPCA_FP8_E4M3 && !col_scale)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "quantize: E4M3 needs col_scale");
  if (m * n > ((int64_t)1 << 40)) return fail(ctx, RPCA_ERR_UNSUPPORTED, "quantize: too large");
  if (dtype == RPCA_FP8_E4M3) {
    rpca_status s = ensure_ws(ctx, quantize_work_bytes(m, n) + 256);
    if (s != RPCA_OK) return s;
  }
  launch_quantize(ctx->stream, A, lda, m, n, dtype, out, ldo, col_scale,
                  reinterpret_cast<float*>(ctx->ws));
  HIP_OK(hipGetLastError());
  return RPCA_OK;
}

rpca_status rpca_gaussian(rpca_ctx ctx, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                          float* out, int64_t ldo, uint32_t* words_out) {
  if (!ctx || !out || n < 0 || l < 0 || ldo < l) return fail(ctx, RPCA_ERR_INVALID_ARG, "bad arguments");
  launch_gaussian(ctx->stream, seed, stream, n, l, out, ldo, words_out);
  HIP_OK(hipGetLastError());
  return RPCA_OK;
}

rpca_status rpca_uniform(rpca_ctx ctx, uint64_t seed, uint32_t stream, int64_t n, int64_t l,
                         float* out, int64_t ldo) {
  if (!ctx || !out || n < 0 || l < 0 || ldo < l) return fail(ctx, RPCA_ERR_INVALID_ARG, "bad arguments");
  launch_gaussian(ctx->stream, seed, stream, n, l, out, ldo, nullptr, true);
  HIP_OK(hipGetLastError());
  return RPCA_OK;
}

rpca_status rpca_svd(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its, uint64_t seed,
                     unsigned flags, float* U, int64_t ldu, double* S, float* V, int64_t ldv) {
  return svd_impl(ctx, A, k, l, its, seed, flags, U, ldu, S, V, ldv, nullptr);
}

}  // extern "C"

namespace {
// slot (nullable, device): the problem's status entry in a batch.  Whether
// the shifted factor was found is known on the device only: it reaches the
// caller at the next synchronizing call (RPCA_SYNC here, rpca_sync, ...).
// sym: the Rayleigh-Ritz eigenpairs of a general self-adjoint A (rpca_eig_sym)
// instead of the Nystrom method
rpca_status eig_psd_impl(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its,
                         uint64_t seed, unsigned flags, float* U, int64_t ldu, double* lambda,
                         int* slot, bool sym = false) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_status s = check_matrix(ctx, A, false);
  if (s != RPCA_OK) return s;
  if (A->m != A->n) return fail(ctx, RPCA_ERR_INVALID_ARG, "eig_psd / eig_sym need a square matrix");
  s = check_kl(ctx, k, l, A->m, A->n);
  if (s != RPCA_OK) return s;
  if (its < 0) return fail(ctx, RPCA_ERR_INVALID_ARG, "its must be >= 0");
  if (!U || !lambda) return fail(ctx, RPCA_ERR_INVALID_ARG, "null output");
  if (ldu < k) return fail(ctx, RPCA_ERR_INVALID_ARG, "ldu must be >= k");
  if (flags & RPCA_CENTER) return fail(ctx, RPCA_ERR_INVALID_ARG, "centering does not apply to eig_psd");
  if (flags & RPCA_FUSED_ATA)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "RPCA_FUSED_ATA applies to rpca_svd only");
  const int64_t n = A->n;
  Work w;
  s = prepare(ctx, w, n, n, l, true, layout_kind(A),
              (flags & RPCA_DETERMINISTIC) ? &kBuiltin : nullptr);
  if (s != RPCA_OK) return s;
  hipStream_t st = ctx->stream;
  ctx->stats.calls++;
  launch_fill_zero(st, reinterpret_cast<float*>(w.state + kStRetries), 4);
  const AView Av = native_view(A);  // the self-adjoint range finder
  const AView Ar = rr_view(A);      // B1 = A Q

  // Q = Omega; its times Q = A Q renormalized (LU, QR after the last).
  launch_fill_zero(st, w.Y, n * w.lp);
  launch_gaussian(st, seed, 0u, n, l, w.Y, w.lp, nullptr, (flags & RPCA_OMEGA_UNIFORM) != 0);
  if (its == 0) orth_renorm(ctx, w, w.Y, n, false, seed);
  for (int it = 1; it <= its; ++it) {
    apply_A(ctx, A, Av, w, w.Y, w.Y2);
    launch_copy(st, w.Y, w.Y2, n * w.lp);
    if (it < its) renorm_mid(ctx, w, w.Y, n, flags & (RPCA_RENORM_ORTH | RPCA_RENORM_LU), seed);
    else orth_renorm(ctx, w, w.Y, n, false, seed);
  }
  // B1 = A Q (start); B2 = Q* B1 (second)
  apply_A(ctx, A, Ar, w, w.Y, w.Y2);
  launch_fro2_d(st, w.Y2, w.lp, n, l, w.colpart, w.colpart2, w.scal);
  launch_gram(st, w.Y, w.lp, n, w.lp, w.Y2, w.lp, w.gpart, w.G, nullptr);
  if (sym) {
    // Rayleigh-Ritz for a self-adjoint A: B2 = W diag(lambda) W^T (Jacobi SVD
    // of the symmetrized B2, signs from W^T X), U = Q W, the k eigenvalues
    // largest in magnitude
    launch_symmetrize(st, w.G, l, w.lp);
    launch_jacobi_svd(st, w.G, l, w.lp, 0, w.sv, w.Wacc, w.Xn, w.jwork, w.state + 6, k);
    launch_small_gemm(st, w.Y, w.lp, n, l, w.Wacc, w.lp, k, U, ldu, ctx->num_cus);
    launch_sym_eig_finish(st, w.sv, w.Wacc, w.Xn, l, k, w.lp, lambda, w.state, ctx->dstat, slot);
    launch_sign_fix(st, U, ldu, n, k, nullptr, 0, 0, w.signwork);
    HIP_OK(hipGetLastError());
    if (flags & RPCA_SYNC) return sync_status(ctx);
    return RPCA_OK;
  }
  // unit roundoff of the product B1 = A Q: a float32 A is multiplied as three
  // bfloat16 products of split operands (about 16 significant bits), a
  // bfloat16 / E4M3 copy with the operand rounded to bfloat16 (8 bits; 4 for
  // the E4M3 values themselves)
  const double u = std::ldexp(1.0, Ar.dtype == RPCA_F32 ? -16 : (Ar.dtype == RPCA_BF16 ? -8 : -4));
  if (flags & RPCA_NYSTROM_SQRT) {
    // Section 3's square-root stabilization: C = W diag(w)^1/2 W^T from the
    // eigendecomposition B2 = W diag(w) W^T (Jacobi SVD of the symmetrized
    // B2), F = B1 C^+ with the eigenvalues below the shift's scale
    // sqrt(n) u ||B1||_F discarded.  F = (B1 W diag(w)^-1/2) W^T shares its
    // left singular pairs with F' = B1 W diag(w)^-1/2: F' = QF R, R^T's
    // Jacobi SVD, U = QF X, lambda = s^2.
    launch_symmetrize(st, w.G, l, w.lp);
    launch_jacobi_svd(st, w.G, l, w.lp, 0, w.sv, w.Wacc, w.Xn, w.jwork, w.state + 6, l);
    launch_sqrt_pinv(st, w.Wacc, w.sv, l, w.lp, w.scal, std::sqrt((double)n) * u, w.jwork);
    launch_fill_zero(st, w.Y, n * w.lp);
    launch_small_gemm(st, w.Y2, w.lp, n, l, w.jwork, w.lp, l, w.Y, w.lp, ctx->num_cus);
    launch_fill_zero(st, reinterpret_cast<float*>(w.scal + 2), 4);  // no shift to remove
    orth_renorm(ctx, w, w.Y, n, true, seed + 1);
    launch_jacobi_svd(st, w.G, l, w.lp, 1, w.sv, w.Wacc, w.Xn, w.jwork, w.state + 6, k);
    launch_small_gemm(st, w.Y, w.lp, n, l, w.Wacc, w.lp, k, U, ldu, ctx->num_cus);
    launch_finish_values(st, w.sv, k, w.scal + 2, lambda, w.state, ctx->dstat, slot);
    launch_sign_fix(st, U, ldu, n, k, nullptr, 0, 0, w.signwork);
    HIP_OK(hipGetLastError());
    if (flags & RPCA_SYNC) return sync_status(ctx);
    return RPCA_OK;
  }
  // the shift nu; C = chol(B2 + nu I) (Cholesky)
  launch_chol_nystrom(st, w.G, l, w.lp, w.scal, std::sqrt((double)n) * u, w.Rf, w.scal + 1,
                      w.nu_f, w.state, ctx->nys_retries);
  // F = (B1 + nu Q) C^-1 (pseudo), then its SVD: F = QF RF, RF^T = ...
  launch_trsm(st, w.Y2, w.lp, n, l, w.lp, w.Rf, nullptr, nullptr, w.nu_f, w.Y, w.lp, ctx->num_cus);
  orth_renorm(ctx, w, w.Y2, n, true, seed + 1);
  launch_jacobi_svd(st, w.G, l, w.lp, 1, w.sv, w.Wacc, w.Xn, w.jwork, w.state + 6, k);
  launch_small_gemm(st, w.Y2, w.lp, n, l, w.Wacc, w.lp, k, U, ldu, ctx->num_cus);
  launch_finish_values(st, w.sv, k, w.scal + 1, lambda, w.state, ctx->dstat, slot);
  launch_sign_fix(st, U, ldu, n, k, nullptr, 0, 0, w.signwork);
  HIP_OK(hipGetLastError());
  if (flags & RPCA_SYNC) return sync_status(ctx);
  return RPCA_OK;
}
}  // namespace

extern "C" {

rpca_status rpca_eig_psd(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its, uint64_t seed,
                         unsigned flags, float* U, int64_t ldu, double* lambda) {
  return eig_psd_impl(ctx, A, k, l, its, seed, flags, U, ldu, lambda, nullptr);
}

rpca_status rpca_eig_sym(rpca_ctx ctx, const rpca_matrix* A, int k, int l, int its, uint64_t seed,
                         unsigned flags, float* U, int64_t ldu, double* lambda) {
  if (flags & RPCA_NYSTROM_SQRT)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "eig_sym: RPCA_NYSTROM_SQRT applies to eig_psd");
  return eig_psd_impl(ctx, A, k, l, its, seed, flags, U, ldu, lambda, nullptr, true);
}

rpca_status rpca_spectral_err(rpca_ctx ctx, const rpca_matrix* A, int k, const float* U,
                              int64_t ldu, const double* S, const float* V, int64_t ldv, int iters,
                              uint64_t seed, unsigned flags, double* err_host) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_status s = check_matrix(ctx, A);
  if (s != RPCA_OK) return s;
  const int64_t m = A->m, n = A->n;
  if (k < 0 || k > 128) return fail(ctx, RPCA_ERR_INVALID_ARG, "spectral_err needs 0 <= k <= 128");
  if (iters < 0 || iters > 100000) return fail(ctx, RPCA_ERR_INVALID_ARG, "iters out of range");
  if (std::min(m, n) < 4) return fail(ctx, RPCA_ERR_INVALID_ARG, "spectral_err needs min(m, n) >= 4");
  if (!err_host) return fail(ctx, RPCA_ERR_INVALID_ARG, "null err_host");
  if (k > 0) {
    if (!U || !S) return fail(ctx, RPCA_ERR_INVALID_ARG, "null U or S");
    if (ldu < k) return fail(ctx, RPCA_ERR_INVALID_ARG, "ldu must be >= k");
    if (V && ldv < k) return fail(ctx, RPCA_ERR_INVALID_ARG, "ldv must be >= k");
    if (!V && m != n) return fail(ctx, RPCA_ERR_INVALID_ARG, "V == NULL needs a square A");
  }
  const bool center = (flags & RPCA_CENTER) != 0;
  const AView Ar = rr_view(A);
  if (!is_sparse(A) && Ar.dtype != RPCA_F32)
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "spectral_err reads float32 A (give data_f32)");
  SpecSparse sp{A->row_ptr, A->col_idx, A->val, A->col_ptr, A->row_idx, A->val_t,
                (int)A->dtype, A->nnz};
  const size_t wb = round_up(spectral_work_bytes(m, n, k), 256);
  s = ensure_ws(ctx, wb + 256);
  if (s != RPCA_OK) return s;
  double* result = reinterpret_cast<double*>(ctx->ws + wb);
  hipStream_t st = ctx->stream;
  launch_spectral(st, static_cast<const float*>(Ar.data), Ar.ld, m, n, center, U, ldu, S, V, ldv, k,
                  iters, seed, ctx->ws, result, is_sparse(A) ? &sp : nullptr);
  HIP_OK(hipGetLastError());
  double r = 0.0;
  HIP_OK(hipMemcpyAsync(&r, result, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_OK(hipStreamSynchronize(st));
  *err_host = r;
  return RPCA_OK;
}

rpca_status rpca_op_matmul(rpca_ctx ctx, const rpca_matrix* A, int trans, int l, const float* X,
                           int64_t ldx, float* Y, int64_t ldy, unsigned flags) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_status s = check_matrix(ctx, A, trans != 0);
  if (s != RPCA_OK) return s;
  if (l < 1 || l > 128) return fail(ctx, RPCA_ERR_INVALID_ARG, "1 <= l <= 128");
  if (!X || !Y) return fail(ctx, RPCA_ERR_INVALID_ARG, "null operand");
  const int64_t m = A->m, n = A->n;
  const int64_t xr = trans ? m : n, yr = trans ? n : m;
  if (ldx < l || ldy < l) return fail(ctx, RPCA_ERR_INVALID_ARG, "ld < l");
  const bool center = (flags & RPCA_CENTER) != 0;
  Work w;
  s = prepare(ctx, w, m, n, l, false, layout_kind(A));
  if (s != RPCA_OK) return s;
  hipStream_t st = ctx->stream;
  const AView Av = native_view(A);
  // copy X into the lp-padded tall buffer
  float* Xt = trans ? w.Y : w.Z;
  HIP_OK(hipMemsetAsync(Xt, 0, (size_t)xr * w.lp * sizeof(float), st));
  HIP_OK(hipMemcpy2DAsync(Xt, w.lp * sizeof(float), X, ldx * sizeof(float), l * sizeof(float), xr,
                          hipMemcpyDeviceToDevice, st));
  float* Yt = trans ? w.Z : w.Y;
  if (trans) {
    apply_At(ctx, A, Av, w, Xt, Yt, center);
  } else {
    apply_A(ctx, A, Av, w, Xt, Yt);
    if (center) center_rows(ctx, w, Yt, m);
  }
  HIP_OK(hipMemcpy2DAsync(Y, ldy * sizeof(float), Yt, w.lp * sizeof(float), l * sizeof(float), yr,
                          hipMemcpyDeviceToDevice, st));
  HIP_OK(hipGetLastError());
  if (flags & RPCA_SYNC) HIP_OK(hipStreamSynchronize(st));
  return RPCA_OK;
}

rpca_status rpca_op_renorm(rpca_ctx ctx, int kind, int64_t rows, int l, float* Y, int64_t ldy,
                           int32_t* piv, double* R) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (!Y || rows < l || l < 1 || l > 128 || ldy < l)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "bad renorm arguments");
  if (kind != 0 && kind != 1) return fail(ctx, RPCA_ERR_INVALID_ARG, "kind must be 0 or 1");
  Work w;
  rpca_status s = prepare(ctx, w, rows, l, l, false);
  if (s != RPCA_OK) return s;
  hipStream_t st = ctx->stream;
  HIP_OK(hipMemsetAsync(w.Y, 0, (size_t)rows * w.lp * sizeof(float), st));
  HIP_OK(hipMemcpy2DAsync(w.Y, w.lp * sizeof(float), Y, ldy * sizeof(float), l * sizeof(float),
                          rows, hipMemcpyDeviceToDevice, st));
  if (kind == 0) {
    lu_renorm(ctx, w, w.Y, rows);
    if (piv) HIP_OK(hipMemcpyAsync(piv, w.piv, l * sizeof(int), hipMemcpyDeviceToDevice, st));
  } else {
    orth_renorm(ctx, w, w.Y, rows, R != nullptr, 12345u);
    if (R)
      HIP_OK(hipMemcpy2DAsync(R, l * sizeof(double), w.G, w.lp * sizeof(double),
                              l * sizeof(double), l, hipMemcpyDeviceToDevice, st));
  }
  HIP_OK(hipMemcpy2DAsync(Y, ldy * sizeof(float), w.Y, w.lp * sizeof(float), l * sizeof(float),
                          rows, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipGetLastError());
  return RPCA_OK;
}

rpca_status rpca_op_small_svd(rpca_ctx ctx, int l, const double* M, double* s, double* W,
                              double* X) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (l < 1 || l > 128 || !M || !s || !W || !X) return fail(ctx, RPCA_ERR_INVALID_ARG, "bad arguments");
  Work w;
  rpca_status st_ = prepare(ctx, w, l, l, l, false);
  if (st_ != RPCA_OK) return st_;
  hipStream_t st = ctx->stream;
  HIP_OK(hipMemsetAsync(w.G, 0, (size_t)w.lp * w.lp * sizeof(double), st));
  HIP_OK(hipMemcpy2DAsync(w.G, w.lp * sizeof(double), M, l * sizeof(double), l * sizeof(double), l,
                          hipMemcpyDeviceToDevice, st));
  // the accumulating form at every size: this entry promises orthogonality to rounding
  launch_jacobi_svd(st, w.G, l, w.lp, 0, w.sv, w.Wacc, w.Xn, w.jwork, nullptr);
  HIP_OK(hipMemcpyAsync(s, w.sv, l * sizeof(double), hipMemcpyDeviceToDevice, st));
  // M = Xn diag(s) Wacc^T: left vectors Xn, right vectors Wacc
  HIP_OK(hipMemcpy2DAsync(W, l * sizeof(double), w.Xn, w.lp * sizeof(double), l * sizeof(double), l,
                          hipMemcpyDeviceToDevice, st));
  HIP_OK(hipMemcpy2DAsync(X, l * sizeof(double), w.Wacc, w.lp * sizeof(double), l * sizeof(double),
                          l, hipMemcpyDeviceToDevice, st));
  HIP_OK(hipGetLastError());
  return RPCA_OK;
}

rpca_status rpca_set_timing(rpca_ctx ctx, int enable) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  ctx->timing = enable != 0;
  return RPCA_OK;
}

rpca_status rpca_get_stats(rpca_ctx ctx, rpca_stats* out) {
  if (!ctx || !out) return RPCA_ERR_INVALID_ARG;
  HIP_OK(hipStreamSynchronize(ctx->stream));
  // the retry count of the last Nystrom solve (its status stays for rpca_sync)
  HIP_OK(hipMemcpyAsync(ctx->host_state, ctx->dstat, 2 * sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  ctx->stats.shift_retries = ctx->host_state[1];
  for (auto& t : ctx->pending) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.a, t.b) == hipSuccess) {
      switch (t.kind) {
        case 0: ctx->stats.ms_ax += ms; ctx->stats.n_ax++; ctx->stats.bytes_ax += t.bytes; break;
        case 1: ctx->stats.ms_atx += ms; ctx->stats.n_atx++; ctx->stats.bytes_atx += t.bytes; break;
        case 2: ctx->stats.ms_ax_lp += ms; ctx->stats.n_ax_lp++; ctx->stats.bytes_ax_lp += t.bytes; break;
        default: ctx->stats.ms_atx_lp += ms; ctx->stats.n_atx_lp++; ctx->stats.bytes_atx_lp += t.bytes; break;
      }
      ctx->stats.timed_launches++;
    }
    ctx->event_pool.push_back(t.a);
    ctx->event_pool.push_back(t.b);
  }
  ctx->pending.clear();
  *out = ctx->stats;
  return RPCA_OK;
}

rpca_status rpca_reset_stats(rpca_ctx ctx) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_stats tmp;
  rpca_status s = rpca_get_stats(ctx, &tmp);
  ctx->stats = rpca_stats{};
  return s;
}


}  // extern "C"

namespace {
struct ctx_s_pers_plan {
  std::vector<PersProblem> table;  // the split problems' shares, then the rest, largest first
  int64_t maxdim = 0;
  int grid = 0;
  int teams = 0;  // problems split over workgroups (their arrival counters)
};

// grow a device buffer outside capture; the old one is kept for graphs that use it
template <class T>
rpca_status pers_grow(rpca_ctx ctx, T*& buf, size_t bytes, const char* what) {
  void* q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) {
    (void)hipGetLastError();
    return fail(ctx, RPCA_ERR_NO_MEMORY, std::string("persistent batch: allocation of the ") +
                                             what + " failed");
  }
  if (buf) ctx->pers_retired.push_back(buf);
  buf = static_cast<T*>(q);
  return RPCA_OK;
}

// Table (largest problems first) and working memory of the persistent launch.
rpca_status pers_prepare(rpca_ctx ctx, const rpca_problem* problems, const std::vector<int>& pers,
                         bool capturing, ctx_s_pers_plan& plan) {
  std::vector<PersProblem> tab;
  std::vector<double> cost;
  int64_t maxdim = 1;
  for (int p : pers) {
    const rpca_problem& q = problems[p];
    const rpca_matrix* A = q.A;
    PersProblem e{};
    e.A = static_cast<const float*>(A->data);
    e.lda = A->ld;
    e.U = q.U;
    e.ldu = q.ldu;
    e.S = q.S;
    e.V = q.kind == 0 ? q.V : nullptr;
    e.ldv = q.kind == 0 ? q.ldv : 0;
    e.seed = q.seed;
    e.m = (int32_t)A->m;
    e.n = (int32_t)A->n;
    e.kind = q.kind;
    e.k = q.k;
    e.l = q.l > 0 ? q.l : q.k + 2;
    e.its = q.its;
    e.center = (q.flags & RPCA_CENTER) ? 1 : 0;
    e.mid = (q.flags & RPCA_RENORM_LU) ? 1 : ((q.flags & RPCA_RENORM_ORTH) ? 2 : 0);
    e.uniform = (q.flags & RPCA_OMEGA_UNIFORM) ? 1 : 0;
    e.status = ctx->bstat + p;
    e.gstatus = ctx->dstat;
    e.parts = 1;
    e.part = 0;
    tab.push_back(e);
    // the work of the problem on one workgroup (ns): passes over A, and the
    // steps on the tall m x lp and n x lp matrices (renormalizations, packs,
    // Gram matrices) -- a fit to single-problem times on MI355X (median error
    // 10% on the 512-problem workload)
    const double lpf = e.l <= 32 ? 32.0 : 64.0;
    const double passes = q.kind == 0 ? 2.0 * q.its + 2.0 : q.its + 1.0;
    const double steps = q.kind == 0 ? 2.0 * q.its + 2.0 : q.its + 2.0;
    const double side = q.kind == 0 ? (double)(A->m + A->n) : 2.0 * (double)A->n;
    cost.push_back(0.1667 * passes * (double)A->m * (double)A->n * lpf / 64.0 +
                   1.213 * steps * side * lpf);
    maxdim = std::max<int64_t>(maxdim, std::max(A->m, A->n));
  }
  // Teams.  A problem takes about kFixed + work on one workgroup and
  // kTeamFixed + work / g as a share of a team of g (the waits and the l x l
  // steps every share repeats).  For a few targets T, every problem whose
  // single-workgroup time exceeds T gets the g that brings its shares under
  // T (at most split_max_parts, one per 64 rows of its smaller side, and all
  // shares within one round of the grid); the launch's list scheduling --
  // the shares first, then the other problems by decreasing cost, each to the
  // first free workgroup -- is simulated and the T with the shortest
  // simulated makespan is kept.
  const double kFixed = 450e3, kTeamFixed = 900e3;
  const int nprob = (int)tab.size();
  const int slots = std::max(1, ctx->num_cus);
  double total = 0.0;
  for (double c : cost) total += c + kFixed;
  auto split_for = [&](double T, std::vector<int>& parts) {
    int shares = 0;
    for (int i = 0; i < nprob; ++i) {
      const PersProblem& e = tab[i];
      int g = 1;
      if (ctx->split_max_parts > 1 && e.mid != 1 && cost[i] + kFixed > T && T > kTeamFixed) {
        const int64_t cap = std::min<int64_t>(ctx->split_max_parts, std::min(e.m, e.n) / 64);
        g = (int)std::min<double>(std::ceil(cost[i] / (T - kTeamFixed)), (double)cap);
      }
      parts[i] = g < 2 ? 1 : g;
      if (parts[i] > 1) shares += parts[i];
    }
    return shares;
  };
  auto simulate = [&](const std::vector<int>& parts) {
    std::vector<double> items;
    for (int i = 0; i < nprob; ++i)
      if (parts[i] > 1)
        for (int g = 0; g < parts[i]; ++g) items.push_back(kTeamFixed + cost[i] / parts[i]);
    std::vector<double> rest;
    for (int i = 0; i < nprob; ++i)
      if (parts[i] < 2) rest.push_back(kFixed + cost[i]);
    std::sort(rest.begin(), rest.end(), std::greater<double>());
    items.insert(items.end(), rest.begin(), rest.end());
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (int w = 0; w < std::min<int>(slots, (int)items.size()); ++w) free_at.push(0.0);
    double span = 0.0;
    for (double t : items) {
      const double s0 = free_at.top();
      free_at.pop();
      free_at.push(s0 + t);
      span = std::max(span, s0 + t);
    }
    return span;
  };
  std::vector<int> parts(nprob, 1), trial(nprob, 1);
  double best = simulate(parts);
  // targets: multiples of the average load, the times that cut the largest
  // problem into 2 .. split_max_parts shares, and short ones that split every
  // problem worth splitting (a small batch leaves workgroups idle)
  std::vector<double> targets;
  const double avg = total / slots;
  for (double f : {0.5, 0.65, 0.8, 1.0, 1.25, 1.6, 2.0}) targets.push_back(f * avg);
  const double cmax = nprob ? *std::max_element(cost.begin(), cost.end()) : 0.0;
  for (int g = 2; g <= ctx->split_max_parts; ++g) targets.push_back(kTeamFixed + cmax / g + 1.0);
  for (double f : {1.25, 1.5, 2.0, 3.0}) targets.push_back(f * kTeamFixed);
  for (double T : targets) {
    if (split_for(T, trial) > slots) continue;
    const double span = simulate(trial);
    if (span < best) {
      best = span;
      parts = trial;
    }
  }
  // the caller's minimum number of shares for every problem that can be split
  if (ctx->split_min_parts > 1) {
    trial = parts;
    int shares = 0;
    for (int i = 0; i < nprob; ++i) {
      const PersProblem& e = tab[i];
      const int64_t cap = std::min<int64_t>(ctx->split_max_parts, std::min(e.m, e.n) / 64);
      if (e.mid != 1 && cap >= 2)
        trial[i] = (int)std::max<int64_t>(trial[i], std::min<int64_t>(ctx->split_min_parts, cap));
      if (trial[i] > 1) shares += trial[i];
    }
    if (shares <= slots) parts = trial;
  }
  std::vector<int> ord(nprob);
  for (int i = 0; i < nprob; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) {
    if ((parts[a] > 1) != (parts[b] > 1)) return parts[a] > 1;
    return cost[a] > cost[b];
  });
  int64_t sh_need = 0;
  int teams = 0;
  std::vector<int64_t> sh_off(nprob, -1);
  for (int i : ord) {
    if (parts[i] < 2) continue;
    const PersProblem& e = tab[i];
    sh_off[i] = sh_need;
    sh_need += round_up(team_floats(parts[i], round_up(std::max(e.m, e.n), 64),
                                    round_up(e.n, 64)), 64);
    ++teams;
  }
  const int cnt_items = [&] {
    int c = 0;
    for (int i = 0; i < nprob; ++i) c += parts[i];
    return c;
  }();
  const int cnt = cnt_items;
  const int grid = (int)std::min<int64_t>(cnt, ctx->num_cus);
  const int64_t need = (int64_t)grid * pers_slot_floats(maxdim);
  if (ctx->pers_ws_floats < need || ctx->pers_tab_cap < cnt || !ctx->pers_counter ||
      ctx->pers_sh_floats < sh_need || ctx->pers_bar_cap < teams) {
    if (capturing) return fail(ctx, RPCA_ERR_UNSUPPORTED, "run the batch once before capturing it");
    if (ctx->ws_limit && (size_t)(need + sh_need) * sizeof(float) > ctx->ws_limit)
      return fail(ctx, RPCA_ERR_NO_MEMORY, "batch workspace exceeds the limit");
    HIP_OK(hipStreamSynchronize(ctx->stream));
    rpca_status s = RPCA_OK;
    if (ctx->pers_ws_floats < need) {
      s = pers_grow(ctx, ctx->pers_ws, (size_t)need * sizeof(float), "working memory");
      if (s != RPCA_OK) return s;
      ctx->pers_ws_floats = need;
    }
    if (ctx->pers_tab_cap < cnt) {
      s = pers_grow(ctx, ctx->pers_tab, (size_t)cnt * sizeof(PersProblem), "problem table");
      if (s != RPCA_OK) return s;
      ctx->pers_tab_cap = cnt;
    }
    if (!ctx->pers_counter) {
      s = pers_grow(ctx, ctx->pers_counter, 256, "work counter");
      if (s != RPCA_OK) return s;
    }
    if (ctx->pers_sh_floats < sh_need) {
      s = pers_grow(ctx, ctx->pers_sh, (size_t)sh_need * sizeof(float), "shared team buffers");
      if (s != RPCA_OK) return s;
      ctx->pers_sh_floats = sh_need;
    }
    if (ctx->pers_bar_cap < teams) {
      const int cap = (int)round_up(teams, 64);
      s = pers_grow(ctx, ctx->pers_bar, (size_t)cap * sizeof(int), "team counters");
      if (s != RPCA_OK) return s;
      ctx->pers_bar_cap = cap;
    }
  }
  int team = 0;
  for (int i : ord) {
    PersProblem e = tab[i];
    if (parts[i] < 2) {
      plan.table.push_back(e);
      continue;
    }
    e.parts = parts[i];
    e.sh = ctx->pers_sh + sh_off[i];
    e.bar = ctx->pers_bar + team++;
    for (int g = 0; g < parts[i]; ++g) {
      e.part = g;
      plan.table.push_back(e);
    }
  }
  plan.maxdim = maxdim;
  plan.grid = grid;
  plan.teams = teams;
  return RPCA_OK;
}
}  // namespace

extern "C" {

rpca_status rpca_set_batch_split(rpca_ctx ctx, int32_t max_parts, int32_t min_parts,
                                 int32_t spin_limit) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (max_parts < 1 || max_parts > kPersMaxParts || min_parts < 1 || min_parts > max_parts ||
      spin_limit < 0)
    return fail(ctx, RPCA_ERR_INVALID_ARG,
                "batch split: 1 <= min_parts <= max_parts <= 16, spin_limit >= 0");
  ctx->split_max_parts = max_parts;
  ctx->split_min_parts = min_parts;
  ctx->team_spins = spin_limit ? spin_limit : (1 << 22);
  return RPCA_OK;
}

rpca_status rpca_set_batch_mode(rpca_ctx ctx, int32_t mode) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (mode != 0 && mode != 1) return fail(ctx, RPCA_ERR_INVALID_ARG, "batch mode must be 0 or 1");
  ctx->batch_mode = mode;
  return RPCA_OK;
}

rpca_status rpca_svd_batched(rpca_ctx ctx, int count, const rpca_problem* problems,
                             unsigned flags) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (count < 0 || (count > 0 && !problems)) return fail(ctx, RPCA_ERR_INVALID_ARG, "bad batch");
  if (count == 0) return RPCA_OK;
  const int kSlots = ctx->batch_streams;
  // check every problem and size its workspace
  std::vector<size_t> ws_need(count), ctr_need(count);
  std::vector<double> cost(count);
  for (int p = 0; p < count; ++p) {
    const rpca_problem& q = problems[p];
    const std::string at = "problem " + std::to_string(p) + ": ";
    if (q.kind != 0 && q.kind != 1) return fail(ctx, RPCA_ERR_INVALID_ARG, at + "kind must be 0 or 1");
    rpca_status s = check_matrix(ctx, q.A, q.kind == 0);
    if (s != RPCA_OK) return fail(ctx, s, at + ctx->err);
    int l = q.l;
    s = check_kl(ctx, q.k, l, q.A->m, q.A->n);
    if (s != RPCA_OK) return fail(ctx, s, at + ctx->err);
    if (q.its < 0) return fail(ctx, RPCA_ERR_INVALID_ARG, at + "its must be >= 0");
    if (!q.U || !q.S || q.ldu < q.k) return fail(ctx, RPCA_ERR_INVALID_ARG, at + "bad U or S");
    if (q.kind == 0 && (!q.V || q.ldv < q.k)) return fail(ctx, RPCA_ERR_INVALID_ARG, at + "bad V");
    if (q.kind == 1 && (q.A->m != q.A->n || (q.flags & RPCA_CENTER)))
      return fail(ctx, RPCA_ERR_INVALID_ARG, at + "PSD problems are square and not centered");
    Work w;
    Arena probe;
    layout(probe, w, q.A->m, q.A->n, l, ctx->num_cus, q.kind == 1, layout_kind(q.A));
    ws_need[p] = probe.off + 256;
    ctr_need[p] = (size_t)w.lu_ctr + 16;
    cost[p] = (double)q.A->m * q.A->n * (2.0 * q.its + 2.0) + 1e6;
  }
  // problems the persistent launch takes: dense float32, m, n <= 8192, l <= 64
  std::vector<int> pers, rest;
  for (int p = 0; p < count; ++p) {
    const rpca_problem& q = problems[p];
    const int l = q.l > 0 ? q.l : q.k + 2;
    const bool ok = ctx->batch_mode == 0 && !is_sparse(q.A) && q.A->dtype == RPCA_F32 &&
                    l <= kPersMaxL && q.A->m <= kPersMaxDim && q.A->n <= kPersMaxDim &&
                    !(q.flags & (RPCA_NYSTROM_SQRT | RPCA_FUSED_ATA));
    (ok ? pers : rest).push_back(p);
  }
  const int ns = std::min(kSlots, (int)rest.size());
  // largest problems first, each to the least loaded stream
  std::vector<int> order(rest), slot_of(count);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
  std::vector<double> load(ns, 0.0);
  std::vector<size_t> ws_max(ns, 0), ctr_max(ns, 0);
  for (int p : order) {
    const int b = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    slot_of[p] = b;
    load[b] += cost[p];
    ws_max[b] = std::max(ws_max[b], ws_need[p]);
    ctr_max[b] = std::max(ctr_max[b], ctr_need[p]);
  }
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIP_OK(hipStreamIsCapturing(ctx->stream, &cap));
  const bool capturing = cap != hipStreamCaptureStatusNone;
  // per-problem status entries (allocated outside capture only; a buffer a
  // larger one replaces is kept for the graphs that use it)
  if (ctx->bstat_cap < count) {
    if (capturing) return fail(ctx, RPCA_ERR_UNSUPPORTED, "run the batch once before capturing it");
    HIP_OK(hipStreamSynchronize(ctx->stream));
    rpca_status s = pers_grow(ctx, ctx->bstat, (size_t)round_up(count, 4) * sizeof(int),
                              "status table");
    if (s != RPCA_OK) return s;
    ctx->bstat_cap = (int)round_up(count, 4);
  }
  ctx->bstat_count = count;
  launch_fill_zero(ctx->stream, reinterpret_cast<float*>(ctx->bstat), round_up(count, 4));
  // the persistent launch's table and working memory (allocated outside capture only)
  ctx_s_pers_plan plan;
  if (!pers.empty()) {
    rpca_status s = pers_prepare(ctx, problems, pers, capturing, plan);
    if (s != RPCA_OK) return s;
  }
  if ((int)ctx->slots.size() < ns && capturing)
    return fail(ctx, RPCA_ERR_UNSUPPORTED, "run the batch once before capturing it");
  if (!ctx->fork) HIP_OK(hipEventCreateWithFlags(&ctx->fork, hipEventDisableTiming));
  while ((int)ctx->slots.size() < ns) {
    BatchSlot b;
    HIP_OK(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
    HIP_OK(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    ctx->slots.push_back(b);
  }
  for (int b = 0; b < ns; ++b) {
    BatchSlot& sl = ctx->slots[b];
    if (sl.ws_bytes < ws_max[b] || sl.counters_n < ctr_max[b]) {
      if (capturing) return fail(ctx, RPCA_ERR_UNSUPPORTED, "run the batch once before capturing it");
      if (ctx->ws_limit && ws_max[b] > ctx->ws_limit)
        return fail(ctx, RPCA_ERR_NO_MEMORY, "batch workspace exceeds the limit");
      HIP_OK(hipStreamSynchronize(sl.stream));
      if (sl.ws_bytes < ws_max[b]) {
        if (sl.ws) HIP_OK(hipFree(sl.ws));
        sl.ws = nullptr;
        sl.ws_bytes = 0;
        void* p = nullptr;
        if (hipMalloc(&p, ws_max[b]) != hipSuccess) {
          (void)hipGetLastError();
          return fail(ctx, RPCA_ERR_NO_MEMORY, "batch workspace allocation failed");
        }
        sl.ws = static_cast<char*>(p);
        sl.ws_bytes = ws_max[b];
      }
      if (sl.counters_n < ctr_max[b]) {
        if (sl.counters) HIP_OK(hipFree(sl.counters));
        sl.counters = nullptr;
        sl.counters_n = 0;
        void* p = nullptr;
        if (hipMalloc(&p, ctr_max[b] * sizeof(unsigned)) != hipSuccess) {
          (void)hipGetLastError();
          return fail(ctx, RPCA_ERR_NO_MEMORY, "batch counter allocation failed");
        }
        HIP_OK(hipMemset(p, 0, ctr_max[b] * sizeof(unsigned)));
        sl.counters = static_cast<unsigned*>(p);
        sl.counters_n = ctr_max[b];
      }
    }
  }
  // fork: every stream starts after the work already on the context stream
  HIP_OK(hipEventRecord(ctx->fork, ctx->stream));
  for (int b = 0; b < ns; ++b) HIP_OK(hipStreamWaitEvent(ctx->slots[b].stream, ctx->fork, 0));
  // the persistent launch runs on the context stream beside them
  if (!pers.empty()) {
    launch_pers_table(ctx->stream, plan.table.data(), (int)plan.table.size(), ctx->pers_tab);
    launch_fill_zero(ctx->stream, reinterpret_cast<float*>(ctx->pers_counter), 4);
    if (plan.teams)
      launch_fill_zero(ctx->stream, reinterpret_cast<float*>(ctx->pers_bar),
                       round_up(plan.teams, 4));
    launch_persistent(ctx->stream, ctx->pers_tab, (int)plan.table.size(), ctx->pers_counter,
                      ctx->pers_ws, plan.maxdim, plan.grid, ctx->nys_retries, ctx->team_spins);
    HIP_OK(hipGetLastError());
    ctx->stats.calls += pers.size();
  }
  // issue each problem on its stream with that stream's workspace
  const hipStream_t st0 = ctx->stream;
  char* const ws0 = ctx->ws;
  const size_t wsb0 = ctx->ws_bytes;
  unsigned* const ctr0 = ctx->counters;
  const size_t ctrn0 = ctx->counters_n;
  rpca_status res = RPCA_OK;
  for (size_t r = 0; r < rest.size() && res == RPCA_OK; ++r) {
    const int p = rest[r];
    const rpca_problem& q = problems[p];
    BatchSlot& sl = ctx->slots[slot_of[p]];
    ctx->stream = sl.stream;
    ctx->ws = sl.ws;
    ctx->ws_bytes = sl.ws_bytes;
    ctx->counters = sl.counters;
    ctx->counters_n = sl.counters_n;
    const unsigned f =
        (q.flags & (RPCA_CENTER | RPCA_RENORM_ORTH | RPCA_RENORM_LU | RPCA_OMEGA_UNIFORM |
                    RPCA_NYSTROM_SQRT | RPCA_FUSED_ATA)) |
        (flags & RPCA_DETERMINISTIC);
    if (q.kind == 0)
      res = svd_impl(ctx, q.A, q.k, q.l, q.its, q.seed, f, q.U, q.ldu, q.S, q.V, q.ldv,
                     ctx->bstat + p);
    else
      res = eig_psd_impl(ctx, q.A, q.k, q.l, q.its, q.seed, f, q.U, q.ldu, q.S, ctx->bstat + p);
  }
  ctx->stream = st0;
  ctx->ws = ws0;
  ctx->ws_bytes = wsb0;
  ctx->counters = ctr0;
  ctx->counters_n = ctrn0;
  // join: the context stream continues after every stream's last solve
  for (int b = 0; b < ns; ++b) {
    HIP_OK(hipEventRecord(ctx->slots[b].done, ctx->slots[b].stream));
    HIP_OK(hipStreamWaitEvent(ctx->stream, ctx->slots[b].done, 0));
  }
  if (res != RPCA_OK) return res;
  if (flags & RPCA_SYNC) return sync_status(ctx);
  return RPCA_OK;
}

rpca_status rpca_batch_status(rpca_ctx ctx, int32_t count, int32_t* status_host) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (count < 0 || count > ctx->bstat_count || (count > 0 && !status_host))
    return fail(ctx, RPCA_ERR_INVALID_ARG, "batch_status: count must be <= the last batch's");
  HIP_OK(hipStreamSynchronize(ctx->stream));
  if (count == 0) return RPCA_OK;
  std::vector<int> bits(count);
  HIP_OK(hipMemcpyAsync(bits.data(), ctx->bstat, count * sizeof(int), hipMemcpyDeviceToHost,
                        ctx->stream));
  HIP_OK(hipStreamSynchronize(ctx->stream));
  for (int i = 0; i < count; ++i)
    status_host[i] = (bits[i] & kErrTimeout) ? RPCA_ERR_TIMEOUT
                     : (bits[i] & kErrNonFinite) ? RPCA_ERR_NUMERICAL
                     : (bits[i] & kErrNotPsd) ? RPCA_ERR_NOT_PSD : RPCA_OK;
  return RPCA_OK;
}

rpca_status rpca_sync(rpca_ctx ctx) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  return sync_status(ctx);
}

rpca_status rpca_set_nystrom_retries(rpca_ctx ctx, int32_t retries) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (retries < 0 || retries > 30)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "Nystrom retries must be in [0, 30]");
  ctx->nys_retries = retries;
  return RPCA_OK;
}

rpca_status rpca_tune(rpca_ctx ctx, const rpca_matrix* A, int32_t l, int32_t reps,
                      rpca_tune_result* out) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  rpca_status s = check_matrix(ctx, A);
  if (s != RPCA_OK) return s;
  if (is_sparse(A)) return fail(ctx, RPCA_ERR_UNSUPPORTED, "tune: dense A only");
  s = check_kl(ctx, 1, l, A->m, A->n);
  if (s != RPCA_OK) return s;
  if (reps < 1) reps = 3;
  const int64_t m = A->m, n = A->n;
  const AView Av = native_view(A);
  const bool f32 = Av.dtype == RPCA_F32;
  Work w;
  const TuneCfg base{};
  s = prepare(ctx, w, m, n, l, false, Av.dtype, &base);
  if (s != RPCA_OK) return s;
  hipStream_t st = ctx->stream;
  hipEvent_t ea = take_event(ctx), eb = take_event(ctx);
  if (!ea || !eb) return fail(ctx, RPCA_ERR_HIP, "tune: no events");
  // average device time of one launch sequence over reps runs after a warm-up
  auto timed = [&](auto&& run, double* ms) -> rpca_status {
    run();
    HIP_OK(hipEventRecord(ea, st));
    for (int r = 0; r < reps; ++r) run();
    HIP_OK(hipEventRecord(eb, st));
    HIP_OK(hipGetLastError());
    HIP_OK(hipEventSynchronize(eb));
    float t = 0.f;
    HIP_OK(hipEventElapsedTime(&t, ea, eb));
    *ms = (double)t / reps;
    return RPCA_OK;
  };
  rpca_tune_result res{};
  TuneCfg best{};
  // operands: a Gaussian X (n x l), Y = A X, Q = Y for A^T Q, Z = A^T Q
  launch_fill_zero(st, w.Z, n * w.lp);
  launch_gaussian(st, 0x7475ull, 0u, n, l, w.Z, w.lp, nullptr);
  pack_n_side(ctx, w, w.Z, n, Av);
  int cand[8][2], acand[8][2];
  const int nc = ax_candidates(w.nb, cand);
  const int nac = atx_candidates(w.nb, acand);
  if (f32 && dma_ok_shape(Av.data, Av.ld, n)) {
    double bms = 1e30;
    for (int i = 0; i < nc; ++i) {
      TuneCfg c{};
      c.ax_waves = cand[i][0];
      c.ax_ring = cand[i][1];
      double ms = 0;
      s = timed([&] { launch_ax(st, Av.data, Av.dtype, Av.ld, m, n, w.Xp, w.Y, w.lp, w.nb,
                                ctx->num_cus, &c); }, &ms);
      if (s != RPCA_OK) break;
      ++res.candidates;
      if (ms < bms) { bms = ms; best.ax_waves = c.ax_waves; best.ax_ring = c.ax_ring; }
    }
    res.ms_ax = bms;
  }
  if (s == RPCA_OK) {
    // Y = A X with the chosen configuration (the tournament's input)
    w.cfg = best;
    run_ax(ctx, Av, w, w.Xp, w.Y);
    pack_m_side(ctx, w, w.Y, m, false);
  }
  if (s == RPCA_OK && f32 && dma_ok_shape(Av.data, Av.ld, n)) {
    double bms = 1e30;
    for (int i = 0; i < nac && s == RPCA_OK; ++i) {
      TuneCfg c{};
      c.atx_waves = acand[i][0];
      c.atx_ring = acand[i][1];
      const AtxPlan plan = plan_atx(m, n, w.nb, ctx->num_cus, RPCA_F32, &c);
      double ms = 0;
      s = timed([&] {
        launch_atx(st, Av.data, Av.dtype, Av.ld, m, n, w.Xp, w.P, plan, w.nb);
        launch_atx_reduce(st, w.P, plan, w.nb, n, nullptr, w.Z, w.lp);
      }, &ms);
      ++res.candidates;
      if (ms < bms) { bms = ms; best.atx_waves = c.atx_waves; best.atx_ring = c.atx_ring; }
    }
    res.ms_atx = bms;
  } else if (s == RPCA_OK) {
    apply_at(ctx, Av, w, w.Z);
  }
  if (s == RPCA_OK) {
    // the tournament on both sides, for each block height
    double bms = 1e30;
    for (int r : {256, 512, 1024}) {
      if (r == 1024 && w.lp > 64) continue;
      const LuPlan pm = plan_lu(m, w.lp, r), pn = plan_lu(n, w.lp, r);
      double ms = 0;
      s = timed([&] {
        launch_lu_tree(st, w.Y, w.lp, m, w.l, pm, w.cand, ctx->counters, w.Ulu, w.piv);
        launch_lu_tree(st, w.Z, w.lp, n, w.l, pn, w.cand, ctx->counters, w.Ulu, w.piv);
      }, &ms);
      if (s != RPCA_OK) break;
      ++res.candidates;
      if (ms < bms) { bms = ms; best.lu_rows = r; }
    }
    res.ms_lu = bms;
  }
  ctx->event_pool.push_back(ea);
  ctx->event_pool.push_back(eb);
  if (s != RPCA_OK) return s;
  ctx->tune[tune_key(m, n, w.lp, Av.dtype)] = best;
  res.ax_waves = best.ax_waves;
  res.ax_ring = best.ax_ring;
  res.atx_waves = best.atx_waves;
  res.atx_ring = best.atx_ring;
  res.lu_rows = best.lu_rows;
  if (out) *out = res;
  return RPCA_OK;
}

rpca_status rpca_tune_save(rpca_ctx ctx, const char* path) {
  if (!ctx || !path) return RPCA_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "w");
  if (!f) return fail(ctx, RPCA_ERR_INVALID_ARG, std::string("tune: cannot write ") + path);
  std::fprintf(f, "# log2m log2n lp dtype ax_waves ax_ring atx_waves atx_ring lu_rows\n");
  for (const auto& kv : ctx->tune) {
    const TuneCfg& c = kv.second;
    std::fprintf(f, "%d %d %d %d %d %d %d %d %d\n", kv.first[0], kv.first[1], kv.first[2],
                 kv.first[3], c.ax_waves, c.ax_ring, c.atx_waves, c.atx_ring, c.lu_rows);
  }
  const bool ok = std::fclose(f) == 0;
  return ok ? RPCA_OK : fail(ctx, RPCA_ERR_INVALID_ARG, std::string("tune: write failed: ") + path);
}

rpca_status rpca_tune_load(rpca_ctx ctx, const char* path) {
  if (!ctx || !path) return RPCA_ERR_INVALID_ARG;
  FILE* f = std::fopen(path, "r");
  if (!f) return fail(ctx, RPCA_ERR_INVALID_ARG, std::string("tune: cannot read ") + path);
  std::map<std::array<int, 4>, TuneCfg> add;
  char line[512];
  int lineno = 0;
  bool bad = false;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    const char* p = line;
    while (*p == ' ' || *p == '\t') ++p;
    if (*p == '#' || *p == '\n' || *p == '\r' || *p == 0) continue;
    int v[9];
    char tail[8];
    const int got = std::sscanf(p, "%d %d %d %d %d %d %d %d %d %7s", &v[0], &v[1], &v[2], &v[3],
                                &v[4], &v[5], &v[6], &v[7], &v[8], tail);
    const bool lp_ok = v[2] == 32 || v[2] == 64 || v[2] == 128;
    if (got != 9 || !lp_ok || v[0] < 0 || v[0] > 62 || v[1] < 0 || v[1] > 62 || v[3] < 0 ||
        v[3] > 2 || v[4] < 0 || v[5] < 0 || v[6] < 0 || v[7] < 0 || v[8] < 0) {
      bad = true;
      break;
    }
    TuneCfg c;
    c.ax_waves = v[4];
    c.ax_ring = v[5];
    c.atx_waves = v[6];
    c.atx_ring = v[7];
    c.lu_rows = v[8];
    add[{v[0], v[1], v[2], v[3]}] = c;
  }
  std::fclose(f);
  if (bad)
    return fail(ctx, RPCA_ERR_INVALID_ARG,
                std::string("tune: malformed line ") + std::to_string(lineno) + " of " + path);
  for (const auto& kv : add) ctx->tune[kv.first] = kv.second;
  return RPCA_OK;
}

rpca_status rpca_set_batch_streams(rpca_ctx ctx, int32_t streams) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  if (streams < 1 || streams > 64)
    return fail(ctx, RPCA_ERR_INVALID_ARG, "batch streams must be in [1, 64]");
  ctx->batch_streams = streams;
  return RPCA_OK;
}

rpca_status rpca_tune_clear(rpca_ctx ctx) {
  if (!ctx) return RPCA_ERR_INVALID_ARG;
  ctx->tune.clear();
  return RPCA_OK;
}

rpca_status rpca_tune_count(rpca_ctx ctx, int32_t* count) {
  if (!ctx || !count) return RPCA_ERR_INVALID_ARG;
  *count = (int32_t)ctx->tune.size();
  return RPCA_OK;
}

}  // extern "C"
