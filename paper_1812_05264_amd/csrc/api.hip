// C ABI of the randomized Fermi-operator library: validation, device buffers and
// the orchestration of the kernels (see include/rfo.h for the contract).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "rfo.h"
#include "rfo_internal.h"

namespace {

std::string g_create_error;

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

}  // namespace

struct rfo_ctx {
  int device = 0;
  int cus = 256;  // compute units of the device
  hipStream_t stream = nullptr;
  std::string err;

  // Hamiltonian
  bool has_h = false;
  int64_t nb = 0, n = 0, nnzb = 0;
  int64_t max_row = 0;  // largest number of blocks in a block row
  int bd = 0, prec = 0;
  double e_min = 0.0, e_max = 0.0;
  std::vector<int64_t> row_ptr_h;
  std::vector<int32_t> col_h;
  DevBuf row_ptr, col, brow, tpos, hraw, h64, h32, hbf16, gscratch, nz_up, nz_low;
  int64_t n_up = 0, n_low = 0;
  // BF16 9x9 steps: groups of consecutive upper blocks of one block row (at most
  // kSddmmGroup blocks) for the segment gradient on the matrix cores
  DevBuf up_grp;
  int64_t n_up_grp = 0;
  bool has_up_grp = false;
  // BF16 steps: K chunks of 16 rows per block row (first chunk of each row,
  // gathered row J*9 + c and source nz*9 + c of every K row)
  DevBuf kc_ptr, kc_idx, kc_src;
  int64_t n_chunks = 0;

  // probes
  bool has_r = false;
  int64_t s = 0;
  int sp = 0;
  bool signs = false;
  double w_uniform = 0.0;  // the common weight of the real probes, 0 if they differ
  DevBuf sgn, rden, w;

  // work buffers
  DevBuf vec, acc, ring, moments, coef, samples, costab, small, flags, G, dHdR, forces;
  bool has_grad = false;

  bool doubling = true;  // moment-only calls via T_2j, T_2j-1 identities
  // nonorthogonal basis: overlap S on H's pattern, S^{-1} by conjugate gradients
  bool has_s = false, interval_given = false, has_q = false, has_dens = false;
  double cg_tol = 1e-13;
  DevBuf s64, cg_part, cg_sc, GQ;
  double *cg_res_h = nullptr;
  int64_t cg_iters = 0, cg_solves = 0;
  int64_t mom_p = 0;     // moments of the last call still valid on the device (0 = none)
  // rational expansion: complex CGLS planes, column partials, scalars, r . x per pole
  DevBuf rat, rat_part, rat_sc, rat_rho, rat_coef;
  std::vector<double> rat_coef_h;
  double *rat_res_h = nullptr;
  int64_t cgls_iters = 0, cgls_solves = 0;

  // instrumentation
  bool timing = false;
  double t_ms = 0.0;
  int64_t t_steps = 0;
  std::vector<hipEvent_t> events;
  int *flags_h = nullptr;

  // second stream (default priority) on which the doubled adjoint runs a segment's
  // gradient while the next segment's steps run on `stream`
  hipStream_t side = nullptr;
  hipEvent_t ev_rev = nullptr, ev_sd[2] = {nullptr, nullptr};

  ~rfo_ctx() {
    hipSetDevice(device);
    DevBuf *all[] = {&row_ptr, &col, &brow, &tpos, &hraw, &h64, &h32, &hbf16, &gscratch, &nz_up, &nz_low,
                     &kc_ptr, &kc_idx, &kc_src, &up_grp,
                     &s64, &cg_part, &cg_sc, &GQ, &rat, &rat_part, &rat_sc, &rat_rho, &rat_coef,
                     &sgn, &rden, &w, &vec, &acc, &ring, &moments, &coef, &samples,
                     &costab, &small, &flags, &G, &dHdR, &forces};
    for (DevBuf *b : all)
      if (b->p) hipFree(b->p);
    for (hipEvent_t e : events) hipEventDestroy(e);
    if (side) {
      hipStreamSynchronize(side);
      hipStreamDestroy(side);
    }
    for (hipEvent_t e : {ev_rev, ev_sd[0], ev_sd[1]})
      if (e) hipEventDestroy(e);
    if (flags_h) hipHostFree(flags_h);
    if (cg_res_h) hipHostFree(cg_res_h);
    if (rat_res_h) hipHostFree(rat_res_h);
  }
};

namespace {

int fail(rfo_ctx *c, int code, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return code;
}

#define HIPCHK(call)                                                                     \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      return fail(ctx, RFO_E_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                  __FILE__, __LINE__);                                                   \
  } while (0)

#define TRY(expr)             \
  do {                        \
    int r_ = (expr);          \
    if (r_ != RFO_OK) return r_; \
  } while (0)

int ensure(rfo_ctx *ctx, DevBuf &b, size_t bytes) {
  if (bytes == 0) bytes = 8;
  if (b.bytes >= bytes) return RFO_OK;
  if (b.p) {
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    b.p = nullptr;
    return fail(ctx, RFO_E_NOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
  }
  b.bytes = bytes;
  return RFO_OK;
}

void release(DevBuf &b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

template <typename T>
T *P(DevBuf &b) {
  return static_cast<T *>(b.p);
}

// Launch decomposition of the Chebyshev step for the current H, probes and precision.
struct Plan {
  int vt_bytes;    // bytes per vector element
  int ppl;         // probes per lane
  int n_pt;        // probe tiles
  int rows_per_wg; // block rows per workgroup
  int n_rg;        // row groups
  int ring;        // moment ring depth
  int rpi;         // rows per wave iteration
  int grid;        // resident workgroups of the step kernels
  int n_pt_step;   // probe tiles of the step kernel (BF16: tiles of 16 * ntiles probes)
  int ntiles;      // BF16: MFMA column tiles per wave
  size_t vec_elems;
  // bytes per vector slot: the vector, and in BF16 mode its BF16 copy (the
  // operand the steps gather) right after it
  size_t slot_bytes;
};

Plan make_plan(const rfo_ctx *c) {
  Plan pl;
  pl.vt_bytes = c->prec == RFO_FP64 ? 8 : 4;
  // 16 bytes per lane (FP64) or 16 (FP32, 9x9: 32 measured best) per gather
  int want = 16 / pl.vt_bytes;
  if (c->bd == 9 && c->prec != RFO_FP64) want = 4;
  if (const char *env = getenv("RFO_PPL")) want = atoi(env);
  pl.ppl = 1;
  for (int q = 4; q >= 1; q >>= 1)
    if (q <= want && c->sp % (64 * q) == 0) {
      pl.ppl = q;
      break;
    }
  pl.n_pt = c->sp / (64 * pl.ppl);
  // rows per workgroup: small enough that the resident workgroups of an XCD
  // cover a narrow band of rows, large enough to keep the moment partials small
  int64_t rows = c->bd == 1 ? 8 : 4;
  if (const char *env = getenv("RFO_ROWS_PER_WG")) {
    const int64_t r = atoll(env);
    if (r >= 1) rows = r;
  }
  pl.rows_per_wg = (int)rows;
  pl.n_rg = (int)((c->nb + rows - 1) / rows);
  pl.ring = 32;
  // 1x1 blocks: rows per wave iteration, or 7 when every row fits one chunk of 7
  // neighbours (measured faster on the 7-point lattice); 9x9: blocks per chunk
  pl.rpi = c->bd == 1 ? (c->max_row <= 7 ? 7 : 1) : 2;
  if (const char *env = getenv("RFO_RPI")) {
    const int r = atoi(env);
    if (r == 1 || r == 2 || (c->bd == 1 && r == 7)) pl.rpi = r;
  }
  pl.n_pt_step = pl.n_pt;
  pl.ntiles = 0;
  int occ = 1;
  if (c->prec == RFO_BF16) {
    // 4 MFMA column tiles (64 probes) per wave, 2 blocks per chunk: measured best
    // (wider tiles or chunks cost more registers than the loads they add in flight)
    pl.ntiles = 4;
    pl.rpi = 2;
    pl.n_pt_step = c->sp / (16 * pl.ntiles);
    if (const char *env = getenv("RFO_BF16_U")) {
      const int u = atoi(env);
      if (u == 1 || u == 2 || u == 4) pl.rpi = u;
    }
    occ = std::max(1, rfo::step_bf16_blocks_per_cu(pl.ntiles, pl.rpi));
  } else {
    occ = std::max(1, rfo::step_blocks_per_cu(c->bd, c->prec == RFO_FP64 ? 0 : 1, pl.ppl, pl.rpi));
  }
  // one resident wave of workgroups, a multiple of 8 (one share per XCD), at
  // most four per CU: more workgroups widen the band of rows in flight on an XCD
  // past what its L2 holds of their neighbour rows (measured slower)
  int64_t grid = (int64_t)c->cus * std::min(occ, 4);
  if (const char *env = getenv("RFO_GRID")) grid = std::max<int64_t>(8, atoll(env));
  const int64_t units = (int64_t)pl.n_pt_step * pl.n_rg;
  grid = std::min(grid, (units + 7) / 8 * 8);
  grid = std::max<int64_t>(8, grid / 8 * 8);
  pl.grid = (int)grid;
  pl.vec_elems = (size_t)c->n * (size_t)c->sp;
  pl.slot_bytes = pl.vec_elems * (pl.vt_bytes + (c->prec == RFO_BF16 ? 2 : 0));
  return pl;
}

void fill_step(rfo_ctx *c, const Plan &pl, rfo::StepArgs &a) {
  memset(&a, 0, sizeof(a));
  a.row_ptr = P<int64_t>(c->row_ptr);
  a.col = P<int32_t>(c->col);
  a.hval = c->prec == RFO_FP64 ? c->h64.p : (c->prec == RFO_FP32 ? c->h32.p : c->hbf16.p);
  if (c->prec == RFO_BF16) {
    a.kc_ptr = P<int64_t>(c->kc_ptr);
    a.kc_idx = P<int32_t>(c->kc_idx);
  }
  a.sgn = c->signs ? P<uint64_t>(c->sgn) : nullptr;
  a.rden = c->signs ? nullptr : P<double>(c->rden);
  a.nb = c->nb;
  a.sp = c->sp;
  a.rows_per_wg = pl.rows_per_wg;
  a.n_rg = pl.n_rg;
  a.n_pt = pl.n_pt_step;
  a.rpi = pl.rpi;
  a.grid = pl.grid;
}

void fill_init(rfo_ctx *c, const Plan &pl, rfo::InitArgs &a) {
  memset(&a, 0, sizeof(a));
  a.sgn = c->signs ? P<uint64_t>(c->sgn) : nullptr;
  a.rden = c->signs ? nullptr : P<double>(c->rden);
  a.nb = c->nb;
  a.bd = c->bd;
  a.sp = c->sp;
  a.rows_per_wg = pl.rows_per_wg;
  a.n_rg = pl.n_rg;
  a.n_pt = pl.n_pt;
  a.ppl = pl.ppl;
  a.grid = pl.grid;
}

int kernel_precision(const rfo_ctx *c) { return c->prec == RFO_FP64 ? 0 : 1; }

// The segment gradient of the BF16 steps runs on the matrix cores when every real
// probe has the same weight (the weight is applied in FP64 after each step's
// contraction).  FP32 steps keep the VALU contraction: an FP32-MFMA version
// measured no faster at full size and sums in FP32.
bool use_mfma_sddmm(const rfo_ctx *c) {
  if (c->bd != 9 || c->prec != RFO_BF16 || c->w_uniform == 0.0 || !c->has_up_grp) return false;
  if (c->sp % 32 != 0) return false;
  if (const char *env = getenv("RFO_SDDMM_MFMA")) return atoi(env) != 0;
  return true;
}

int sddmm_ppl(const rfo_ctx *c) {
  int ppl = (c->sp % 128 == 0) ? 2 : 1;
  if (const char *env = getenv("RFO_SDDMM_PPL")) ppl = atoi(env) == 2 && c->sp % 128 == 0 ? 2 : 1;
  return ppl;
}

hipError_t launch_any_step(const rfo_ctx *c, const Plan &pl, const rfo::StepArgs &a) {
  // three accumulator terms need y_{k-1}, which the first pass does not have
  if (a.acc_terms < 0 || a.acc_terms > 3 || (a.acc_terms == 3 && a.c2 == 0.0))
    return hipErrorInvalidValue;
  if (c->prec == RFO_BF16) {
    // x and out are vector slots; their BF16 copies follow the FP32 vectors
    rfo::StepArgs b = a;
    b.xb = static_cast<const char *>(a.x) + pl.vec_elems * sizeof(float);
    b.outb = static_cast<char *>(a.out) + pl.vec_elems * sizeof(float);
    return rfo::launch_step_bf16(pl.ntiles, b, c->stream);
  }
  return rfo::launch_step(c->bd, kernel_precision(c), pl.ppl, a, c->stream);
}

// y = scale r into a vector slot (and its BF16 copy in BF16 mode)
hipError_t launch_init_slot(const rfo_ctx *c, const Plan &pl, rfo::InitArgs &a) {
  a.outb = c->prec == RFO_BF16 ? static_cast<char *>(a.out) + pl.vec_elems * sizeof(float) : nullptr;
  return rfo::launch_init(kernel_precision(c), a, c->stream);
}

char *vec_at(rfo_ctx *c, const Plan &pl, DevBuf &b, int64_t i) {
  return static_cast<char *>(b.p) + (size_t)i * pl.slot_bytes;
}

hipEvent_t next_event(rfo_ctx *c, size_t idx) {
  while (c->events.size() <= idx) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->events.push_back(e);
  }
  return c->events[idx];
}

int copy_out(rfo_ctx *ctx, void *dst, const void *src, size_t bytes) {
  if (!dst || bytes == 0) return RFO_OK;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, ctx->stream));
  return RFO_OK;
}

int check_flags_and_finish(rfo_ctx *ctx, size_t n_events) {
  HIPCHK(hipMemcpyAsync(ctx->flags_h, ctx->flags.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (ctx->timing) {
    for (size_t i = 0; i + 1 < n_events; i += 2) {
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, ctx->events[i], ctx->events[i + 1]));
      ctx->t_ms += ms;
    }
  }
  const int f = *ctx->flags_h;
  if (f & 4)
    return fail(ctx, RFO_E_NUMERIC,
                "a Chebyshev moment exceeded ||r||^2 or is not finite: the spectrum is not "
                "inside [e_min, e_max] = [%g, %g]", ctx->e_min, ctx->e_max);
  return RFO_OK;
}

// Forward recurrence over n_terms terms with moments (and optionally the density
// accumulator and checkpoints).  Vectors live in `bufs` (first two slots used as
// the rolling pair).  On return *last/*before hold the pointers of y_{p-1}, y_{p-2}.
struct Checkpoints {
  int64_t m = 0, Q = 0;
  DevBuf *store = nullptr;  // 2 (Q - 1) vectors: [q-1][0] = y_{qm-1}, [q-1][1] = y_{qm}
};

int ensure_cg(rfo_ctx *ctx) {
  TRY(ensure(ctx, ctx->cg_part, (size_t)rfo::cg_nparts(ctx->n) * ctx->sp * sizeof(double)));
  TRY(ensure(ctx, ctx->cg_sc, ((size_t)6 * ctx->sp + 1) * sizeof(double)));
  if (!ctx->cg_res_h) HIPCHK(hipHostMalloc((void **)&ctx->cg_res_h, sizeof(double), 0));
  return RFO_OK;
}

// t = S^{-1} y for every probe column by conjugate gradients (S symmetric positive
// definite), to |r_c| <= cg_tol |y_c|.  Work vectors: slots 3..5 of bufs.
int cg_solve(rfo_ctx *ctx, const Plan &pl, DevBuf &bufs, const void *y, void *t) {
  const int64_t n = ctx->n;
  const int sp = ctx->sp;
  double *r = reinterpret_cast<double *>(vec_at(ctx, pl, bufs, 3));
  double *pv = reinterpret_cast<double *>(vec_at(ctx, pl, bufs, 4));
  double *q = reinterpret_cast<double *>(vec_at(ctx, pl, bufs, 5));
  double *part = P<double>(ctx->cg_part), *sc = P<double>(ctx->cg_sc);
  double *res_d = sc + 6 * sp;
  HIPCHK(rfo::launch_cg_init(static_cast<const double *>(y), static_cast<double *>(t), r, pv, n, sp,
                             part, sc, ctx->stream));
  rfo::StepArgs sa;
  fill_step(ctx, pl, sa);
  sa.hval = ctx->s64.p;  // q = S p
  sa.x = pv;
  sa.prev = nullptr;
  sa.out = q;
  sa.c1 = 1.0;
  sa.c2 = 0.0;
  const double tol2 = ctx->cg_tol * ctx->cg_tol;
  const int max_it = 2000;
  for (int it = 1; it <= max_it; ++it) {
    HIPCHK(launch_any_step(ctx, pl, sa));
    HIPCHK(rfo::launch_cg_alpha(pv, q, n, sp, part, sc, ctx->stream));
    HIPCHK(rfo::launch_cg_update(static_cast<double *>(t), r, pv, q, n, sp, part, sc, res_d,
                                 ctx->stream));
    ++ctx->cg_iters;
    // the host looks at the residual every 4th iteration: up to three extra
    // iterations only shrink it further (a column whose residual is exactly zero
    // gets alpha = beta = 0)
    if (it % 4 != 0 && it != max_it) continue;
    HIPCHK(hipMemcpyAsync(ctx->cg_res_h, res_d, sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double res = *ctx->cg_res_h;
    if (!std::isfinite(res))
      return fail(ctx, RFO_E_NUMERIC, "conjugate gradients broke down: S is not positive definite");
    if (res <= tol2) {
      ++ctx->cg_solves;
      return RFO_OK;
    }
  }
  return fail(ctx, RFO_E_NUMERIC, "conjugate gradients did not reach %g in %d iterations", ctx->cg_tol,
              max_it);
}

int run_forward(rfo_ctx *ctx, const Plan &pl, int64_t p, DevBuf &bufs, bool use_acc,
                const Checkpoints *ck, size_t *n_events, bool dbl = false) {
  if (dbl && use_acc) return fail(ctx, RFO_E_INVALID, "the density needs every y_k");
  const int kp = kernel_precision(ctx);
  const double tol = ctx->prec == RFO_FP64 ? 1e-6 : (ctx->prec == RFO_FP32 ? 1e-3 : 1e-2);
  const size_t slot = (size_t)pl.grid * ctx->sp;
  double *ring = P<double>(ctx->ring);
  double *mom = P<double>(ctx->moments);
  double *coef = P<double>(ctx->coef);
  int *flags = P<int>(ctx->flags);
  char *A = vec_at(ctx, pl, bufs, 0);
  char *B = vec_at(ctx, pl, bufs, 1);
  void *accp = use_acc ? ctx->acc.p : nullptr;

  auto save = [&](int64_t k, const void *src) -> int {
    if (!ck || ck->Q < 2) return RFO_OK;
    const int64_t m = ck->m;
    for (int64_t q = 1; q < ck->Q; ++q) {
      int which = -1;
      if (k == q * m - 1) which = 0;
      if (k == q * m) which = 1;
      if (which >= 0) {
        char *dst = vec_at(ctx, pl, *ck->store, 2 * (q - 1) + which);
        HIPCHK(hipMemcpyAsync(dst, src, pl.slot_bytes, hipMemcpyDeviceToDevice,
                              ctx->stream));
      }
    }
    return RFO_OK;
  };

  rfo::InitArgs ia;
  fill_init(ctx, pl, ia);
  ia.out = A;
  ia.scale = nullptr;
  ia.acc = accp;
  ia.alpha = coef;  // alpha^f_0
  ia.part = ring;
  HIPCHK(launch_init_slot(ctx, pl, ia));
  HIPCHK(rfo::launch_moment_reduce(ring, pl.ring, 0, 1, pl.grid, ctx->sp, mom, 0, tol, flags, 0,
                                   ctx->stream));
  TRY(save(0, A));

  rfo::StepArgs sa;
  fill_step(ctx, pl, sa);
  char *cur = A, *prev = B;
  // direct: step k makes y_{k+1} and moment k+1 = r . y_{k+1} (p - 1 steps);
  // doubling: step k makes y_j (j = k+1) and the inner products that give
  // moments 2j-1 and 2j, so floor(p/2) steps reach moment p-1
  const int64_t n_steps = dbl ? p / 2 : p - 1;
  int64_t batch_start = 1;  // first moment index not yet reduced
  int64_t batch_steps = 0;
  int64_t acc_done = 0;     // the accumulator holds alpha_j y_j for j <= acc_done
  size_t ev = 0;
  for (int64_t k = 0; k < n_steps; ++k) {
    if (ctx->timing && batch_steps == 0) {
      hipEvent_t e = next_event(ctx, ev++);
      if (!e) return fail(ctx, RFO_E_DEVICE, "hipEventCreate failed");
      HIPCHK(hipEventRecord(e, ctx->stream));
    }
    char *out = (k == 0) ? B : prev;
    sa.x = cur;
    sa.prev = prev;
    sa.out = out;
    sa.c1 = (k == 0) ? 1.0 : 2.0;
    sa.c2 = (k == 0) ? 0.0 : -1.0;
    sa.beta = nullptr;
    // terms y_{acc_done+1} .. y_{k+1} wait; add them when three are held by the
    // pass (y_{k-1}, y_k, y_{k+1}) or at the last step
    const int64_t pending = k + 1 - acc_done;
    sa.acc = accp;
    // with an overlap the pass gathers t_k = S^{-1} y_k, not y_k: one term per pass
    sa.acc_terms = (accp && (ctx->has_s || pending == 3 || k + 2 == p)) ? (int)pending : 0;
    sa.alpha = coef + (acc_done + 1);
    if (sa.acc_terms) acc_done = k + 1;
    const int64_t hi = dbl ? 2 * (k + 1) : k + 1;  // highest moment index of this step
    sa.part = ring + (size_t)(hi % pl.ring) * slot;
    sa.part2 = dbl ? ring + (size_t)((hi - 1) % pl.ring) * slot : nullptr;
    if (ctx->has_s) {
      // y_{k+1} = 2 H_hat S^{-1} y_k - y_{k-1}: gather t_k = S^{-1} y_k (slot 2)
      char *t = vec_at(ctx, pl, bufs, 2);
      TRY(cg_solve(ctx, pl, bufs, cur, t));
      sa.x = t;
    }
    HIPCHK(launch_any_step(ctx, pl, sa));
    prev = cur;
    cur = out;
    ++batch_steps;
    const int64_t next_hi = hi + (dbl ? 2 : 1);
    // moments 0 and 1 must be final before a doubling reduction uses them
    const bool flush = (k + 1 == n_steps) || (dbl && k == 0) || (next_hi - batch_start + 1 > pl.ring);
    if (flush) {
      if (ctx->timing) {
        hipEvent_t e = next_event(ctx, ev++);
        if (!e) return fail(ctx, RFO_E_DEVICE, "hipEventCreate failed");
        HIPCHK(hipEventRecord(e, ctx->stream));
        ctx->t_steps += batch_steps;
      }
      const int64_t last = std::min(hi, p - 1);
      HIPCHK(rfo::launch_moment_reduce(ring, pl.ring, batch_start, (int)(last - batch_start + 1),
                                       pl.grid, ctx->sp, mom, ctx->has_s ? 0 : 1, tol, flags,
                                       dbl ? 1 : 0, ctx->stream));
      batch_start = last + 1;
      batch_steps = 0;
    }
    TRY(save(k + 1, cur));
  }
  *n_events = ev;
  return RFO_OK;
}

int prepare_call(rfo_ctx *ctx, double T, double mu, int64_t p, Plan &pl) {
  if (!ctx) return RFO_E_INVALID;
  if (!ctx->has_h) return fail(ctx, RFO_E_STATE, "no Hamiltonian: call rfo_set_hamiltonian first");
  if (!ctx->has_r) return fail(ctx, RFO_E_STATE, "no probes: call rfo_set_probes first");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(ctx, RFO_E_INVALID, "T must be finite and > 0");
  if (!std::isfinite(mu)) return fail(ctx, RFO_E_INVALID, "mu must be finite");
  if (p < 1 || p > (1 << 20)) return fail(ctx, RFO_E_INVALID, "n_terms must be in [1, 2^20]");
  HIPCHK(hipSetDevice(ctx->device));
  pl = make_plan(ctx);
  const int64_t nq = 4 * p;
  TRY(ensure(ctx, ctx->ring, (size_t)pl.ring * pl.grid * ctx->sp * sizeof(double)));
  TRY(ensure(ctx, ctx->moments, (size_t)p * ctx->sp * sizeof(double)));
  TRY(ensure(ctx, ctx->coef, (size_t)3 * p * sizeof(double)));
  TRY(ensure(ctx, ctx->samples, (size_t)3 * nq * sizeof(double)));
  TRY(ensure(ctx, ctx->costab, (size_t)4 * nq * sizeof(double)));
  TRY(ensure(ctx, ctx->small, 64 * sizeof(double)));
  HIPCHK(hipMemsetAsync(ctx->flags.p, 0, sizeof(int), ctx->stream));
  HIPCHK(rfo::launch_coefficients(ctx->e_min, ctx->e_max, T, mu, p, nq, P<double>(ctx->samples),
                                  P<double>(ctx->costab), P<double>(ctx->coef), ctx->stream));
  return RFO_OK;
}

int copy_moments_out(rfo_ctx *ctx, int64_t p, double *moments_out) {
  if (!moments_out) return RFO_OK;
  // internal [p][sp] -> caller [s][p]
  std::vector<double> tmp((size_t)p * ctx->sp);
  HIPCHK(hipMemcpyAsync(tmp.data(), ctx->moments.p, tmp.size() * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<double> outv((size_t)ctx->s * p);
  for (int64_t c = 0; c < ctx->s; ++c)
    for (int64_t k = 0; k < p; ++k) outv[(size_t)c * p + k] = tmp[(size_t)k * ctx->sp + c];
  HIPCHK(hipMemcpy(moments_out, outv.data(), outv.size() * sizeof(double), hipMemcpyDefault));
  return RFO_OK;
}

// ---------------------------------------------------------------------------
// Rational expansion with S = I (Rational approximation, Eq. rational_PQ; the
// rational free-energy derivative, Eq. rational_derivative with dS = 0).  The
// solves run on the mapped H_hat already on the device:
//   H - z = c (H_hat - z_hat),  c = (e_max - e_min)/2,  z_hat = (z - d)/c,
//   d = (e_max + e_min)/2,  so (H - z)^{-1} y = x / c  with  (H_hat - z_hat) x = y.
// ---------------------------------------------------------------------------
struct CxWork {
  double *x, *r, *p, *q, *s;  // complex: two planes each
  double *acc;                // real plane: P r accumulator
  double *part, *part2;       // column partials
  double *sc;                 // CGLS scalars [7][sp] + resmax
  int nparts;                 // rows of part / part2
  int ppl;                    // probes per lane of the complex product
  int u;                      // neighbours (1x1) or blocks (9x9) per chunk
  rfo::CspArgs ca;            // complex product arguments (x, out, z, part set per launch)
};

int cspmm(rfo_ctx *ctx, CxWork &w, const double *x, double *out, double zr, double zi,
          double *part) {
  w.ca.x = x;
  w.ca.out = out;
  w.ca.zr = zr;
  w.ca.zi = zi;
  w.ca.part = part;
  HIPCHK(rfo::launch_cspmm(ctx->bd, w.ppl, w.u, w.ca, ctx->stream));
  return RFO_OK;
}

// CGLS for (H_hat - z) x = y on every probe column, from the current x (first:
// x = 0), until |y - (H_hat - z) x| <= tol |y| for every column (checked on the
// host every fourth iteration; later iterations only shrink the residuals).
int cgls_solve(rfo_ctx *ctx, CxWork &w, double zr, double zi, double tol, int64_t max_iter,
               bool first, int64_t *iters) {
  const int64_t n = ctx->n;
  const int sp = ctx->sp;
  const int G = rfo::cg_nparts(n), grid = w.ca.grid;
  const uint64_t *sgn = ctx->signs ? P<uint64_t>(ctx->sgn) : nullptr;
  const double *rden = ctx->signs ? nullptr : P<double>(ctx->rden);
  double *sc = w.sc;
  double *yy = sc, *qq = sc + 2 * sp, *ssn = sc + 3 * sp, *rr = sc + 4 * sp, *al = sc + 5 * sp,
         *be = sc + 6 * sp, *res_d = sc + 7 * sp;
  const double tol2 = tol * tol;
  auto converged = [&](bool &done) -> int {
    HIPCHK(hipMemcpyAsync(ctx->rat_res_h, res_d, sizeof(double), hipMemcpyDeviceToHost,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    const double res = *ctx->rat_res_h;
    if (!std::isfinite(res))
      return fail(ctx, RFO_E_NUMERIC, "CGLS produced a non-finite residual (shift %g%+gi)", zr, zi);
    done = res <= tol2;
    return RFO_OK;
  };
  if (!first) TRY(cspmm(ctx, w, w.x, w.q, zr, zi, nullptr));
  HIPCHK(rfo::launch_cx_resid(sgn, rden, first ? nullptr : w.q, w.r, n, sp, w.part, w.part2,
                              ctx->stream));
  HIPCHK(rfo::launch_colreduce(w.part, G, sp, rr, ctx->stream));
  HIPCHK(rfo::launch_colreduce(w.part2, G, sp, yy, ctx->stream));
  // s = A^H r (A^H = H_hat - conj(z)), p = s
  TRY(cspmm(ctx, w, w.r, w.s, zr, -zi, w.part));
  HIPCHK(rfo::launch_colreduce(w.part, grid, sp, ssn, ctx->stream));
  HIPCHK(rfo::launch_cgls_scalars(sc, sp, 0, res_d, ctx->stream));
  HIPCHK(hipMemcpyAsync(w.p, w.s, (size_t)2 * n * sp * sizeof(double), hipMemcpyDeviceToDevice,
                        ctx->stream));
  bool done = false;
  TRY(converged(done));
  if (done) {
    *iters = 0;
    ++ctx->cgls_solves;
    return RFO_OK;
  }
  for (int64_t it = 1; it <= max_iter; ++it) {
    TRY(cspmm(ctx, w, w.p, w.q, zr, zi, w.part));  // q = A p
    HIPCHK(rfo::launch_colreduce(w.part, grid, sp, qq, ctx->stream));
    HIPCHK(rfo::launch_cgls_scalars(sc, sp, 1, res_d, ctx->stream));
    HIPCHK(rfo::launch_cx_update(w.r, w.q, al, n, sp, w.part, ctx->stream));
    HIPCHK(rfo::launch_colreduce(w.part, G, sp, rr, ctx->stream));
    TRY(cspmm(ctx, w, w.r, w.s, zr, -zi, w.part));  // s = A^H r
    HIPCHK(rfo::launch_colreduce(w.part, grid, sp, ssn, ctx->stream));
    HIPCHK(rfo::launch_cgls_scalars(sc, sp, 2, res_d, ctx->stream));
    HIPCHK(rfo::launch_cx_dir(w.s, w.p, w.x, al, be, n, sp, ctx->stream));  // x += alpha p, new p
    ++ctx->cgls_iters;
    if (it % 4 != 0 && it != max_iter) continue;
    TRY(converged(done));
    if (done) {
      *iters = it;
      ++ctx->cgls_solves;
      return RFO_OK;
    }
  }
  return fail(ctx, RFO_E_NUMERIC, "CGLS did not reach %g in %lld iterations (shift %g%+gi)", tol,
              (long long)max_iter, zr, zi);
}

// Free energy and gradient with the doubling moments: the forward pass runs
// K = floor(p/2) steps and F~ = const + sum_j a_j <y_j, y_j> + b_j <y_j, y_{j-1}>
// (a_j = 2 beta_2j, b_j = 2 beta_2j-1, b_1 = beta_1 - sum_{j>=2} beta_2j-1 for
// the terms below p).  Reverse recurrence as in the direct form, with the
// vector source g_j = dF~/dy_j = 2 a_j y_j + b_j y_{j-1} + b_{j+1} y_{j+1}:
//   z_K = g_K, z_{K-1} = g_{K-1} + 2 H_hat z_K, z_j = g_j + 2 H_hat z_{j+1} - z_{j+2},
//   dF~/dH_hat = z_1 y_0^T + 2 sum_{j=1}^{K-1} z_{j+1} y_j^T,
// symmetrized (the doubled form is a function of H_hat^T as well as H_hat; the
// gradient of F~ on symmetric matrices is the symmetric part).
int energy_grad_doubling(rfo_ctx *ctx, const Plan &pl, int64_t p, double *NEF_out,
                         double *dFdH_out) {
  const int kp = kernel_precision(ctx);
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  const int64_t K = p / 2;
  int64_t m = 2;
  while (m * m < K) ++m;
  const int64_t Q = (K + m - 1) / m;
  // with more than one segment, segment q's gradient can run on the side stream while
  // segment q - 1 replays and reverses on the main stream, the segments alternating
  // between two sets of y and z slots.  Measured on cu16k: FP32 5.62 against 5.80 s,
  // FP64 10.05 against 9.56 s (the persistent step kernels lose the CUs the gradient
  // holds), BF16 unchanged; so it is the default for FP32 only.
  bool overlap = Q > 1 && ctx->prec == RFO_FP32;
  if (const char *env = getenv("RFO_OVERLAP")) overlap = Q > 1 && atoi(env) != 0;
  const int n_sets = overlap ? 2 : 1;
  // vector slots: n_sets x (ys [m + 2] | zs [m + 2]) | checkpoints [2 (Q - 1)]
  const int64_t n_ys = m + 2, n_zs = m + 2, n_ck = Q > 1 ? 2 * (Q - 1) : 0;
  const int64_t set_slots = n_ys + n_zs;
  TRY(ensure(ctx, ctx->vec, (size_t)(n_sets * set_slots + n_ck) * pl.slot_bytes));
  if (overlap) {
    if (!ctx->side) HIPCHK(hipStreamCreateWithFlags(&ctx->side, hipStreamNonBlocking));
    for (hipEvent_t *e : {&ctx->ev_rev, &ctx->ev_sd[0], &ctx->ev_sd[1]})
      if (!*e) HIPCHK(hipEventCreateWithFlags(e, hipEventDisableTiming));
  }
  // the side stream has finished every gradient when this call returns, also on errors
  struct SideJoin {
    hipStream_t s;
    ~SideJoin() {
      if (s) (void)hipStreamSynchronize(s);
    }
  } side_join{overlap ? ctx->side : nullptr};
  DevBuf ckview;
  ckview.p = vec_at(ctx, pl, ctx->vec, n_sets * set_slots);
  ckview.bytes = (size_t)n_ck * pl.slot_bytes;
  Checkpoints ck;
  ck.m = m;
  ck.Q = Q;
  ck.store = &ckview;
  size_t n_events = 0;
  TRY(run_forward(ctx, pl, p, ctx->vec, false, &ck, &n_events, true));
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                            ctx->sp, obs, ctx->stream));
  // source weights from beta^g (host copy of the device coefficients)
  std::vector<double> beta((size_t)p);
  HIPCHK(hipMemcpyAsync(beta.data(), P<double>(ctx->coef) + 2 * p, p * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  std::vector<double> a(K + 2, 0.0), b(K + 2, 0.0);
  for (int64_t j = 1; j <= K; ++j) {
    if (2 * j <= p - 1) a[j] = 2.0 * beta[2 * j];
    if (j >= 2 && 2 * j - 1 <= p - 1) b[j] = 2.0 * beta[2 * j - 1];
  }
  b[1] = beta[1];
  for (int64_t j = 2; j <= K; ++j)
    if (2 * j - 1 <= p - 1) b[1] -= beta[2 * j - 1];

  const size_t vb = pl.slot_bytes;
  int cur = 0;  // slot set of the segment being processed
  auto ys = [&](int64_t t) { return vec_at(ctx, pl, ctx->vec, cur * set_slots + t); };
  auto zs = [&](int64_t t) { return vec_at(ctx, pl, ctx->vec, cur * set_slots + n_ys + t); };
  auto zs_of = [&](int set, int64_t t) { return vec_at(ctx, pl, ctx->vec, set * set_slots + n_ys + t); };
  auto cka = [&](int64_t q) { return vec_at(ctx, pl, ctx->vec, n_sets * set_slots + 2 * (q - 1)); };
  auto ckb = [&](int64_t q) { return vec_at(ctx, pl, ctx->vec, n_sets * set_slots + 2 * (q - 1) + 1); };
  bool sd_pending[2] = {false, false};  // a gradient on the side stream still reads the set
  rfo::StepArgs sa;
  fill_step(ctx, pl, sa);
  rfo::InitArgs ia;
  fill_init(ctx, pl, ia);
  for (int64_t q = Q - 1; q >= 0; --q) {
    const int64_t j0 = q * m, j1 = std::min(j0 + m, K), len = j1 - j0;
    cur = overlap ? (int)(q & 1) : 0;
    if (sd_pending[cur]) {
      // the gradient of segment q + 2 read this set: wait before rewriting it
      HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_sd[cur], 0));
      sd_pending[cur] = false;
    }
    // replay y_j, j in [j0, min(j1 + 2, K + 1)), into ys[0 ..): the sources of
    // z_{j1} and z_{j1-1} need y_{j1} and y_{j1+1}
    const int64_t rlen = std::min(j1 + 2, K + 1) - j0;
    if (q == 0) {
      ia.out = ys(0);
      ia.scale = nullptr;
      ia.acc = nullptr;
      ia.part = nullptr;
      HIPCHK(launch_init_slot(ctx, pl, ia));
    } else {
      HIPCHK(hipMemcpyAsync(ys(0), ckb(q), vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    sa.beta = nullptr;
    sa.acc = nullptr;
    sa.part = nullptr;
    sa.part2 = nullptr;
    for (int64_t t = 1; t < rlen; ++t) {
      sa.x = ys(t - 1);
      if (t == 1) {
        sa.prev = (j0 == 0) ? nullptr : cka(q);
        sa.c1 = (j0 == 0) ? 1.0 : 2.0;
        sa.c2 = (j0 == 0) ? 0.0 : -1.0;
      } else {
        sa.prev = ys(t - 2);
        sa.c1 = 2.0;
        sa.c2 = -1.0;
      }
      sa.out = ys(t);
      sa.nsrc = 0;
      HIPCHK(launch_any_step(ctx, pl, sa));
    }
    // reverse: zs[t] = z_i, i = j0 + 1 + t; y_i is ys[t + 1]
    for (int64_t t = len - 1; t >= 0; --t) {
      const int64_t i = j0 + 1 + t;
      sa.src[0] = ys(t + 1);
      sa.srcw[0] = 2.0 * a[i];
      sa.src[1] = ys(t);
      sa.srcw[1] = b[i];
      sa.nsrc = 2;
      if (i + 1 <= K) {
        sa.src[2] = ys(t + 2);
        sa.srcw[2] = b[i + 1];
        sa.nsrc = 3;
      }
      if (i == K) {
        sa.x = ys(t + 1);  // any valid vector: c1 = 0
        sa.prev = nullptr;
        sa.c1 = 0.0;
        sa.c2 = 0.0;
      } else {
        sa.x = zs(t + 1);
        sa.prev = (i == K - 1) ? nullptr : zs(t + 2);
        sa.c1 = 2.0;
        sa.c2 = (i == K - 1) ? 0.0 : -1.0;
      }
      sa.out = zs(t);
      HIPCHK(launch_any_step(ctx, pl, sa));
    }
    sa.nsrc = 0;
    // G += 1/2 sum_{j in segment} c_j (z_{j+1} y_j^T + y_j z_{j+1}^T) on the blocks on
    // and above the diagonal, c_0 = 1, c_j = 2; times 2/(e_max - e_min)
    rfo::SddmmArgs sd;
    memset(&sd, 0, sizeof(sd));
    sd.brow = P<int64_t>(ctx->brow);
    sd.col = P<int32_t>(ctx->col);
    sd.nnzb = ctx->nnzb;
    sd.bd = ctx->bd;
    sd.sp = ctx->sp;
    sd.xbase = zs(0);
    sd.xstride = (int64_t)(pl.slot_bytes / pl.vt_bytes);
    sd.ybase = ys(0);
    sd.ystride = (int64_t)(pl.slot_bytes / pl.vt_bytes);
    sd.w = P<double>(ctx->w);
    sd.count = (int)len;
    sd.j0 = j0;
    sd.scale = 1.0 / (ctx->e_max - ctx->e_min);
    sd.first = 1.0;
    sd.rest = 2.0;
    sd.G = P<double>(ctx->G);
    sd.accumulate = (q == Q - 1) ? 0 : 1;
    sd.nzlist = P<int64_t>(ctx->nz_up);
    sd.nlist = ctx->n_up;
    sd.ppl = sddmm_ppl(ctx);
    sd.sym = 1;
    hipStream_t sd_stream = ctx->stream;
    if (overlap) {
      HIPCHK(hipEventRecord(ctx->ev_rev, ctx->stream));
      HIPCHK(hipStreamWaitEvent(ctx->side, ctx->ev_rev, 0));
      sd_stream = ctx->side;
    }
    if (use_mfma_sddmm(ctx)) {
      // the BF16 copies the BF16 steps gather, on the matrix cores
      rfo::SddmmMfmaArgs sm;
      memset(&sm, 0, sizeof(sm));
      const size_t off = pl.vec_elems * sizeof(float);
      sm.grp = P<int64_t>(ctx->up_grp);
      sm.n_grp = ctx->n_up_grp;
      sm.nzlist = sd.nzlist;
      sm.brow = sd.brow;
      sm.col = sd.col;
      sm.sp = ctx->sp;
      sm.s_real = (int)ctx->s;
      sm.xbase = zs(0) + off;
      sm.ybase = ys(0) + off;
      sm.xstride = sm.ystride = (int64_t)(pl.slot_bytes / 2);
      sm.count = sd.count;
      sm.j0 = j0;
      sm.scale = sd.scale;
      sm.first = sd.first;
      sm.rest = sd.rest;
      sm.w0 = ctx->w_uniform;
      sm.G = sd.G;
      sm.accumulate = sd.accumulate;
      HIPCHK(rfo::launch_sddmm_bf16(sm, sd_stream));
    } else {
      HIPCHK(rfo::launch_sddmm(kp, sd, sd_stream));
    }
    if (overlap) {
      HIPCHK(hipEventRecord(ctx->ev_sd[cur], ctx->side));
      sd_pending[cur] = true;
    }
    if (q > 0) {
      // carries for the segment below (its set): zs[m] = z_{j0+1}, zs[m+1] = z_{j0+2}
      const int next = overlap ? (int)((q - 1) & 1) : 0;
      if (sd_pending[next] && next != cur) {
        HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_sd[next], 0));
        sd_pending[next] = false;
      }
      HIPCHK(hipMemcpyAsync(zs_of(next, m), zs(0), vb, hipMemcpyDeviceToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(zs_of(next, m + 1), zs(1), vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  for (int set = 0; set < 2; ++set)
    if (sd_pending[set]) HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_sd[set], 0));
  HIPCHK(rfo::launch_mirror(P<int64_t>(ctx->nz_low), ctx->n_low, P<int64_t>(ctx->tpos), ctx->bd,
                            P<double>(ctx->G), ctx->stream));
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  TRY(copy_out(ctx, dFdH_out, ctx->G.p, gbytes));
  TRY(check_flags_and_finish(ctx, n_events));
  ctx->has_grad = true;
  ctx->has_dens = false;
  ctx->mom_p = p;
  return RFO_OK;
}

}  // namespace

extern "C" {

int rfo_create(rfo_ctx **out, int device, void *hip_stream) {
  if (!out) {
    g_create_error = "out is NULL";
    return RFO_E_INVALID;
  }
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || count == 0) {
    g_create_error = std::string("no HIP device: ") + hipGetErrorString(e);
    return RFO_E_DEVICE;
  }
  if (device < 0 || device >= count) {
    g_create_error = "device index out of range";
    return RFO_E_INVALID;
  }
  e = hipSetDevice(device);
  if (e != hipSuccess) {
    g_create_error = std::string("hipSetDevice failed: ") + hipGetErrorString(e);
    return RFO_E_DEVICE;
  }
  rfo_ctx *c = new rfo_ctx();
  c->device = device;
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      cus > 0)
    c->cus = cus;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipHostMalloc(reinterpret_cast<void **>(&c->flags_h), sizeof(int)) != hipSuccess ||
      ensure(c, c->flags, sizeof(int)) != RFO_OK) {
    g_create_error = "allocation of the status flag failed";
    delete c;
    return RFO_E_NOMEM;
  }
  *out = c;
  return RFO_OK;
}

void rfo_destroy(rfo_ctx *ctx) { delete ctx; }

const char *rfo_last_error(const rfo_ctx *ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

int rfo_set_hamiltonian(rfo_ctx *ctx, int64_t n_block_rows, int block_dim, const int64_t *row_ptr,
                        const int32_t *col_idx, const double *values, double e_min,
                        double e_max, int precision) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  ctx->mom_p = 0;
  if (block_dim != 1 && block_dim != 9)
    return fail(ctx, RFO_E_INVALID, "block_dim must be 1 or 9 (got %d)", block_dim);
  if (n_block_rows < 1 || n_block_rows > ((int64_t)1 << 30))
    return fail(ctx, RFO_E_INVALID, "n_block_rows out of range");
  if (precision != RFO_FP64 && precision != RFO_FP32 && precision != RFO_BF16)
    return fail(ctx, RFO_E_INVALID, "unknown precision %d", precision);
  if (precision == RFO_BF16 && block_dim != 9)
    return fail(ctx, RFO_E_UNSUPPORTED, "BF16 MFMA steps need 9x9 blocks");
  if (!values) return fail(ctx, RFO_E_INVALID, "values is NULL");
  if (!std::isfinite(e_min) || !std::isfinite(e_max))
    return fail(ctx, RFO_E_INVALID, "e_min and e_max must be finite");
  const bool keep_pattern = (row_ptr == nullptr && col_idx == nullptr);
  if ((row_ptr == nullptr) != (col_idx == nullptr))
    return fail(ctx, RFO_E_INVALID, "row_ptr and col_idx must both be given or both be NULL");
  HIPCHK(hipSetDevice(ctx->device));

  if (keep_pattern) {
    if (!ctx->has_h && ctx->row_ptr_h.empty())
      return fail(ctx, RFO_E_STATE, "no previous pattern to keep");
    if (n_block_rows != ctx->nb || block_dim != ctx->bd)
      return fail(ctx, RFO_E_INVALID, "n_block_rows/block_dim differ from the kept pattern");
  } else {
    // ---- host validation of the pattern
    const int64_t nb = n_block_rows;
    if (row_ptr[0] != 0) return fail(ctx, RFO_E_INVALID, "row_ptr[0] must be 0");
    for (int64_t i = 0; i < nb; ++i)
      if (row_ptr[i + 1] < row_ptr[i]) return fail(ctx, RFO_E_INVALID, "row_ptr not monotone at %lld", (long long)i);
    const int64_t nnzb = row_ptr[nb];
    if (nnzb < nb || nnzb > ((int64_t)1 << 34)) return fail(ctx, RFO_E_INVALID, "bad nnzb %lld", (long long)nnzb);
    std::vector<int64_t> tpos(nnzb), brow(nnzb);
    for (int64_t I = 0; I < nb; ++I) {
      bool diag = false;
      for (int64_t z = row_ptr[I]; z < row_ptr[I + 1]; ++z) {
        const int32_t J = col_idx[z];
        if (J < 0 || J >= nb) return fail(ctx, RFO_E_INVALID, "col_idx out of range in row %lld", (long long)I);
        if (z > row_ptr[I] && col_idx[z - 1] >= J)
          return fail(ctx, RFO_E_INVALID, "col_idx not strictly increasing in row %lld", (long long)I);
        if (J == I) diag = true;
        brow[z] = I;
      }
      if (!diag) return fail(ctx, RFO_E_INVALID, "block row %lld has no diagonal block", (long long)I);
    }
    for (int64_t I = 0; I < nb; ++I) {
      for (int64_t z = row_ptr[I]; z < row_ptr[I + 1]; ++z) {
        const int32_t J = col_idx[z];
        const int32_t *b0 = col_idx + row_ptr[J], *b1 = col_idx + row_ptr[J + 1];
        const int32_t *hit = std::lower_bound(b0, b1, (int32_t)I);
        if (hit == b1 || *hit != (int32_t)I)
          return fail(ctx, RFO_E_INVALID, "pattern not symmetric: (%lld,%d) has no mirror",
                      (long long)I, J);
        tpos[z] = hit - col_idx;
      }
    }
    const int64_t n = nb * block_dim;
    if (ctx->has_r && n != ctx->n) {
      ctx->has_r = false;
      ctx->s = 0;
    }
    ctx->has_h = false;
    ctx->has_grad = false;
    ctx->nb = nb;
    ctx->bd = block_dim;
    ctx->n = n;
    ctx->nnzb = nnzb;
    ctx->row_ptr_h.assign(row_ptr, row_ptr + nb + 1);
    ctx->max_row = 0;
    for (int64_t I = 0; I < nb; ++I) ctx->max_row = std::max(ctx->max_row, row_ptr[I + 1] - row_ptr[I]);
    ctx->col_h.assign(col_idx, col_idx + nnzb);
    TRY(ensure(ctx, ctx->row_ptr, (nb + 1) * sizeof(int64_t)));
    TRY(ensure(ctx, ctx->col, (nnzb + rfo::kStepPad) * sizeof(int32_t)));
    TRY(ensure(ctx, ctx->brow, nnzb * sizeof(int64_t)));
    TRY(ensure(ctx, ctx->tpos, nnzb * sizeof(int64_t)));
    HIPCHK(hipMemcpyAsync(ctx->row_ptr.p, row_ptr, (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->col.p, col_idx, nnzb * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemsetAsync(P<int32_t>(ctx->col) + nnzb, 0, rfo::kStepPad * sizeof(int32_t), ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->brow.p, brow.data(), nnzb * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    HIPCHK(hipMemcpyAsync(ctx->tpos.p, tpos.data(), nnzb * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    // blocks on and above the block diagonal (computed by the gradient) and below it (mirrored)
    std::vector<int64_t> up, low;
    up.reserve(nnzb / 2 + nb);
    low.reserve(nnzb / 2);
    for (int64_t z = 0; z < nnzb; ++z) (brow[z] <= (int64_t)col_idx[z] ? up : low).push_back(z);
    TRY(ensure(ctx, ctx->nz_up, up.size() * sizeof(int64_t)));
    TRY(ensure(ctx, ctx->nz_low, std::max<size_t>(1, low.size()) * sizeof(int64_t)));
    HIPCHK(hipMemcpyAsync(ctx->nz_up.p, up.data(), up.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    if (!low.empty())
      HIPCHK(hipMemcpyAsync(ctx->nz_low.p, low.data(), low.size() * sizeof(int64_t), hipMemcpyHostToDevice, ctx->stream));
    ctx->n_up = (int64_t)up.size();
    ctx->n_low = (int64_t)low.size();

    HIPCHK(hipStreamSynchronize(ctx->stream));  // host vectors go out of scope
  }
  ctx->has_h = false;
  ctx->has_grad = false;
  const size_t nval = (size_t)ctx->nnzb * ctx->bd * ctx->bd;
  const size_t npad = (size_t)rfo::kStepPad * ctx->bd * ctx->bd;
  // H_hat, S and the unmapped H all carry kStepPad zero blocks: the 9x9 step
  // reads whole chunks of blocks
  TRY(ensure(ctx, ctx->hraw, (nval + npad) * sizeof(double)));
  HIPCHK(hipMemsetAsync(P<double>(ctx->hraw) + nval, 0, npad * sizeof(double), ctx->stream));
  TRY(ensure(ctx, ctx->h64, (nval + npad) * sizeof(double)));
  HIPCHK(hipMemsetAsync(P<double>(ctx->h64) + nval, 0, npad * sizeof(double), ctx->stream));
  if (precision == RFO_FP32) {
    TRY(ensure(ctx, ctx->h32, (nval + npad) * sizeof(float)));
    HIPCHK(hipMemsetAsync(P<float>(ctx->h32) + nval, 0, npad * sizeof(float), ctx->stream));
  }
  if (precision == RFO_BF16) {
    // K chunks: block row I's blocks concatenated along K (9 rows each), cut into
    // chunks of 16 K rows; K row k of the row is column c = k % 9 of block
    // nz = row_ptr[I] + k / 9
    const std::vector<int64_t> &rp = ctx->row_ptr_h;
    const std::vector<int32_t> &cl = ctx->col_h;
    if ((int64_t)ctx->nnzb * 9 >= ((int64_t)1 << 31) || ctx->n >= ((int64_t)1 << 31))
      return fail(ctx, RFO_E_UNSUPPORTED, "BF16 steps index rows with 32 bits");
    std::vector<int64_t> kp((size_t)ctx->nb + 1, 0);
    for (int64_t I = 0; I < ctx->nb; ++I) kp[I + 1] = kp[I] + (9 * (rp[I + 1] - rp[I]) + 15) / 16;
    const int64_t nch = kp[ctx->nb];
    std::vector<int32_t> kidx((size_t)nch * 16, -1), ksrc((size_t)nch * 16, -1);
    for (int64_t I = 0; I < ctx->nb; ++I)
      for (int64_t k = 0; k < 9 * (rp[I + 1] - rp[I]); ++k) {
        const int64_t nz = rp[I] + k / 9, c = k % 9;
        kidx[(size_t)(kp[I] * 16 + k)] = (int32_t)((int64_t)cl[nz] * 9 + c);
        ksrc[(size_t)(kp[I] * 16 + k)] = (int32_t)(nz * 9 + c);
      }
    ctx->n_chunks = nch;
    const size_t nq = (size_t)std::max<int64_t>(nch, 1);
    TRY(ensure(ctx, ctx->kc_ptr, kp.size() * sizeof(int64_t)));
    TRY(ensure(ctx, ctx->kc_idx, nq * 16 * sizeof(int32_t)));
    TRY(ensure(ctx, ctx->kc_src, nq * 16 * sizeof(int32_t)));
    TRY(ensure(ctx, ctx->hbf16, nq * 36 * 8));
    HIPCHK(hipMemcpyAsync(ctx->kc_ptr.p, kp.data(), kp.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          ctx->stream));
    if (nch > 0) {
      HIPCHK(hipMemcpyAsync(ctx->kc_idx.p, kidx.data(), kidx.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(ctx->kc_src.p, ksrc.data(), ksrc.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, ctx->stream));
    }
    // the host vectors go out of scope: wait for the copies
    HIPCHK(hipStreamSynchronize(ctx->stream));
  }
  HIPCHK(hipMemcpyAsync(ctx->hraw.p, values, nval * sizeof(double), hipMemcpyDefault, ctx->stream));

  ctx->has_s = false;  // a new H drops the overlap (set it again after this call)
  ctx->has_q = false;
  ctx->has_dens = false;
  ctx->interval_given = e_min < e_max;
  if (e_min >= e_max) {
    const int nblk = (int)((ctx->n + rfo::kWG - 1) / rfo::kWG);
    TRY(ensure(ctx, ctx->gscratch, (size_t)2 * nblk * sizeof(double)));
    TRY(ensure(ctx, ctx->small, 64 * sizeof(double)));
    HIPCHK(rfo::launch_gershgorin(P<double>(ctx->hraw), P<int64_t>(ctx->row_ptr), P<int32_t>(ctx->col),
                                  ctx->nb, ctx->bd, P<double>(ctx->gscratch), P<double>(ctx->small),
                                  ctx->stream));
    double lohi[2];
    HIPCHK(hipMemcpyAsync(lohi, ctx->small.p, sizeof(lohi), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    if (!std::isfinite(lohi[0]) || !std::isfinite(lohi[1]))
      return fail(ctx, RFO_E_NUMERIC, "non-finite Hamiltonian values");
    const double c = 0.5 * (lohi[0] + lohi[1]);
    double h = 1.01 * 0.5 * (lohi[1] - lohi[0]);
    h = std::max(h, 1e-12 * std::max(1.0, std::fabs(c)));
    e_min = c - h;
    e_max = c + h;
  }
  ctx->e_min = e_min;
  ctx->e_max = e_max;
  ctx->prec = precision;
  HIPCHK(hipMemsetAsync(ctx->flags.p, 0, sizeof(int), ctx->stream));
  HIPCHK(rfo::launch_map(P<double>(ctx->hraw), P<int64_t>(ctx->brow), P<int32_t>(ctx->col),
                         P<int64_t>(ctx->tpos), ctx->nnzb, ctx->bd, e_min, e_max,
                         P<double>(ctx->h64), precision == RFO_FP32 ? P<float>(ctx->h32) : nullptr,
                         P<int>(ctx->flags), ctx->stream));
  if (precision == RFO_BF16)
    HIPCHK(rfo::launch_pack_bf16(P<double>(ctx->h64), P<int32_t>(ctx->kc_src), ctx->n_chunks,
                                 ctx->hbf16.p, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->flags_h, ctx->flags.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*ctx->flags_h & 1) return fail(ctx, RFO_E_NUMERIC, "non-finite Hamiltonian values");
  if (*ctx->flags_h & 2) return fail(ctx, RFO_E_INVALID, "Hamiltonian values are not symmetric (H_JI != H_IJ^T)");
  ctx->has_up_grp = false;
  if (block_dim == 9 && precision == RFO_BF16) {
    // groups of the upper blocks (J >= I, in the order of the upper-block list)
    const int gb = rfo::kSddmmGroup;
    const std::vector<int64_t> &rp = ctx->row_ptr_h;
    const std::vector<int32_t> &cl = ctx->col_h;
    std::vector<int64_t> grp(1, 0);
    int64_t q = 0;
    for (int64_t I = 0; I < ctx->nb; ++I) {
      int64_t in_row = 0;
      for (int64_t z = rp[I]; z < rp[I + 1]; ++z) {
        if ((int64_t)cl[z] < I) continue;
        ++q;
        if (++in_row % gb == 0) grp.push_back(q);
      }
      if (in_row % gb != 0) grp.push_back(q);
    }
    if (q != ctx->n_up) return fail(ctx, RFO_E_DEVICE, "internal: upper block count mismatch");
    ctx->n_up_grp = (int64_t)grp.size() - 1;
    TRY(ensure(ctx, ctx->up_grp, grp.size() * sizeof(int64_t)));
    HIPCHK(hipMemcpyAsync(ctx->up_grp.p, grp.data(), grp.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                          ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));  // grp goes out of scope
    ctx->has_up_grp = true;
  }
  ctx->has_h = true;
  return RFO_OK;
}

int rfo_get_interval(const rfo_ctx *ctx, double *e_min, double *e_max) {
  if (!ctx || !e_min || !e_max) return RFO_E_INVALID;
  if (!ctx->has_h) return RFO_E_STATE;
  *e_min = ctx->e_min;
  *e_max = ctx->e_max;
  return RFO_OK;
}

int rfo_set_probes(rfo_ctx *ctx, int64_t n_probes, const double *R, const double *weights) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  ctx->mom_p = 0;
  ctx->has_dens = false;
  ctx->has_q = false;
  if (!ctx->has_h) return fail(ctx, RFO_E_STATE, "set the Hamiltonian before the probes");
  if (!R) return fail(ctx, RFO_E_INVALID, "R is NULL");
  if (n_probes < 1 || n_probes > (1 << 20)) return fail(ctx, RFO_E_INVALID, "n_probes out of range");
  if (weights)
    for (int64_t c = 0; c < n_probes; ++c)
      if (!std::isfinite(weights[c])) return fail(ctx, RFO_E_INVALID, "non-finite weight");
  HIPCHK(hipSetDevice(ctx->device));
  ctx->has_r = false;
  ctx->has_grad = false;
  // padded probe count: a multiple of 64, and of 128 above 64 probes so that FP64
  // waves can take 2 probes per lane (16 B loads); padding probes have weight 0
  const int sp = n_probes <= 64 ? 64 : (int)((n_probes + 127) / 128 * 128);
  const size_t n = (size_t)ctx->n;
  TRY(ensure(ctx, ctx->rden, n * sp * sizeof(double)));
  TRY(ensure(ctx, ctx->sgn, n * (sp / 64) * sizeof(uint64_t)));
  TRY(ensure(ctx, ctx->w, sp * sizeof(double)));
  HIPCHK(hipMemsetAsync(ctx->rden.p, 0, n * sp * sizeof(double), ctx->stream));
  HIPCHK(hipMemcpy2DAsync(ctx->rden.p, sp * sizeof(double), R, n_probes * sizeof(double),
                          n_probes * sizeof(double), n, hipMemcpyHostToDevice, ctx->stream));
  std::vector<double> w(sp, 0.0);
  for (int64_t c = 0; c < n_probes; ++c) w[c] = weights ? weights[c] : 1.0 / (double)n_probes;
  ctx->w_uniform = w[0];
  for (int64_t c = 1; c < n_probes; ++c)
    if (w[c] != w[0]) ctx->w_uniform = 0.0;
  HIPCHK(hipMemcpyAsync(ctx->w.p, w.data(), sp * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->flags.p, 0, sizeof(int), ctx->stream));
  HIPCHK(rfo::launch_probe_pack(P<double>(ctx->rden), (int64_t)n, (int)n_probes, sp,
                                P<uint64_t>(ctx->sgn), P<int>(ctx->flags), ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->flags_h, ctx->flags.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*ctx->flags_h & 2) return fail(ctx, RFO_E_NUMERIC, "non-finite probe entries");
  ctx->signs = (*ctx->flags_h & 1) == 0;
  if (ctx->signs) release(ctx->rden);
  ctx->s = n_probes;
  ctx->sp = sp;
  ctx->has_r = true;
  return RFO_OK;
}

int rfo_fermi_moments(rfo_ctx *ctx, double T, double mu, int64_t n_terms, double *moments_out,
                      double *NEF_out, double *density_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  Plan pl;
  TRY(prepare_call(ctx, T, mu, n_terms, pl));
  const bool dens = density_out != nullptr;
  // vector slots: y pair; with an overlap also t and the CG vectors r, p, q
  TRY(ensure(ctx, ctx->vec, (ctx->has_s ? 6 : 2) * pl.slot_bytes));
  if (dens) TRY(ensure(ctx, ctx->acc, pl.vec_elems * pl.vt_bytes));
  if (ctx->has_s) TRY(ensure_cg(ctx));
  size_t n_events = 0;
  TRY(run_forward(ctx, pl, n_terms, ctx->vec, dens, nullptr, &n_events,
                  !dens && ctx->doubling && !ctx->has_s));
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef),
                            n_terms, ctx->sp, obs, ctx->stream));
  ctx->has_q = false;
  ctx->has_dens = false;
  if (dens) {
    TRY(ensure(ctx, ctx->G, (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double)));
    // P r = S^{-1} acc and Q r = S^{-1} H S^{-1} acc with an overlap (Eq. poly_PQ)
    void *px = ctx->acc.p, *qx = nullptr;
    if (ctx->has_s) {
      px = vec_at(ctx, pl, ctx->vec, 2);
      TRY(cg_solve(ctx, pl, ctx->vec, ctx->acc.p, px));
      rfo::StepArgs sa;
      fill_step(ctx, pl, sa);
      sa.hval = ctx->hraw.p;  // v = H u with the unmapped Hamiltonian
      sa.x = px;
      sa.prev = nullptr;
      sa.out = vec_at(ctx, pl, ctx->vec, 0);
      sa.c1 = 1.0;
      sa.c2 = 0.0;
      HIPCHK(launch_any_step(ctx, pl, sa));
      qx = vec_at(ctx, pl, ctx->vec, 1);
      TRY(cg_solve(ctx, pl, ctx->vec, vec_at(ctx, pl, ctx->vec, 0), qx));
      TRY(ensure(ctx, ctx->GQ, (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double)));
    }
    rfo::SddmmArgs a;
    memset(&a, 0, sizeof(a));
    a.brow = P<int64_t>(ctx->brow);
    a.col = P<int32_t>(ctx->col);
    a.nnzb = ctx->nnzb;
    a.bd = ctx->bd;
    a.sp = ctx->sp;
    a.xbase = px;
    a.ybase = nullptr;
    a.sgn = ctx->signs ? P<uint64_t>(ctx->sgn) : nullptr;
    a.rden = ctx->signs ? nullptr : P<double>(ctx->rden);
    a.w = P<double>(ctx->w);
    a.count = 1;
    a.scale = 1.0;
    a.first = 1.0;
    a.rest = 1.0;
    a.G = P<double>(ctx->G);
    a.accumulate = 0;
    a.nzlist = nullptr;
    a.ppl = sddmm_ppl(ctx);
    HIPCHK(rfo::launch_sddmm(kernel_precision(ctx), a, ctx->stream));
    if (qx) {
      a.xbase = qx;
      a.G = P<double>(ctx->GQ);
      HIPCHK(rfo::launch_sddmm(kernel_precision(ctx), a, ctx->stream));
      ctx->has_q = true;
    }
    ctx->has_grad = false;  // G now holds the density
    ctx->has_dens = true;
    TRY(copy_out(ctx, density_out, ctx->G.p, (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double)));
  }
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  TRY(check_flags_and_finish(ctx, n_events));
  TRY(copy_moments_out(ctx, n_terms, moments_out));
  ctx->mom_p = n_terms;
  return RFO_OK;
}

int rfo_traces_at(rfo_ctx *ctx, double T, double mu, double *NEF_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (ctx->mom_p < 1) return fail(ctx, RFO_E_STATE, "no moments: call rfo_fermi_moments first");
  if (!NEF_out) return fail(ctx, RFO_E_INVALID, "NEF_out is NULL");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(ctx, RFO_E_INVALID, "T must be finite and > 0");
  if (!std::isfinite(mu)) return fail(ctx, RFO_E_INVALID, "mu must be finite");
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t p = ctx->mom_p, nq = 4 * p;
  HIPCHK(rfo::launch_coefficients(ctx->e_min, ctx->e_max, T, mu, p, nq, P<double>(ctx->samples),
                                  P<double>(ctx->costab), P<double>(ctx->coef), ctx->stream));
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                            ctx->sp, obs, ctx->stream));
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RFO_OK;
}

int rfo_energy_and_dEdH(rfo_ctx *ctx, double T, double mu, int64_t n_terms, double *NEF_out,
                        double *dFdH_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  Plan pl;
  TRY(prepare_call(ctx, T, mu, n_terms, pl));
  const int64_t p = n_terms;
  if (ctx->has_s)
    return fail(ctx, RFO_E_UNSUPPORTED,
                "the free-energy gradient with an overlap is not implemented; use the density "
                "blocks and rfo_density_forces");
  if (ctx->doubling && p >= 2) {
    TRY(ensure(ctx, ctx->G, (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double)));
    ctx->has_grad = false;
    return energy_grad_doubling(ctx, pl, p, NEF_out, dFdH_out);
  }
  const int kp = kernel_precision(ctx);
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  TRY(ensure(ctx, ctx->G, gbytes));
  ctx->has_grad = false;
  const int64_t P1 = p - 1;  // gradient terms use y_j, j = 0 .. p-2
  int64_t m = 2;
  while (m * m < P1) ++m;
  const int64_t Q = P1 > 0 ? (P1 + m - 1) / m : 0;
  // vector slots: ys [m] | zs [m + 2] | checkpoints [2 (Q - 1)]
  const int64_t n_ys = m, n_zs = m + 2, n_ck = Q > 1 ? 2 * (Q - 1) : 0;
  TRY(ensure(ctx, ctx->vec, (size_t)(n_ys + n_zs + n_ck) * pl.slot_bytes));
  const double *beta = P<double>(ctx->coef) + 2 * p;

  // forward pass (rolling pair in ys[0], ys[1]) with checkpoints y_{qm-1}, y_{qm}
  DevBuf ckview;
  ckview.p = vec_at(ctx, pl, ctx->vec, n_ys + n_zs);
  ckview.bytes = (size_t)n_ck * pl.slot_bytes;
  Checkpoints ck;
  ck.m = m;
  ck.Q = Q;
  ck.store = &ckview;
  size_t n_events = 0;
  TRY(run_forward(ctx, pl, p, ctx->vec, false, &ck, &n_events));
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                            ctx->sp, obs, ctx->stream));

  if (P1 == 0) {
    HIPCHK(hipMemsetAsync(ctx->G.p, 0, gbytes, ctx->stream));
  } else {
    const size_t vb = pl.slot_bytes;
    auto ys = [&](int64_t t) { return vec_at(ctx, pl, ctx->vec, t); };
    auto zs = [&](int64_t t) { return vec_at(ctx, pl, ctx->vec, n_ys + t); };
    auto cka = [&](int64_t q) { return vec_at(ctx, pl, ctx->vec, n_ys + n_zs + 2 * (q - 1)); };
    auto ckb = [&](int64_t q) { return vec_at(ctx, pl, ctx->vec, n_ys + n_zs + 2 * (q - 1) + 1); };
    rfo::StepArgs sa;
    fill_step(ctx, pl, sa);
    rfo::InitArgs ia;
    fill_init(ctx, pl, ia);
    for (int64_t q = Q - 1; q >= 0; --q) {
      const int64_t j0 = q * m, j1 = std::min(j0 + m, P1), len = j1 - j0;
      // replay y_j, j in [j0, j1), into ys[0 .. len)
      if (q == 0) {
        ia.out = ys(0);
        ia.scale = nullptr;
        ia.acc = nullptr;
        ia.part = nullptr;
        HIPCHK(launch_init_slot(ctx, pl, ia));
      } else {
        HIPCHK(hipMemcpyAsync(ys(0), ckb(q), vb, hipMemcpyDeviceToDevice, ctx->stream));
      }
      for (int64_t t = 1; t < len; ++t) {
        sa.x = ys(t - 1);
        if (t == 1) {
          sa.prev = (j0 == 0) ? nullptr : cka(q);
          sa.c1 = (j0 == 0) ? 1.0 : 2.0;
          sa.c2 = (j0 == 0) ? 0.0 : -1.0;
        } else {
          sa.prev = ys(t - 2);
          sa.c1 = 2.0;
          sa.c2 = -1.0;
        }
        sa.out = ys(t);
        sa.beta = nullptr;
        sa.acc = nullptr;
        sa.part = nullptr;
        HIPCHK(launch_any_step(ctx, pl, sa));
      }
      // reverse recurrence: zs[t] = z_{j0+1+t}; z_{p-1} = beta_{p-1} r,
      // z_{p-2} = 2 H_hat z_{p-1} + beta_{p-2} r, z_i = 2 H_hat z_{i+1} - z_{i+2} + beta_i r
      for (int64_t t = len - 1; t >= 0; --t) {
        const int64_t i = j0 + 1 + t;
        if (i == p - 1) {
          ia.out = zs(t);
          ia.scale = beta + (p - 1);
          ia.acc = nullptr;
          ia.part = nullptr;
          HIPCHK(launch_init_slot(ctx, pl, ia));
        } else {
          sa.x = zs(t + 1);
          sa.prev = (i == p - 2) ? nullptr : zs(t + 2);
          sa.c1 = 2.0;
          sa.c2 = (i == p - 2) ? 0.0 : -1.0;
          sa.out = zs(t);
          sa.beta = beta + i;
          sa.acc = nullptr;
          sa.part = nullptr;
          HIPCHK(launch_any_step(ctx, pl, sa));
        }
      }
      // G += sum_{j in segment} c_j z_{j+1} y_j^T, c_0 = 1, c_j = 2; times 2/(e_max - e_min)
      rfo::SddmmArgs a;
      memset(&a, 0, sizeof(a));
      a.brow = P<int64_t>(ctx->brow);
      a.col = P<int32_t>(ctx->col);
      a.nnzb = ctx->nnzb;
      a.bd = ctx->bd;
      a.sp = ctx->sp;
      a.xbase = zs(0);
      a.xstride = (int64_t)(pl.slot_bytes / pl.vt_bytes);
      a.ybase = ys(0);
      a.ystride = (int64_t)(pl.slot_bytes / pl.vt_bytes);
      a.w = P<double>(ctx->w);
      a.count = (int)len;
      a.j0 = j0;
      a.scale = 2.0 / (ctx->e_max - ctx->e_min);
      a.first = 1.0;
      a.rest = 2.0;
      a.G = P<double>(ctx->G);
      a.accumulate = (q == Q - 1) ? 0 : 1;
      // the full gradient is symmetric: blocks on and above the diagonal only
      a.nzlist = P<int64_t>(ctx->nz_up);
      a.nlist = ctx->n_up;
      a.ppl = sddmm_ppl(ctx);
      HIPCHK(rfo::launch_sddmm(kp, a, ctx->stream));
      if (q > 0) {
        // carries for the segment below: zs[m] = z_{j0+1}, zs[m+1] = z_{j0+2}
        HIPCHK(hipMemcpyAsync(zs(m), zs(0), vb, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(zs(m + 1), zs(1), vb, hipMemcpyDeviceToDevice, ctx->stream));
      }
    }
  }
  if (P1 > 0)
    HIPCHK(rfo::launch_mirror(P<int64_t>(ctx->nz_low), ctx->n_low, P<int64_t>(ctx->tpos), ctx->bd,
                              P<double>(ctx->G), ctx->stream));
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  TRY(copy_out(ctx, dFdH_out, ctx->G.p, gbytes));
  TRY(check_flags_and_finish(ctx, n_events));
  ctx->has_grad = true;
  ctx->has_dens = false;
  ctx->mom_p = p;
  return RFO_OK;
}

int rfo_hf_forces(rfo_ctx *ctx, const double *dHdR, double *forces_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_grad) return fail(ctx, RFO_E_STATE, "no gradient: call rfo_energy_and_dEdH first");
  if (!dHdR || !forces_out) return fail(ctx, RFO_E_INVALID, "NULL argument");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t dbytes = (size_t)ctx->nnzb * 3 * ctx->bd * ctx->bd * sizeof(double);
  TRY(ensure(ctx, ctx->dHdR, dbytes));
  TRY(ensure(ctx, ctx->forces, (size_t)ctx->nb * 3 * sizeof(double)));
  HIPCHK(hipMemcpyAsync(ctx->dHdR.p, dHdR, dbytes, hipMemcpyDefault, ctx->stream));
  HIPCHK(rfo::launch_forces(P<int64_t>(ctx->row_ptr), P<int64_t>(ctx->tpos), P<double>(ctx->G),
                            P<double>(ctx->dHdR), ctx->nb, ctx->bd, P<double>(ctx->forces), 1.0, 0,
                            ctx->stream));
  TRY(copy_out(ctx, forces_out, ctx->forces.p, (size_t)ctx->nb * 3 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RFO_OK;
}

int rfo_set_overlap(rfo_ctx *ctx, const double *values, double cg_tol) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_h) return fail(ctx, RFO_E_STATE, "set the Hamiltonian before the overlap");
  HIPCHK(hipSetDevice(ctx->device));
  ctx->mom_p = 0;
  ctx->has_q = false;
  ctx->has_grad = false;
  ctx->has_dens = false;
  if (!values) {  // back to S = I: the plain map of H
    ctx->has_s = false;
    HIPCHK(hipMemsetAsync(ctx->flags.p, 0, sizeof(int), ctx->stream));
    HIPCHK(rfo::launch_map(P<double>(ctx->hraw), P<int64_t>(ctx->brow), P<int32_t>(ctx->col),
                           P<int64_t>(ctx->tpos), ctx->nnzb, ctx->bd, ctx->e_min, ctx->e_max,
                           P<double>(ctx->h64), nullptr, P<int>(ctx->flags), ctx->stream));
    HIPCHK(hipStreamSynchronize(ctx->stream));
    return RFO_OK;
  }
  if (ctx->prec != RFO_FP64)
    return fail(ctx, RFO_E_UNSUPPORTED, "an overlap needs FP64 precision");
  if (!ctx->interval_given)
    return fail(ctx, RFO_E_STATE,
                "with an overlap pass the spectral interval of the pencil (H, S) to "
                "rfo_set_hamiltonian (the Gershgorin fallback bounds H alone)");
  if (!(cg_tol > 0.0) || !(cg_tol < 1.0)) cg_tol = 1e-13;
  const size_t nval = (size_t)ctx->nnzb * ctx->bd * ctx->bd;
  const size_t npad = (size_t)rfo::kStepPad * ctx->bd * ctx->bd;
  TRY(ensure(ctx, ctx->s64, (nval + npad) * sizeof(double)));
  HIPCHK(hipMemsetAsync(P<double>(ctx->s64) + nval, 0, npad * sizeof(double), ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->s64.p, values, nval * sizeof(double), hipMemcpyDefault, ctx->stream));
  HIPCHK(hipMemsetAsync(ctx->flags.p, 0, sizeof(int), ctx->stream));
  HIPCHK(rfo::launch_map_overlap(P<double>(ctx->hraw), P<double>(ctx->s64), P<int64_t>(ctx->tpos),
                                 ctx->nnzb, ctx->bd, ctx->e_min, ctx->e_max, P<double>(ctx->h64),
                                 P<int>(ctx->flags), ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->flags_h, ctx->flags.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*ctx->flags_h & 1) return fail(ctx, RFO_E_NUMERIC, "non-finite overlap values");
  if (*ctx->flags_h & 2) return fail(ctx, RFO_E_INVALID, "overlap values are not symmetric (S_JI != S_IJ^T)");
  ctx->has_s = true;
  ctx->cg_tol = cg_tol;
  return RFO_OK;
}

int rfo_get_density_q(rfo_ctx *ctx, double *q_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_q)
    return fail(ctx, RFO_E_STATE, "no Q blocks: call rfo_fermi_moments with density and an overlap");
  if (!q_out) return fail(ctx, RFO_E_INVALID, "q_out is NULL");
  TRY(copy_out(ctx, q_out, ctx->GQ.p, (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RFO_OK;
}

int rfo_density_forces(rfo_ctx *ctx, const double *dHdR, const double *dSdR, double *forces_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!dHdR || !forces_out) return fail(ctx, RFO_E_INVALID, "NULL argument");
  if (!ctx->has_dens)
    return fail(ctx, RFO_E_STATE, "no density blocks: call rfo_fermi_moments with density first");
  if (dSdR && !ctx->has_q)
    return fail(ctx, RFO_E_STATE, "no Q blocks: the last call had no overlap");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t dbytes = (size_t)ctx->nnzb * 3 * ctx->bd * ctx->bd * sizeof(double);
  TRY(ensure(ctx, ctx->dHdR, dbytes));
  TRY(ensure(ctx, ctx->forces, (size_t)ctx->nb * 3 * sizeof(double)));
  HIPCHK(hipMemcpyAsync(ctx->dHdR.p, dHdR, dbytes, hipMemcpyDefault, ctx->stream));
  // force_a = -(tr[P dH/dR_a] - tr[Q dS/dR_a]) (Observable response)
  HIPCHK(rfo::launch_forces(P<int64_t>(ctx->row_ptr), P<int64_t>(ctx->tpos), P<double>(ctx->G),
                            P<double>(ctx->dHdR), ctx->nb, ctx->bd, P<double>(ctx->forces), 1.0, 0,
                            ctx->stream));
  if (dSdR) {
    HIPCHK(hipMemcpyAsync(ctx->dHdR.p, dSdR, dbytes, hipMemcpyDefault, ctx->stream));
    HIPCHK(rfo::launch_forces(P<int64_t>(ctx->row_ptr), P<int64_t>(ctx->tpos), P<double>(ctx->GQ),
                              P<double>(ctx->dHdR), ctx->nb, ctx->bd, P<double>(ctx->forces), -1.0, 1,
                              ctx->stream));
  }
  TRY(copy_out(ctx, forces_out, ctx->forces.p, (size_t)ctx->nb * 3 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RFO_OK;
}

int rfo_rational_estimate(rfo_ctx *ctx, double mu, int64_t n_poles, const double *poles,
                          const double *res_f, const double *res_g, const double *poly, double tol,
                          int64_t max_iter, double *NEF_out, double *density_out,
                          double *dFdH_out, int64_t *iterations_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_h) return fail(ctx, RFO_E_STATE, "no Hamiltonian: call rfo_set_hamiltonian first");
  if (!ctx->has_r) return fail(ctx, RFO_E_STATE, "no probes: call rfo_set_probes first");
  if (ctx->prec != RFO_FP64)
    return fail(ctx, RFO_E_UNSUPPORTED, "the rational expansion runs in FP64 only");
  if (ctx->has_s && dFdH_out)
    return fail(ctx, RFO_E_UNSUPPORTED, "the rational free-energy gradient supports S = I only");
  if (n_poles < 1 || n_poles > 4096) return fail(ctx, RFO_E_INVALID, "n_poles must be in [1, 4096]");
  if (!poles || !res_f || !res_g || !poly) return fail(ctx, RFO_E_INVALID, "NULL fit argument");
  if (!(tol > 0.0 && tol < 1.0)) return fail(ctx, RFO_E_INVALID, "tol must be in (0, 1)");
  if (max_iter < 1 || max_iter > (1 << 24))
    return fail(ctx, RFO_E_INVALID, "max_iter must be in [1, 2^24]");
  if (!std::isfinite(mu)) return fail(ctx, RFO_E_INVALID, "mu must be finite");
  for (int t = 0; t < 3; ++t)
    if (!std::isfinite(poly[t])) return fail(ctx, RFO_E_INVALID, "non-finite polynomial part");
  for (int64_t k = 0; k < 2 * n_poles; ++k)
    if (!std::isfinite(poles[k]) || !std::isfinite(res_f[k]) || !std::isfinite(res_g[k]))
      return fail(ctx, RFO_E_INVALID, "non-finite pole or residue");
  for (int64_t k = 0; k < n_poles; ++k)
    if (!(poles[2 * k + 1] > 0.0))
      return fail(ctx, RFO_E_INVALID, "pole %lld is not in the upper half plane", (long long)k);
  HIPCHK(hipSetDevice(ctx->device));
  const int64_t n = ctx->n;
  const int sp = ctx->sp;
  const int64_t plane = n * sp;
  const bool dens = density_out != nullptr, grad = dFdH_out != nullptr;
  const double c = 0.5 * (ctx->e_max - ctx->e_min), d = 0.5 * (ctx->e_max + ctx->e_min);

  // launch decomposition of the complex product: the step kernel's row groups
  const Plan pl = make_plan(ctx);
  CxWork w;
  // two probes per lane where the tiles allow: one tile of 128 probes reads the
  // H_hat blocks once per product (measured faster for 1x1 and 9x9 blocks)
  w.ppl = sp % 128 == 0 ? 2 : 1;
  // with an overlap the 9x9 product keeps four row sums per probe: one probe per lane
  if (ctx->has_s && ctx->bd == 9) w.ppl = 1;
  if (const char *env = getenv("RFO_CPPL")) w.ppl = atoi(env) == 2 && sp % 128 == 0 ? 2 : 1;
  w.u = ctx->bd == 1 ? 4 : 1;
  if (const char *env = getenv("RFO_CU")) {
    const int u = atoi(env);
    if (ctx->bd == 1 ? (u == 4 || u == 8) : (u == 1 || u == 2)) w.u = u;
  }
  memset(&w.ca, 0, sizeof(w.ca));
  w.ca.row_ptr = P<int64_t>(ctx->row_ptr);
  w.ca.col = P<int32_t>(ctx->col);
  w.ca.hval = P<double>(ctx->h64);                            // H_hat (mapped with S when set)
  w.ca.sval = ctx->has_s ? P<double>(ctx->s64) : nullptr;
  w.ca.nb = ctx->nb;
  w.ca.plane = plane;
  w.ca.sp = sp;
  w.ca.rows_per_wg = pl.rows_per_wg;
  w.ca.n_rg = pl.n_rg;
  w.ca.n_pt = sp / (64 * w.ppl);
  {
    const int occ = std::max(1, rfo::cspmm_blocks_per_cu(ctx->bd, w.ppl, w.u, ctx->has_s));
    int64_t grid = (int64_t)ctx->cus * std::min(occ, 4);
    if (const char *env = getenv("RFO_CGRID")) grid = std::max<int64_t>(8, atoll(env));
    const int64_t units = (int64_t)w.ca.n_pt * w.ca.n_rg;
    grid = std::min(grid, (units + 7) / 8 * 8);
    w.ca.grid = (int)std::max<int64_t>(8, grid / 8 * 8);
  }
  w.nparts = std::max(rfo::cg_nparts(n), w.ca.grid);
  // planes: x, r, p, q, s (complex), the P r accumulator, and S r with an overlap
  TRY(ensure(ctx, ctx->rat, (size_t)(ctx->has_s ? 12 : 11) * plane * sizeof(double)));
  if (ctx->has_s) {
    TRY(ensure(ctx, ctx->vec, 6 * pl.slot_bytes));  // CG work slots
    TRY(ensure_cg(ctx));
  }
  TRY(ensure(ctx, ctx->rat_part, (size_t)2 * w.nparts * sp * sizeof(double)));
  TRY(ensure(ctx, ctx->rat_sc, ((size_t)7 * sp + 1) * sizeof(double)));
  TRY(ensure(ctx, ctx->rat_rho, ((size_t)2 * n_poles + 2) * sp * sizeof(double)));
  TRY(ensure(ctx, ctx->rat_coef, (size_t)6 * n_poles * sizeof(double)));
  TRY(ensure(ctx, ctx->small, 64 * sizeof(double)));
  if (!ctx->rat_res_h) HIPCHK(hipHostMalloc((void **)&ctx->rat_res_h, sizeof(double), 0));
  double *base = P<double>(ctx->rat);
  w.x = base;
  w.r = base + 2 * plane;
  w.p = base + 4 * plane;
  w.q = base + 6 * plane;
  w.s = base + 8 * plane;
  w.acc = base + 10 * plane;
  w.part = P<double>(ctx->rat_part);
  w.part2 = w.part + (size_t)w.nparts * sp;
  w.sc = P<double>(ctx->rat_sc);
  double *rho = P<double>(ctx->rat_rho);
  double *m01 = rho + (size_t)2 * n_poles * sp;
  const uint64_t *sgn = ctx->signs ? P<uint64_t>(ctx->sgn) : nullptr;
  const double *rden = ctx->signs ? nullptr : P<double>(ctx->rden);

  // trace coefficients of r . x_k per pole: N w_k / c, E w_k z_k / c, F tau_k / c
  ctx->rat_coef_h.assign((size_t)6 * n_poles, 0.0);
  double ew = 0.0;
  for (int64_t k = 0; k < n_poles; ++k) {
    const double zr = poles[2 * k], zi = poles[2 * k + 1];
    const double wr = res_f[2 * k], wi = res_f[2 * k + 1];
    const double tr = res_g[2 * k], ti = res_g[2 * k + 1];
    double *cf = ctx->rat_coef_h.data();
    cf[2 * k] = wr / c;
    cf[2 * k + 1] = wi / c;
    cf[2 * (n_poles + k)] = (wr * zr - wi * zi) / c;
    cf[2 * (n_poles + k) + 1] = (wr * zi + wi * zr) / c;
    cf[2 * (2 * n_poles + k)] = tr / c;
    cf[2 * (2 * n_poles + k) + 1] = ti / c;
    ew += 2.0 * wr;
  }
  HIPCHK(hipMemcpyAsync(ctx->rat_coef.p, ctx->rat_coef_h.data(), ctx->rat_coef_h.size() * sizeof(double),
                        hipMemcpyHostToDevice, ctx->stream));
  // the host array is rewritten by the next call: let the copy finish here
  HIPCHK(hipStreamSynchronize(ctx->stream));

  // x = R;  q = H R / c, the product with the shift -d/c (H = c H_hat + d S)
  HIPCHK(rfo::launch_cx_fill(sgn, rden, n, sp, 1.0, w.x, w.x + plane, ctx->stream));
  TRY(cspmm(ctx, w, w.x, w.q, -d / c, 0.0, nullptr));
  // with an overlap: S r (kept for the whole call) and S^{-1} r (in p, by CG)
  double *Sr = nullptr, *SiR = nullptr;
  if (ctx->has_s) {
    Sr = base + 11 * plane;
    SiR = w.p;
    const double *hv = w.ca.hval, *sv = w.ca.sval;
    w.ca.hval = sv;  // the plain product with S
    w.ca.sval = nullptr;
    TRY(cspmm(ctx, w, w.x, w.s, 0.0, 0.0, nullptr));
    w.ca.hval = hv;
    w.ca.sval = sv;
    HIPCHK(rfo::launch_cx_scale(w.s, Sr, plane, 1.0, ctx->stream));
    TRY(cg_solve(ctx, pl, ctx->vec, w.x, SiR));
  }
  // m0 = r . r and h = (H r) . (S^{-1} r) per column
  HIPCHK(rfo::launch_cx_pdot(sgn, rden, nullptr, w.x, w.x, n, sp, nullptr, 0.0, 0.0, w.part, w.part2,
                             ctx->stream));
  HIPCHK(rfo::launch_colreduce(w.part, rfo::cg_nparts(n), sp, m01, ctx->stream));
  HIPCHK(rfo::launch_cx_pdot(sgn, rden, SiR, w.q, w.q, n, sp, nullptr, 0.0, 0.0, w.part, w.part2,
                             ctx->stream));
  HIPCHK(rfo::launch_colreduce(w.part, rfo::cg_nparts(n), sp, m01 + sp, ctx->stream));
  HIPCHK(rfo::launch_cx_scale(m01 + sp, m01 + sp, sp, c, ctx->stream));

  rfo::SddmmArgs sa;
  memset(&sa, 0, sizeof(sa));
  sa.brow = P<int64_t>(ctx->brow);
  sa.col = P<int32_t>(ctx->col);
  sa.nnzb = ctx->nnzb;
  sa.bd = ctx->bd;
  sa.sp = sp;
  sa.sgn = sgn;
  sa.rden = rden;
  sa.w = P<double>(ctx->w);
  sa.count = 1;
  sa.scale = 1.0;
  sa.rest = 1.0;
  sa.ppl = sddmm_ppl(ctx);
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  ctx->has_grad = ctx->has_dens = ctx->has_q = false;
  if (grad) {
    // the linear part of g: dF/dH = g1 sum_c w_c r_c r_c^T on the pattern
    TRY(ensure(ctx, ctx->G, gbytes));
    sa.xbase = w.x;
    sa.ybase = nullptr;
    sa.first = poly[2];
    sa.G = P<double>(ctx->G);
    sa.accumulate = 0;
    HIPCHK(rfo::launch_sddmm(0, sa, ctx->stream));
  }
  // P r starts at f0 S^{-1} r
  if (dens) {
    if (SiR) HIPCHK(rfo::launch_cx_scale(SiR, w.acc, plane, poly[0], ctx->stream));
    else HIPCHK(rfo::launch_cx_fill(sgn, rden, n, sp, poly[0], w.acc, nullptr, ctx->stream));
  }
  HIPCHK(rfo::launch_cx_fill(sgn, rden, n, sp, 0.0, w.x, w.x + plane, ctx->stream));  // x = 0

  // poles far from mu first, each solve warm-started from the previous solution
  std::vector<int64_t> order((size_t)n_poles);
  for (int64_t k = 0; k < n_poles; ++k) order[k] = k;
  std::stable_sort(order.begin(), order.end(), [&](int64_t a, int64_t b) {
    const double da = std::hypot(poles[2 * a] - mu, poles[2 * a + 1]);
    const double db = std::hypot(poles[2 * b] - mu, poles[2 * b + 1]);
    return da > db;
  });
  std::vector<int64_t> iters((size_t)n_poles, 0);
  for (size_t t = 0; t < order.size(); ++t) {
    const int64_t k = order[t];
    const double zr = (poles[2 * k] - d) / c, zi = poles[2 * k + 1] / c;
    TRY(cgls_solve(ctx, w, zr, zi, tol, max_iter, t == 0, &iters[k]));
    // rho_k = (S r) . x_k, and P r += 2 Re[(w_k / c) x_k]
    const double wr = 2.0 * res_f[2 * k] / c, wi = 2.0 * res_f[2 * k + 1] / c;
    HIPCHK(rfo::launch_cx_pdot(sgn, rden, Sr, w.x, w.x + plane, n, sp, dens ? w.acc : nullptr, wr, wi,
                               w.part, w.part2, ctx->stream));
    HIPCHK(rfo::launch_colreduce(w.part, rfo::cg_nparts(n), sp, rho + (size_t)2 * k * sp, ctx->stream));
    HIPCHK(rfo::launch_colreduce(w.part2, rfo::cg_nparts(n), sp, rho + (size_t)(2 * k + 1) * sp,
                                 ctx->stream));
    if (grad) {
      // -2 Re[(tau_k / c^2) x_a x_b] = -2 Re t (xr xr - xi xi) + 2 Im t (xr xi + xi xr)
      const double tr = res_g[2 * k] / (c * c), ti = res_g[2 * k + 1] / (c * c);
      sa.accumulate = 1;
      sa.sym = 0;
      sa.xbase = w.x;
      sa.ybase = w.x;
      sa.first = -2.0 * tr;
      HIPCHK(rfo::launch_sddmm(0, sa, ctx->stream));
      sa.xbase = w.x + plane;
      sa.ybase = w.x + plane;
      sa.first = 2.0 * tr;
      HIPCHK(rfo::launch_sddmm(0, sa, ctx->stream));
      sa.sym = 1;
      sa.xbase = w.x;
      sa.ybase = w.x + plane;
      sa.first = 2.0 * ti;
      HIPCHK(rfo::launch_sddmm(0, sa, ctx->stream));
      sa.sym = 0;
    }
  }
  rfo::RationalScalars ks;
  ks.f0 = poly[0];
  ks.ew = ew;
  ks.g0 = poly[1];
  ks.g1 = poly[2];
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_rational_traces(rho, m01, P<double>(ctx->w), P<double>(ctx->rat_coef),
                                     (int)n_poles, sp, ks, obs, ctx->stream));
  if (dens) {
    // with the gradient in G the density goes through the Q buffer
    DevBuf &db = grad ? ctx->GQ : ctx->G;
    TRY(ensure(ctx, db, gbytes));
    sa.accumulate = 0;
    sa.sym = 0;
    sa.xbase = w.acc;
    sa.ybase = nullptr;
    sa.first = 1.0;
    sa.G = P<double>(db);
    HIPCHK(rfo::launch_sddmm(0, sa, ctx->stream));
    TRY(copy_out(ctx, density_out, db.p, gbytes));
    ctx->has_dens = !grad;
    if (ctx->has_s) {
      // Q r = S^{-1} H P r: x = (P r, 0), q = H P r / c, then CG
      HIPCHK(rfo::launch_cx_scale(w.acc, w.x, plane, 1.0, ctx->stream));
      HIPCHK(hipMemsetAsync(w.x + plane, 0, (size_t)plane * sizeof(double), ctx->stream));
      TRY(cspmm(ctx, w, w.x, w.q, -d / c, 0.0, nullptr));
      HIPCHK(rfo::launch_cx_scale(w.q, w.r, plane, c, ctx->stream));
      TRY(cg_solve(ctx, pl, ctx->vec, w.r, w.p));
      TRY(ensure(ctx, ctx->GQ, gbytes));
      sa.xbase = w.p;
      sa.G = P<double>(ctx->GQ);
      HIPCHK(rfo::launch_sddmm(0, sa, ctx->stream));
      ctx->has_q = true;
    }
  }
  if (grad) {
    TRY(copy_out(ctx, dFdH_out, ctx->G.p, gbytes));
    ctx->has_grad = true;
  }
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (iterations_out) std::copy(iters.begin(), iters.end(), iterations_out);
  return RFO_OK;
}

int rfo_rational_stats(const rfo_ctx *ctx, int64_t *iterations, int64_t *solves) {
  if (!ctx || !iterations || !solves) return RFO_E_INVALID;
  *iterations = ctx->cgls_iters;
  *solves = ctx->cgls_solves;
  return RFO_OK;
}

int rfo_cg_stats(const rfo_ctx *ctx, int64_t *iterations, int64_t *solves) {
  if (!ctx || !iterations || !solves) return RFO_E_INVALID;
  *iterations = ctx->cg_iters;
  *solves = ctx->cg_solves;
  return RFO_OK;
}

int rfo_set_moment_doubling(rfo_ctx *ctx, int enabled) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  ctx->doubling = enabled != 0;
  return RFO_OK;
}

int rfo_set_timing(rfo_ctx *ctx, int enabled) {
  if (!ctx) return RFO_E_INVALID;
  ctx->timing = enabled != 0;
  ctx->t_ms = 0.0;
  ctx->t_steps = 0;
  return RFO_OK;
}

int rfo_step_timing(rfo_ctx *ctx, double *mean_ms, int64_t *n_steps) {
  if (!ctx || !mean_ms || !n_steps) return RFO_E_INVALID;
  *n_steps = ctx->t_steps;
  *mean_ms = ctx->t_steps > 0 ? ctx->t_ms / (double)ctx->t_steps : 0.0;
  return RFO_OK;
}

}  // extern "C"
