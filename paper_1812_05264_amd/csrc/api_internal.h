// Internal state and helpers shared by the C ABI translation units: the
// context, device buffers, the launch plan of the Chebyshev step, the forward
// recurrence and conjugate gradients for S^{-1}.  Not part of the ABI.
#pragma once

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

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

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
  bool grad_s = false;  // the gradient of the last rfo_energy_and_dEdH has dF/dS (in GQ)

  bool doubling = true;  // moment-only calls via T_2j, T_2j-1 identities
  // launch geometry and schedule (rfo_set_tuning); -1 = the measured default
  int64_t tune[RFO_TUNE_COUNT];
  mutable uint64_t sweeps = 0;  // step launches so far (direction of the alternating sweep)
  // nonorthogonal basis: overlap S on H's pattern, S^{-1} by conjugate gradients
  bool has_s = false, interval_given = false, has_q = false, has_dens = false;
  double cg_tol = 1e-13;
  DevBuf s64, cg_part, cg_sc, cg_spart, GQ;
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

  rfo_ctx() {
    for (int64_t &v : tune) v = -1;  // every key at its default
  }

  ~rfo_ctx() {
    hipSetDevice(device);
    DevBuf *all[] = {&row_ptr, &col, &brow, &tpos, &hraw, &h64, &h32, &hbf16, &gscratch, &nz_up, &nz_low,
                     &kc_ptr, &kc_idx, &kc_src, &up_grp,
                     &s64, &cg_part, &cg_sc, &cg_spart, &GQ, &rat, &rat_part, &rat_sc, &rat_rho, &rat_coef,
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

namespace rfo_api {

inline int fail(rfo_ctx *c, int code, const char *fmt, ...) {
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

inline int ensure(rfo_ctx *ctx, DevBuf &b, size_t bytes) {
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

inline void release(DevBuf &b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

// BF16 MFMA steps (H_hat in one BF16 part, or split into hi + lo)
inline bool is_bf16(int prec) { return prec == RFO_BF16 || prec == RFO_BF16X2; }

// a tuning value of the context, or def when it is at its default
inline int64_t tuned(const rfo_ctx *c, int key, int64_t def) {
  return c->tune[key] >= 0 ? c->tune[key] : def;
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

inline Plan make_plan(const rfo_ctx *c) {
  Plan pl;
  pl.vt_bytes = c->prec == RFO_FP64 ? 8 : 4;
  // 16 bytes per lane (FP64) or 16 (FP32, 9x9: 32 measured best) per gather
  int want = 16 / pl.vt_bytes;
  if (c->bd == 9 && c->prec != RFO_FP64) want = 4;
  want = (int)tuned(c, RFO_TUNE_PPL, want);
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
  rows = tuned(c, RFO_TUNE_ROWS_PER_WG, rows);
  pl.rows_per_wg = (int)rows;
  pl.n_rg = (int)((c->nb + rows - 1) / rows);
  pl.ring = 32;
  // 1x1 blocks: rows per wave iteration, or 7 when every row fits one chunk of 7
  // neighbours (measured faster on the 7-point lattice); 9x9: blocks per chunk
  pl.rpi = c->bd == 1 ? (c->max_row <= 7 ? 7 : 1) : 2;
  {
    const int r = (int)tuned(c, RFO_TUNE_RPI, pl.rpi);
    if (r == 1 || r == 2 || (c->bd == 1 && r == 7)) pl.rpi = r;
  }
  pl.n_pt_step = pl.n_pt;
  pl.ntiles = 0;
  int occ = 1;
  if (is_bf16(c->prec)) {
    // 4 MFMA column tiles (64 probes) per wave, one K chunk of 32 rows per
    // iteration: measured best (wider tiles or more chunks cost more registers
    // than the loads they add in flight)
    pl.ntiles = 4;
    pl.rpi = 1;
    pl.n_pt_step = c->sp / (16 * pl.ntiles);
    pl.rpi = (int)tuned(c, RFO_TUNE_BF16_CHUNKS, pl.rpi);
    occ = std::max(1, rfo::step_bf16_blocks_per_cu(pl.ntiles, pl.rpi, c->prec == RFO_BF16X2 ? 1 : 0));
  } else {
    occ = std::max(1, rfo::step_blocks_per_cu(c->bd, c->prec == RFO_FP64 ? 0 : 1, pl.ppl, pl.rpi));
  }
  // one resident wave of workgroups, a multiple of 8 (one share per XCD), at
  // most four per CU: more workgroups widen the band of rows in flight on an XCD
  // past what its L2 holds of their neighbour rows (measured slower)
  int64_t grid = (int64_t)c->cus * std::min(occ, 4);
  grid = tuned(c, RFO_TUNE_GRID, grid);
  const int64_t units = (int64_t)pl.n_pt_step * pl.n_rg;
  grid = std::min(grid, (units + 7) / 8 * 8);
  grid = std::max<int64_t>(8, grid / 8 * 8);
  pl.grid = (int)grid;
  pl.vec_elems = (size_t)c->n * (size_t)c->sp;
  pl.slot_bytes = pl.vec_elems * (pl.vt_bytes + (is_bf16(c->prec) ? 2 : 0));
  return pl;
}

inline void fill_step(rfo_ctx *c, const Plan &pl, rfo::StepArgs &a) {
  memset(&a, 0, sizeof(a));
  a.row_ptr = P<int64_t>(c->row_ptr);
  a.col = P<int32_t>(c->col);
  a.hval = c->prec == RFO_FP64 ? c->h64.p : (c->prec == RFO_FP32 ? c->h32.p : c->hbf16.p);
  if (is_bf16(c->prec)) {
    a.kc_ptr = P<int64_t>(c->kc_ptr);
    a.kc_idx = P<int32_t>(c->kc_idx);
    a.hsplit = c->prec == RFO_BF16X2 ? 1 : 0;
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
  // dense probes carry zero padding columns, and so does every vector made from them
  a.s_live = c->signs ? c->sp : (int)c->s;
}

inline void fill_init(rfo_ctx *c, const Plan &pl, rfo::InitArgs &a) {
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

inline int kernel_precision(const rfo_ctx *c) { return c->prec == RFO_FP64 ? 0 : 1; }

// The segment gradient of the BF16 steps runs on the matrix cores when every real
// probe has the same weight (the weight is applied in FP64 after each step's
// contraction).  FP32 steps keep the VALU contraction: an FP32-MFMA version
// measured no faster at full size and sums in FP32.
inline bool use_mfma_sddmm(const rfo_ctx *c) {
  if (c->bd != 9 || !is_bf16(c->prec) || c->w_uniform == 0.0 || !c->has_up_grp) return false;
  if (c->sp % 32 != 0) return false;
  return tuned(c, RFO_TUNE_SDDMM_MFMA, 1) != 0;
}

// The segment gradient in launches of at most 32 steps each (8 for the BF16
// kernel; RFO_TUNE_SDDMM_STEPS, RFO_TUNE_SDDMM_STEPS_BF16): all resident waves then work on the same few steps, so the
// rows of X_t and Y_t that the blocks of a band of block rows share are read
// while the L2 holds them.  Measured on the 16,000-atom cluster at 8000 terms
// (segments of 64 steps).
inline hipError_t launch_sddmm_segment(const rfo_ctx *c, int precision, const rfo::SddmmArgs &a,
                                       size_t slot_bytes, hipStream_t s) {
  const int tg = (int)tuned(c, RFO_TUNE_SDDMM_STEPS, 32);
  if (tg <= 0 || a.count <= tg) return rfo::launch_sddmm(precision, a, s);
  rfo::SddmmArgs b = a;
  for (int t0 = 0; t0 < a.count; t0 += tg) {
    b.xbase = static_cast<const char *>(a.xbase) + (size_t)t0 * slot_bytes;
    b.ybase = static_cast<const char *>(a.ybase) + (size_t)t0 * slot_bytes;
    b.count = std::min(tg, a.count - t0);
    b.j0 = a.j0 + t0;
    b.accumulate = t0 == 0 ? a.accumulate : 1;
    const hipError_t e = rfo::launch_sddmm(precision, b, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

inline hipError_t launch_sddmm_bf16_segment(const rfo_ctx *c, const rfo::SddmmMfmaArgs &a,
                                            size_t slot_bytes, hipStream_t s) {
  const int tg = (int)tuned(c, RFO_TUNE_SDDMM_STEPS_BF16, 8);
  if (tg <= 0 || a.count <= tg) return rfo::launch_sddmm_bf16(a, s);
  rfo::SddmmMfmaArgs b = a;
  for (int t0 = 0; t0 < a.count; t0 += tg) {
    b.xbase = static_cast<const char *>(a.xbase) + (size_t)t0 * slot_bytes;
    b.ybase = static_cast<const char *>(a.ybase) + (size_t)t0 * slot_bytes;
    b.count = std::min(tg, a.count - t0);
    b.j0 = a.j0 + t0;
    b.accumulate = t0 == 0 ? a.accumulate : 1;
    const hipError_t e = rfo::launch_sddmm_bf16(b, s);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

inline int sddmm_ppl(const rfo_ctx *c) {
  const int64_t want = tuned(c, RFO_TUNE_SDDMM_PPL, 2);
  return (want == 2 && c->sp % 128 == 0) ? 2 : 1;
}

inline hipError_t launch_any_step(const rfo_ctx *c, const Plan &pl, const rfo::StepArgs &a) {
  // three accumulator terms need y_{k-1}, which the first pass does not have
  if (a.acc_terms < 0 || a.acc_terms > 3 || (a.acc_terms == 3 && a.c2 == 0.0))
    return hipErrorInvalidValue;
  rfo::StepArgs b = a;
  // alternating sweeps: every other launch runs each XCD's range backwards
  b.reverse = tuned(c, RFO_TUNE_ALT_SWEEP, 1) != 0 ? (int)(c->sweeps++ & 1) : 0;
  if (is_bf16(c->prec)) {
    // x and out are vector slots; their BF16 copies follow the FP32 vectors
    b.xb = static_cast<const char *>(a.x) + pl.vec_elems * sizeof(float);
    b.outb = static_cast<char *>(a.out) + pl.vec_elems * sizeof(float);
    return rfo::launch_step_bf16(pl.ntiles, b, c->stream);
  }
  return rfo::launch_step(c->bd, kernel_precision(c), pl.ppl, b, c->stream);
}

// y = scale r into a vector slot (and its BF16 copy in BF16 mode)
inline hipError_t launch_init_slot(const rfo_ctx *c, const Plan &pl, rfo::InitArgs &a) {
  a.outb = is_bf16(c->prec) ? static_cast<char *>(a.out) + pl.vec_elems * sizeof(float) : nullptr;
  return rfo::launch_init(kernel_precision(c), a, c->stream);
}

inline char *vec_at(rfo_ctx *c, const Plan &pl, DevBuf &b, int64_t i) {
  return static_cast<char *>(b.p) + (size_t)i * pl.slot_bytes;
}

inline hipEvent_t next_event(rfo_ctx *c, size_t idx) {
  while (c->events.size() <= idx) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    c->events.push_back(e);
  }
  return c->events[idx];
}

inline int copy_out(rfo_ctx *ctx, void *dst, const void *src, size_t bytes) {
  if (!dst || bytes == 0) return RFO_OK;
  HIPCHK(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, ctx->stream));
  return RFO_OK;
}

inline int check_flags_and_finish(rfo_ctx *ctx, size_t n_events) {
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
  // optional tail store: the forward pass writes y_j for j >= tail_j0 into
  // consecutive vector slots from `tail` instead of its two working slots
  char *tail = nullptr;
  int64_t tail_j0 = 0;
};

inline int ensure_cg(rfo_ctx *ctx) {
  TRY(ensure(ctx, ctx->cg_part, (size_t)rfo::cg_nparts(ctx->n) * ctx->sp * sizeof(double)));
  TRY(ensure(ctx, ctx->cg_sc, ((size_t)6 * ctx->sp + 1) * sizeof(double)));
  if (!ctx->cg_res_h) HIPCHK(hipHostMalloc((void **)&ctx->cg_res_h, sizeof(double), 0));
  return RFO_OK;
}

// t = S^{-1} y for every probe column by conjugate gradients (S symmetric positive
// definite), to |r_c| <= cg_tol |y_c|.  Work vectors: slots 3..5 of bufs.
inline int cg_solve(rfo_ctx *ctx, const Plan &pl, DevBuf &bufs, const void *y, void *t) {
  const int64_t n = ctx->n;
  const int sp = ctx->sp;
  // the kernels below write these buffers: never launch them unallocated or too small
  if (!ctx->cg_res_h || ctx->cg_part.bytes < (size_t)rfo::cg_nparts(n) * sp * sizeof(double) ||
      ctx->cg_sc.bytes < ((size_t)6 * sp + 1) * sizeof(double) || bufs.bytes < 6 * pl.slot_bytes)
    return fail(ctx, RFO_E_STATE, "internal: conjugate-gradient buffers not allocated");
  double *r = reinterpret_cast<double *>(vec_at(ctx, pl, bufs, 3));
  double *pv = reinterpret_cast<double *>(vec_at(ctx, pl, bufs, 4));
  double *q = reinterpret_cast<double *>(vec_at(ctx, pl, bufs, 5));
  double *part = P<double>(ctx->cg_part), *sc = P<double>(ctx->cg_sc);
  double *res_d = sc + 6 * sp;
  // the product's column partials of p . q (the step kernel's moment partials with p
  // as the probe block): one pass over p and q fewer per iteration
  TRY(ensure(ctx, ctx->cg_spart, (size_t)pl.grid * sp * sizeof(double)));
  double *spart = P<double>(ctx->cg_spart);
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
  sa.sgn = nullptr;
  sa.rden = pv;
  sa.part = spart;
  const double tol2 = ctx->cg_tol * ctx->cg_tol;
  const int max_it = 2000;
  for (int it = 1; it <= max_it; ++it) {
    HIPCHK(launch_any_step(ctx, pl, sa));
    HIPCHK(rfo::launch_cg_alpha(spart, pl.grid, sp, sc, res_d, ctx->stream));
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

inline int run_forward(rfo_ctx *ctx, const Plan &pl, int64_t p, DevBuf &bufs, bool use_acc,
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
  char *tail = ck ? ck->tail : nullptr;
  const int64_t tail_j0 = ck ? ck->tail_j0 : 0;
  auto tail_at = [&](int64_t j) { return tail + (size_t)(j - tail_j0) * pl.slot_bytes; };
  if (tail && tail_j0 == 0) A = tail_at(0);

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
    char *out = (tail && k + 1 >= tail_j0) ? tail_at(k + 1) : (k == 0) ? B : prev;
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

// argument and state checks shared by the calls that run the recurrence
inline int validate_call(rfo_ctx *ctx, double T, double mu, int64_t p) {
  if (!ctx) return RFO_E_INVALID;
  if (!ctx->has_h) return fail(ctx, RFO_E_STATE, "no Hamiltonian: call rfo_set_hamiltonian first");
  if (!ctx->has_r) return fail(ctx, RFO_E_STATE, "no probes: call rfo_set_probes first");
  if (!(T > 0.0) || !std::isfinite(T)) return fail(ctx, RFO_E_INVALID, "T must be finite and > 0");
  if (!std::isfinite(mu)) return fail(ctx, RFO_E_INVALID, "mu must be finite");
  if (p < 1 || p > (1 << 20)) return fail(ctx, RFO_E_INVALID, "n_terms must be in [1, 2^20]");
  HIPCHK(hipSetDevice(ctx->device));
  ctx->sweeps = 0;  // every call starts forward: repeated calls sum in the same order
  ctx->mom_p = 0;   // the stored moments are overwritten: valid again only when the call succeeds
  return RFO_OK;
}

inline int prepare_call(rfo_ctx *ctx, double T, double mu, int64_t p, Plan &pl) {
  TRY(validate_call(ctx, T, mu, p));
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

// Padded width of a probe block of s_real probes (the rule of rfo_set_probes).
inline int padded_probes(int64_t s_real) { return s_real <= 64 ? 64 : (int)((s_real + 127) / 128 * 128); }

// Probe batches: select() swaps the context's probe block for its columns [c0, c0 + s_b)
// (c0 a multiple of 64: whole sign words, or dense columns, copied into batch buffers,
// with their weights); the whole block comes back with restore() and when this object
// goes out of scope.
struct ProbeBatches {
  rfo_ctx *ctx;
  DevBuf sgn, rden, w;  // the whole block (the context's buffers)
  int64_t s;
  int sp;
  double w_uniform;
  DevBuf bsgn, brden, bw;  // the selected batch
  std::vector<double> w_h;
  explicit ProbeBatches(rfo_ctx *c)
      : ctx(c), sgn(c->sgn), rden(c->rden), w(c->w), s(c->s), sp(c->sp), w_uniform(c->w_uniform) {}
  ProbeBatches(const ProbeBatches &) = delete;
  ProbeBatches &operator=(const ProbeBatches &) = delete;
  int select(int64_t c0, int64_t s_b) {
    if (w_h.empty()) {
      w_h.resize((size_t)sp);
      HIPCHK(hipMemcpy(w_h.data(), w.p, w_h.size() * sizeof(double), hipMemcpyDeviceToHost));
    }
    const int sp_b = padded_probes(s_b);
    const size_t n = (size_t)ctx->n;
    TRY(ensure(ctx, bw, (size_t)sp_b * sizeof(double)));
    std::vector<double> wb((size_t)sp_b, 0.0);
    for (int64_t c = 0; c < s_b; ++c) wb[(size_t)c] = w_h[(size_t)(c0 + c)];
    HIPCHK(hipMemcpy(bw.p, wb.data(), wb.size() * sizeof(double), hipMemcpyHostToDevice));
    if (sgn.p && !rden.p) {
      TRY(ensure(ctx, bsgn, n * (sp_b / 64) * sizeof(uint64_t)));
      HIPCHK(hipMemsetAsync(bsgn.p, 0, n * (sp_b / 64) * sizeof(uint64_t), ctx->stream));
      const size_t words = (size_t)(s_b + 63) / 64;
      HIPCHK(hipMemcpy2DAsync(bsgn.p, (sp_b / 64) * sizeof(uint64_t), P<uint64_t>(sgn) + c0 / 64,
                              (sp / 64) * sizeof(uint64_t), words * sizeof(uint64_t), n,
                              hipMemcpyDeviceToDevice, ctx->stream));
      ctx->sgn = bsgn;
      ctx->rden = DevBuf{};
    } else {
      TRY(ensure(ctx, brden, n * sp_b * sizeof(double)));
      HIPCHK(hipMemsetAsync(brden.p, 0, n * sp_b * sizeof(double), ctx->stream));
      HIPCHK(hipMemcpy2DAsync(brden.p, sp_b * sizeof(double), P<double>(rden) + c0, sp * sizeof(double),
                              s_b * sizeof(double), n, hipMemcpyDeviceToDevice, ctx->stream));
      ctx->rden = brden;
      ctx->sgn = DevBuf{};
    }
    ctx->w = bw;
    ctx->s = s_b;
    ctx->sp = sp_b;
    ctx->w_uniform = wb[0];
    for (int64_t c = 1; c < s_b; ++c)
      if (wb[(size_t)c] != wb[0]) ctx->w_uniform = 0.0;
    return RFO_OK;
  }
  void restore() {
    ctx->sgn = sgn;
    ctx->rden = rden;
    ctx->w = w;
    ctx->s = s;
    ctx->sp = sp;
    ctx->w_uniform = w_uniform;
  }
  ~ProbeBatches() {
    for (DevBuf *b : {&bsgn, &brden, &bw}) release(*b);
    restore();
  }
};

// A last VALU probe tile of 128 columns that holds at most 64 real probes runs as a
// batch of its own, 64 columns wide (a tile costs about the same whatever part of
// it is live): the batches [0, s - r), [s - r, s), or none.
inline std::vector<std::pair<int64_t, int64_t>> last_tile_batches(const rfo_ctx *c) {
  if (c->has_s || is_bf16(c->prec) || c->s <= 128 || c->s % 128 == 0 || c->s % 128 > 64) return {};
  const int64_t r = c->s % 128;
  return {{0, c->s - r}, {c->s - r, r}};
}

inline int copy_moments_out(rfo_ctx *ctx, int64_t p, double *moments_out) {
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
}  // namespace rfo_api

