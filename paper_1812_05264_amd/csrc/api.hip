// C ABI of the randomized Fermi-operator library: the context, the Hamiltonian
// and probes, the Chebyshev moments, traces and density (see include/rfo.h for
// the contract).
#include "api_internal.h"

using namespace rfo_api;

namespace {

// per host thread, so concurrent rfo_create calls do not overwrite each other's message
thread_local std::string g_create_error;

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
  if (precision != RFO_FP64 && precision != RFO_FP32 && !is_bf16(precision))
    return fail(ctx, RFO_E_INVALID, "unknown precision %d", precision);
  if (is_bf16(precision) && block_dim != 9)
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
  if (is_bf16(precision)) {
    // K chunks: block row I's blocks concatenated along K (9 rows each), cut into
    // chunks of kKChunk K rows; K row k of the row is column c = k % 9 of block
    // nz = row_ptr[I] + k / 9
    const std::vector<int64_t> &rp = ctx->row_ptr_h;
    const std::vector<int32_t> &cl = ctx->col_h;
    if ((int64_t)ctx->nnzb * 9 >= ((int64_t)1 << 31) || ctx->n >= ((int64_t)1 << 31))
      return fail(ctx, RFO_E_UNSUPPORTED, "BF16 steps index rows with 32 bits");
    std::vector<int64_t> kp((size_t)ctx->nb + 1, 0);
    constexpr int KC = rfo::kKChunk;
    for (int64_t I = 0; I < ctx->nb; ++I) kp[I + 1] = kp[I] + (9 * (rp[I + 1] - rp[I]) + KC - 1) / KC;
    const int64_t nch = kp[ctx->nb];
    std::vector<int32_t> kidx((size_t)nch * KC, -1), ksrc((size_t)nch * KC, -1);
    for (int64_t I = 0; I < ctx->nb; ++I)
      for (int64_t k = 0; k < 9 * (rp[I + 1] - rp[I]); ++k) {
        const int64_t nz = rp[I] + k / 9, c = k % 9;
        kidx[(size_t)(kp[I] * KC + k)] = (int32_t)((int64_t)cl[nz] * 9 + c);
        ksrc[(size_t)(kp[I] * KC + k)] = (int32_t)(nz * 9 + c);
      }
    ctx->n_chunks = nch;
    const size_t nq = (size_t)std::max<int64_t>(nch, 1);
    TRY(ensure(ctx, ctx->kc_ptr, kp.size() * sizeof(int64_t)));
    TRY(ensure(ctx, ctx->kc_idx, nq * KC * sizeof(int32_t)));
    TRY(ensure(ctx, ctx->kc_src, nq * KC * sizeof(int32_t)));
    // 36 entries of eight BF16 values per chunk (twice that with the low parts)
    TRY(ensure(ctx, ctx->hbf16, nq * 36 * (precision == RFO_BF16X2 ? 32 : 16)));
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
  if (is_bf16(precision))
    HIPCHK(rfo::launch_pack_bf16(P<double>(ctx->h64), P<int32_t>(ctx->kc_src), ctx->n_chunks,
                                 precision == RFO_BF16X2 ? 1 : 0, ctx->hbf16.p, ctx->stream));
  HIPCHK(hipMemcpyAsync(ctx->flags_h, ctx->flags.p, sizeof(int), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  if (*ctx->flags_h & 1) return fail(ctx, RFO_E_NUMERIC, "non-finite Hamiltonian values");
  if (*ctx->flags_h & 2) return fail(ctx, RFO_E_INVALID, "Hamiltonian values are not symmetric (H_JI != H_IJ^T)");
  ctx->has_up_grp = false;
  if (block_dim == 9 && is_bf16(precision)) {
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

namespace {

// Density blocks D (+)= sum_c w_c x_c r_c^T on H's pattern from the vectors x in
// xbase (the density accumulator, or P r with an overlap) and the context's probes.
int density_sddmm(rfo_ctx *ctx, const void *xbase, double *G, int accumulate) {
  rfo::SddmmArgs a;
  memset(&a, 0, sizeof(a));
  a.brow = P<int64_t>(ctx->brow);
  a.col = P<int32_t>(ctx->col);
  a.nnzb = ctx->nnzb;
  a.bd = ctx->bd;
  a.sp = ctx->sp;
  a.xbase = xbase;
  a.ybase = nullptr;
  a.sgn = ctx->signs ? P<uint64_t>(ctx->sgn) : nullptr;
  a.rden = ctx->signs ? nullptr : P<double>(ctx->rden);
  a.w = P<double>(ctx->w);
  a.count = 1;
  a.scale = 1.0;
  a.first = 1.0;
  a.rest = 1.0;
  a.G = G;
  a.accumulate = accumulate;
  a.nzlist = nullptr;
  a.ppl = sddmm_ppl(ctx);
  a.s_live = (int)ctx->s;
  HIPCHK(rfo::launch_sddmm(kernel_precision(ctx), a, ctx->stream));
  return RFO_OK;
}

// rfo_fermi_moments over probe batches: the moments of every batch gathered into
// the whole block's [p][sp] moments, the density blocks summed over the batches in
// batch order.  (No overlap: last_tile_batches takes none with one.)
int fermi_moments_batches(rfo_ctx *ctx, int64_t p, const std::vector<std::pair<int64_t, int64_t>> &batches,
                          double *moments_out, double *NEF_out, double *density_out) {
  const bool dens = density_out != nullptr;
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  if (dens) TRY(ensure(ctx, ctx->G, gbytes));
  ProbeBatches pb(ctx);
  DevBuf mom_all;
  struct Release {
    DevBuf &b;
    ~Release() { release(b); }
  } release_mom{mom_all};
  TRY(ensure(ctx, mom_all, (size_t)p * pb.sp * sizeof(double)));
  HIPCHK(hipMemsetAsync(mom_all.p, 0, (size_t)p * pb.sp * sizeof(double), ctx->stream));
  bool first = true;
  for (const auto &bt : batches) {
    const int64_t c0 = bt.first, s_b = bt.second;
    TRY(pb.select(c0, s_b));
    const Plan bpl = make_plan(ctx);
    TRY(ensure(ctx, ctx->ring, (size_t)bpl.ring * bpl.grid * ctx->sp * sizeof(double)));
    TRY(ensure(ctx, ctx->vec, 2 * bpl.slot_bytes));
    if (dens) TRY(ensure(ctx, ctx->acc, bpl.vec_elems * bpl.vt_bytes));
    size_t n_events = 0;
    TRY(run_forward(ctx, bpl, p, ctx->vec, dens, nullptr, &n_events, !dens && ctx->doubling));
    HIPCHK(hipMemcpy2DAsync(P<double>(mom_all) + c0, pb.sp * sizeof(double), ctx->moments.p,
                            ctx->sp * sizeof(double), s_b * sizeof(double), p, hipMemcpyDeviceToDevice,
                            ctx->stream));
    if (dens) TRY(density_sddmm(ctx, ctx->acc.p, P<double>(ctx->G), first ? 0 : 1));
    TRY(check_flags_and_finish(ctx, n_events));
    first = false;
  }
  pb.restore();
  std::swap(ctx->moments, mom_all);
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                            ctx->sp, obs, ctx->stream));
  ctx->has_q = false;
  ctx->has_dens = dens;
  if (dens) {
    ctx->has_grad = false;  // G now holds the density
    TRY(copy_out(ctx, density_out, ctx->G.p, gbytes));
  }
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  TRY(copy_moments_out(ctx, p, moments_out));
  ctx->mom_p = p;
  return RFO_OK;
}

}  // namespace

int rfo_fermi_moments(rfo_ctx *ctx, double T, double mu, int64_t n_terms, double *moments_out,
                      double *NEF_out, double *density_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  Plan pl;
  TRY(prepare_call(ctx, T, mu, n_terms, pl));
  // a last probe tile of 128 columns with at most 64 real probes runs as a batch
  // of its own, 64 columns wide
  const auto batches = last_tile_batches(ctx);
  if (!batches.empty()) return fermi_moments_batches(ctx, n_terms, batches, moments_out, NEF_out, density_out);
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
    TRY(density_sddmm(ctx, px, P<double>(ctx->G), 0));
    if (qx) {
      TRY(density_sddmm(ctx, qx, P<double>(ctx->GQ), 0));
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

int rfo_set_tuning(rfo_ctx *ctx, int key, int64_t value) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (key < 0 || key >= RFO_TUNE_COUNT) return fail(ctx, RFO_E_INVALID, "unknown tuning key %d", key);
  bool ok = value == -1;
  switch (key) {
    case RFO_TUNE_PPL: ok = ok || value == 1 || value == 2 || value == 4; break;
    case RFO_TUNE_RPI: ok = ok || value == 1 || value == 2 || value == 7; break;
    case RFO_TUNE_ROWS_PER_WG: ok = ok || (value >= 1 && value <= 4096); break;
    case RFO_TUNE_GRID: ok = ok || (value >= 8 && value <= (1 << 20)); break;
    case RFO_TUNE_BF16_CHUNKS: ok = ok || value == 1 || value == 2; break;
    case RFO_TUNE_SDDMM_PPL: ok = ok || value == 1 || value == 2; break;
    case RFO_TUNE_SDDMM_MFMA: ok = ok || value == 0 || value == 1; break;
    case RFO_TUNE_SDDMM_STEPS: ok = ok || (value >= 0 && value <= (1 << 20)); break;
    case RFO_TUNE_SDDMM_STEPS_BF16: ok = ok || (value >= 0 && value <= (1 << 20)); break;
    case RFO_TUNE_OVERLAP: ok = ok || value == 0 || value == 1; break;
    case RFO_TUNE_CPLX_PPL: ok = ok || value == 1 || value == 2; break;
    case RFO_TUNE_CPLX_ROWS: ok = ok || value == 1 || value == 2 || value == 4 || value == 8; break;
    case RFO_TUNE_CPLX_GRID: ok = ok || (value >= 8 && value <= (1 << 20)); break;
    case RFO_TUNE_ADJOINT_BYTES: ok = ok || value >= 0; break;
    case RFO_TUNE_ALT_SWEEP: ok = ok || value == 0 || value == 1; break;
    case RFO_TUNE_ADJOINT_TAIL: ok = ok || value == 0 || value == 1; break;
    default: break;
  }
  if (!ok) return fail(ctx, RFO_E_INVALID, "tuning value %lld out of range for key %d", (long long)value, key);
  ctx->tune[key] = key == RFO_TUNE_GRID || key == RFO_TUNE_CPLX_GRID ? (value < 0 ? -1 : value / 8 * 8) : value;
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
