// C ABI: free energy and its gradient dF/dH by the reverse (Clenshaw) recurrence,
// direct or through the doubled moments, and the Hellmann-Feynman forces.
#include "api_internal.h"

using namespace rfo_api;

namespace {

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
  // between two sets of y and z slots.  Measured on cu16k with the gradient kernels in
  // step-group launches: FP64 10.05 against 9.29 s, FP32 5.63 against 5.46 s, BF16
  // 4.04 against 3.96 s (the persistent step kernels lose the CUs the gradient holds),
  // so the serial schedule is the default and the overlap is taken on request.
  const bool overlap = Q > 1 && tuned(ctx, RFO_TUNE_OVERLAP, 0) != 0;
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
      HIPCHK(launch_sddmm_bf16_segment(ctx, sm, pl.slot_bytes, sd_stream));
    } else {
      HIPCHK(launch_sddmm_segment(ctx, kp, sd, pl.slot_bytes, sd_stream));
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
      HIPCHK(launch_sddmm_segment(ctx, kp, a, pl.slot_bytes, ctx->stream));
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

}  // extern "C"
