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
// tail_bytes: memory the call may add for a tail store (Checkpoints::tail): the last
// vectors of the forward pass stay in place, so the top segments are not replayed.
int energy_grad_doubling(rfo_ctx *ctx, const Plan &pl, int64_t p, bool g_acc, size_t *n_events_out,
                         size_t tail_bytes) {
  const int kp = kernel_precision(ctx);
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
  // vector slots: n_sets x (ys [m + 2] | zs [m + 2]) | checkpoints [2 (Q - 1)] | tail
  const int64_t n_ys = m + 2, n_zs = m + 2, n_ck = Q > 1 ? 2 * (Q - 1) : 0;
  const int64_t set_slots = n_ys + n_zs;
  // tail store: segments q >= q_s keep y_j, j in [q_s m, K], from the forward pass
  int64_t q_s = Q;
  if (!overlap && tail_bytes > 0) {
    const int64_t fit = (int64_t)(tail_bytes / pl.slot_bytes);
    while (q_s > 0 && K + 1 - (q_s - 1) * m <= fit) --q_s;
  }
  const int64_t tail_j0 = q_s * m, n_tail = q_s < Q ? K + 1 - tail_j0 : 0;
  TRY(ensure(ctx, ctx->vec, (size_t)(n_sets * set_slots + n_ck + n_tail) * pl.slot_bytes));
  char *tail = n_tail > 0 ? vec_at(ctx, pl, ctx->vec, n_sets * set_slots + n_ck) : nullptr;
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
  ck.tail = tail;
  ck.tail_j0 = tail_j0;
  TRY(run_forward(ctx, pl, p, ctx->vec, false, &ck, n_events_out, true));
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
  int64_t cur_j0 = 0;
  bool cur_stored = false;  // the segment's y_j are in the tail store
  auto ys = [&](int64_t t) {
    return cur_stored ? tail + (size_t)(cur_j0 + t - tail_j0) * pl.slot_bytes
                      : vec_at(ctx, pl, ctx->vec, cur * set_slots + t);
  };
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
    cur_j0 = j0;
    cur_stored = q >= q_s;
    if (sd_pending[cur]) {
      // the gradient of segment q + 2 read this set: wait before rewriting it
      HIPCHK(hipStreamWaitEvent(ctx->stream, ctx->ev_sd[cur], 0));
      sd_pending[cur] = false;
    }
    // replay y_j, j in [j0, min(j1 + 2, K + 1)), into ys[0 ..): the sources of
    // z_{j1} and z_{j1-1} need y_{j1} and y_{j1+1}
    const int64_t rlen = cur_stored ? 0 : std::min(j1 + 2, K + 1) - j0;
    if (cur_stored) {
      // kept by the forward pass
    } else if (q == 0) {
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
    sd.accumulate = (q == Q - 1 && !g_acc) ? 0 : 1;
    sd.nzlist = P<int64_t>(ctx->nz_up);
    sd.nlist = ctx->n_up;
    sd.ppl = sddmm_ppl(ctx);
    sd.s_live = (int)ctx->s;
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
  return RFO_OK;
}

// Free energy and gradient by the direct reverse recurrence of r . y_k over p - 1
// steps: z_{p-1} = beta_{p-1} r, z_{p-2} = 2 H_hat z_{p-1} + beta_{p-2} r,
// z_i = 2 H_hat z_{i+1} - z_{i+2} + beta_i r, dF~/dH_hat = sum_j c_j z_{j+1} y_j^T
// (c_0 = 1, c_j = 2) on the blocks on and above the diagonal.
int energy_grad_direct(rfo_ctx *ctx, const Plan &pl, int64_t p, bool g_acc, size_t *n_events_out) {
  const int kp = kernel_precision(ctx);
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
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
  TRY(run_forward(ctx, pl, p, ctx->vec, false, &ck, n_events_out));

  if (P1 == 0) {
    if (!g_acc) HIPCHK(hipMemsetAsync(ctx->G.p, 0, gbytes, ctx->stream));
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
      a.accumulate = (q == Q - 1 && !g_acc) ? 0 : 1;
      // the full gradient is symmetric: blocks on and above the diagonal only
      a.nzlist = P<int64_t>(ctx->nz_up);
      a.nlist = ctx->n_up;
      a.ppl = sddmm_ppl(ctx);
      a.s_live = (int)ctx->s;
      HIPCHK(launch_sddmm_segment(ctx, kp, a, pl.slot_bytes, ctx->stream));
      if (q > 0) {
        // carries for the segment below: zs[m] = z_{j0+1}, zs[m+1] = z_{j0+2}
        HIPCHK(hipMemcpyAsync(zs(m), zs(0), vb, hipMemcpyDeviceToDevice, ctx->stream));
        HIPCHK(hipMemcpyAsync(zs(m + 1), zs(1), vb, hipMemcpyDeviceToDevice, ctx->stream));
      }
    }
  }
  return RFO_OK;
}

// Free energy and gradient with an overlap S, by the direct recurrence (paper: Analytical
// free-energy derivatives, Eq. polynomial_response; Polynomial approximation with S).
// A = H_hat S^{-1}; the forward pass forms y_{k+1} = 2 H_hat t_k - y_{k-1}, t_k = S^{-1} y_k.
// The reverse recurrence of the direct form runs with A^T = S^{-1} H_hat and is carried as
// v_i = S z_i:
//   v_{p-1} = beta_{p-1} S r,  v_i = 2 H_hat z_{i+1} - v_{i+2} + beta_i S r,  z_i = S^{-1} v_i,
// so a reverse step is one step kernel and one conjugate-gradient solve, like a forward
// step.  With c_0 = 1, c_j = 2, kappa = (e_max + e_min)/(e_max - e_min) and
// A^T z_{j+1} = (z_j + z_{j+2} - beta_j r)/2 (the reverse recurrence itself; z_p = 0),
//   dF/dH = 2/(e_max - e_min) sum_j c_j z_{j+1} t_j^T,
//   dF/dS = -sum_j c_j (kappa z_{j+1} + A^T z_{j+1}) t_j^T,
// both as their symmetric parts (A is not symmetric, and symmetric variations of H and S
// see only that part), summed on the blocks on and above the diagonal and mirrored.
// Memory: the sqrt(p) checkpoints of the direct form, and per segment t_j, z_j and the
// dF/dS left factors.
int energy_grad_overlap(rfo_ctx *ctx, const Plan &pl, int64_t p, size_t *n_events_out) {
  const int kp = kernel_precision(ctx);
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  const int64_t P1 = p - 1;
  int64_t m = 2;
  while (m * m < P1) ++m;
  const int64_t Q = P1 > 0 ? (P1 + m - 1) / m : 0;
  // slots: 0, 1 y pair | 2 t of the forward pass | 3..5 CG work | 6 S r | 7, 8 v pair |
  //        ts [m] | zs [m + 2] | xs [m] | checkpoints [2 (Q - 1)]
  const int64_t o_sr = 6, o_v = 7, o_ts = 9, o_zs = o_ts + m, o_xs = o_zs + m + 2, o_ck = o_xs + m;
  const int64_t n_ck = Q > 1 ? 2 * (Q - 1) : 0;
  TRY(ensure(ctx, ctx->vec, (size_t)(o_ck + n_ck) * pl.slot_bytes));
  TRY(ensure(ctx, ctx->GQ, gbytes));
  TRY(ensure_cg(ctx));  // the solves' column partials and scalars
  auto slot = [&](int64_t i) { return vec_at(ctx, pl, ctx->vec, i); };
  DevBuf ckview;
  ckview.p = slot(o_ck);
  ckview.bytes = (size_t)n_ck * pl.slot_bytes;
  Checkpoints ck;
  ck.m = m;
  ck.Q = Q;
  ck.store = &ckview;
  TRY(run_forward(ctx, pl, p, ctx->vec, false, &ck, n_events_out));
  if (P1 == 0) {
    HIPCHK(hipMemsetAsync(ctx->G.p, 0, gbytes, ctx->stream));
    HIPCHK(hipMemsetAsync(ctx->GQ.p, 0, gbytes, ctx->stream));
    return RFO_OK;
  }
  std::vector<double> beta((size_t)p);
  HIPCHK(hipMemcpyAsync(beta.data(), P<double>(ctx->coef) + 2 * p, p * sizeof(double),
                        hipMemcpyDeviceToHost, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  const double *beta_d = P<double>(ctx->coef) + 2 * p;
  const double kappa = (ctx->e_max + ctx->e_min) / (ctx->e_max - ctx->e_min);
  const uint64_t *sgn = ctx->signs ? P<uint64_t>(ctx->sgn) : nullptr;
  const double *rden = ctx->signs ? nullptr : P<double>(ctx->rden);
  auto dptr = [](char *c) { return reinterpret_cast<double *>(c); };

  rfo::StepArgs sa;
  fill_step(ctx, pl, sa);
  rfo::InitArgs ia;
  fill_init(ctx, pl, ia);
  ia.scale = nullptr;
  ia.acc = nullptr;
  ia.part = nullptr;
  // S r (slot 6), from r written into slot 2
  ia.out = slot(2);
  HIPCHK(launch_init_slot(ctx, pl, ia));
  {
    rfo::StepArgs ss = sa;
    ss.hval = ctx->s64.p;
    ss.x = slot(2);
    ss.prev = nullptr;
    ss.out = slot(o_sr);
    ss.c1 = 1.0;
    ss.c2 = 0.0;
    HIPCHK(launch_any_step(ctx, pl, ss));
  }
  // reverse steps: the probe term beta_i S r comes from S r as a dense probe block (its
  // padding columns are S times those of r: zero for dense probes, whose loads the
  // padding variant skips, and computed in full for sign-bit probes)
  rfo::StepArgs rs = sa;
  rs.sgn = nullptr;
  rs.rden = dptr(slot(o_sr));
  auto ts = [&](int64_t t) { return slot(o_ts + t); };
  auto zs = [&](int64_t t) { return slot(o_zs + t); };
  auto xs = [&](int64_t t) { return slot(o_xs + t); };
  auto cka = [&](int64_t q) { return slot(o_ck + 2 * (q - 1)); };
  auto ckb = [&](int64_t q) { return slot(o_ck + 2 * (q - 1) + 1); };
  const size_t vb = pl.slot_bytes;
  char *vnear = slot(o_v), *vfar = slot(o_v + 1);  // v_{i+1}, v_{i+2} before step i
  for (int64_t q = Q - 1; q >= 0; --q) {
    const int64_t j0 = q * m, j1 = std::min(j0 + m, P1), len = j1 - j0;
    // replay: ts[t] = t_{j0+t} = S^{-1} y_{j0+t}, y pair in slots 0 and 1
    char *ycur = slot(0), *yprv = slot(1);
    if (q == 0) {
      ia.out = ycur;
      ia.scale = nullptr;
      HIPCHK(launch_init_slot(ctx, pl, ia));
    } else {
      HIPCHK(hipMemcpyAsync(ycur, ckb(q), vb, hipMemcpyDeviceToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(yprv, cka(q), vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
    TRY(cg_solve(ctx, pl, ctx->vec, ycur, ts(0)));
    for (int64_t t = 1; t < len; ++t) {
      const bool first = j0 + t == 1;  // y_1 = H_hat t_0
      sa.x = ts(t - 1);
      sa.prev = first ? nullptr : yprv;
      sa.out = yprv;
      sa.c1 = first ? 1.0 : 2.0;
      sa.c2 = first ? 0.0 : -1.0;
      sa.beta = nullptr;
      sa.acc = nullptr;
      sa.part = nullptr;
      HIPCHK(launch_any_step(ctx, pl, sa));
      std::swap(ycur, yprv);
      TRY(cg_solve(ctx, pl, ctx->vec, ycur, ts(t)));
    }
    // reverse: zs[t] = z_{j0+t}, t = 0 .. len + 1.  The top segment starts from
    // z_{p-1} = beta_{p-1} r and v_{p-1} = beta_{p-1} S r (z_p = 0 is not stored); the
    // others find z_{j1}, z_{j1+1} in zs[len], zs[len+1] and v_{j1}, v_{j1+1} in the v pair
    if (q == Q - 1) {
      ia.out = zs(len);
      ia.scale = beta_d + (p - 1);
      HIPCHK(launch_init_slot(ctx, pl, ia));
      ia.scale = nullptr;
      HIPCHK(rfo::launch_combine(dptr(vnear), beta[(size_t)(p - 1)], dptr(slot(o_sr)), 0.0, nullptr, 0.0,
                                 nullptr, 0.0, nullptr, nullptr, ctx->n, ctx->sp, ctx->stream));
    }
    for (int64_t i = j1 - 1; i >= j0; --i) {
      const bool top = i == p - 2;  // v_{i+2} = v_p = 0
      rs.x = zs(i + 1 - j0);
      rs.prev = top ? nullptr : vfar;
      rs.out = vfar;
      rs.c1 = 2.0;
      rs.c2 = top ? 0.0 : -1.0;
      rs.beta = beta_d + i;
      rs.acc = nullptr;
      rs.part = nullptr;
      HIPCHK(launch_any_step(ctx, pl, rs));
      std::swap(vnear, vfar);  // vnear = v_i, vfar = v_{i+1}
      TRY(cg_solve(ctx, pl, ctx->vec, vnear, zs(i - j0)));
    }
    // dF/dS left factors xs[t] = kappa z_{j+1} + (z_j + z_{j+2} - beta_j r)/2, j = j0 + t
    for (int64_t t = 0; t < len; ++t) {
      const int64_t j = j0 + t;
      const bool zp = j + 2 == p;  // z_p = 0
      HIPCHK(rfo::launch_combine(dptr(xs(t)), kappa, dptr(zs(t + 1)), 0.5, dptr(zs(t)), zp ? 0.0 : 0.5,
                                 zp ? nullptr : dptr(zs(t + 2)), -0.5 * beta[(size_t)j], sgn, rden, ctx->n,
                                 ctx->sp, ctx->stream));
    }
    // G (+)= the symmetric parts: sum_t coef_t (X_I t_J^T + t_I X_J^T) / 2 over the segment
    rfo::SddmmArgs a;
    memset(&a, 0, sizeof(a));
    a.brow = P<int64_t>(ctx->brow);
    a.col = P<int32_t>(ctx->col);
    a.nnzb = ctx->nnzb;
    a.bd = ctx->bd;
    a.sp = ctx->sp;
    a.xstride = (int64_t)(pl.slot_bytes / pl.vt_bytes);
    a.ybase = ts(0);
    a.ystride = a.xstride;
    a.w = P<double>(ctx->w);
    a.count = (int)len;
    a.j0 = j0;
    a.first = 1.0;
    a.rest = 2.0;
    a.accumulate = q == Q - 1 ? 0 : 1;
    a.nzlist = P<int64_t>(ctx->nz_up);
    a.nlist = ctx->n_up;
    a.ppl = sddmm_ppl(ctx);
    a.sym = 1;
    a.s_live = (int)ctx->s;
    a.xbase = zs(1);
    a.scale = 1.0 / (ctx->e_max - ctx->e_min);
    a.G = P<double>(ctx->G);
    HIPCHK(launch_sddmm_segment(ctx, kp, a, pl.slot_bytes, ctx->stream));
    a.xbase = xs(0);
    a.scale = -0.5;
    a.G = P<double>(ctx->GQ);
    HIPCHK(launch_sddmm_segment(ctx, kp, a, pl.slot_bytes, ctx->stream));
    if (q > 0) {
      // the segment below starts from z_{j0}, z_{j0+1} (its zs[m], zs[m+1]) and v_{j0}, v_{j0+1}
      HIPCHK(hipMemcpyAsync(zs(m), zs(0), vb, hipMemcpyDeviceToDevice, ctx->stream));
      HIPCHK(hipMemcpyAsync(zs(m + 1), zs(1), vb, hipMemcpyDeviceToDevice, ctx->stream));
    }
  }
  return RFO_OK;
}

// Bytes of the adjoint's vector slots for the current probes (doubled or direct
// form; see the two functions above).
size_t adjoint_slot_bytes(const rfo_ctx *ctx, const Plan &pl, int64_t p, bool dbl) {
  const int64_t K = dbl ? p / 2 : p - 1;
  int64_t m = 2;
  while (m * m < K) ++m;
  const int64_t Q = K > 0 ? (K + m - 1) / m : 0;
  const int64_t n_ck = Q > 1 ? 2 * (Q - 1) : 0;
  if (ctx->has_s) return (size_t)(9 + 3 * m + 2 + n_ck) * pl.slot_bytes;  // energy_grad_overlap
  const int n_sets = dbl && Q > 1 && tuned(ctx, RFO_TUNE_OVERLAP, 0) != 0 ? 2 : 1;
  const int64_t slots = dbl ? n_sets * 2 * (m + 2) + n_ck : m + (m + 2) + n_ck;
  return (size_t)std::max<int64_t>(slots, 2) * pl.slot_bytes;
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
  // with an overlap the direct recurrence (moment doubling needs a symmetric H_hat)
  const bool dbl = ctx->doubling && p >= 2 && !ctx->has_s;
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  TRY(ensure(ctx, ctx->G, gbytes));
  ctx->has_grad = false;
  // Probe batches: the vector slots grow with the probe count, so when they would
  // exceed the memory budget (RFO_TUNE_ADJOINT_BYTES, default 85% of the device
  // memory free at the call plus what the slots already hold) the probe columns
  // are processed in batches of the widest padded width that fits, each adding
  // its sums to G (fixed batch order: bitwise reproducible).
  size_t budget = 0;
  {
    size_t free_b = 0, total_b = 0;
    HIPCHK(hipMemGetInfo(&free_b, &total_b));
    budget = (size_t)(0.85 * (double)(free_b + ctx->vec.bytes));
    if (ctx->tune[RFO_TUNE_ADJOINT_BYTES] >= 0) budget = (size_t)ctx->tune[RFO_TUNE_ADJOINT_BYTES];
  }
  const size_t per_probe = adjoint_slot_bytes(ctx, pl, p, dbl) / (size_t)ctx->sp;
  int width = ctx->sp;
  while (width > 64 && (size_t)width * per_probe > budget) width = width > 128 ? width - 128 : 64;
  if ((size_t)width * per_probe > budget)
    return fail(ctx, RFO_E_NOMEM, "the adjoint needs %zu bytes of vectors for one batch of 64 probes; "
                "the budget is %zu", (size_t)64 * per_probe, budget);
  if (ctx->has_s && width < ctx->sp)
    return fail(ctx, RFO_E_NOMEM, "the gradient with an overlap needs %zu bytes of vectors; the budget "
                "is %zu (probe batches are not taken with an overlap)", (size_t)ctx->sp * per_probe, budget);
  double *obs = P<double>(ctx->small);
  // Probe batches [c0, c0 + s_b): of `width` columns when the budget asks for them.
  // Without that, a last VALU probe tile of 128 columns holding at most 64 real ones
  // runs as a batch of its own, 64 columns wide: a tile costs about the same whatever
  // part of it is live (the Hamiltonian is read and staged once per tile).
  std::vector<std::pair<int64_t, int64_t>> batches;
  if (width < ctx->sp) {
    for (int64_t c0 = 0; c0 < ctx->s; c0 += width) batches.push_back({c0, std::min<int64_t>(width, ctx->s - c0)});
  } else {
    batches = last_tile_batches(ctx);
  }
  if (batches.empty()) {
    const size_t need = adjoint_slot_bytes(ctx, pl, p, dbl);
    if (!dbl) TRY(ensure(ctx, ctx->vec, need));  // the doubled form sizes its slots with the tail
    size_t n_events = 0;
    // on request, what the budget leaves over keeps the last forward vectors (no
    // replay of the top segments of the doubled adjoint)
    const size_t tail = tuned(ctx, RFO_TUNE_ADJOINT_TAIL, 0) != 0 && budget > need ? budget - need : 0;
    TRY(ctx->has_s ? energy_grad_overlap(ctx, pl, p, &n_events)
        : dbl      ? energy_grad_doubling(ctx, pl, p, false, &n_events, tail)
                   : energy_grad_direct(ctx, pl, p, false, &n_events));
    HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                              ctx->sp, obs, ctx->stream));
    TRY(check_flags_and_finish(ctx, n_events));
  } else {
    // the moments of every batch are gathered into the context's [p][sp] moments for
    // the traces (and rfo_traces_at)
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
      const int sp_b = ctx->sp;
      const Plan bpl = make_plan(ctx);
      TRY(ensure(ctx, ctx->ring, (size_t)bpl.ring * bpl.grid * sp_b * sizeof(double)));
      TRY(ensure(ctx, ctx->vec, adjoint_slot_bytes(ctx, bpl, p, dbl)));
      size_t n_events = 0;
      TRY(dbl ? energy_grad_doubling(ctx, bpl, p, !first, &n_events, 0)
              : energy_grad_direct(ctx, bpl, p, !first, &n_events));
      HIPCHK(hipMemcpy2DAsync(P<double>(mom_all) + c0, pb.sp * sizeof(double), ctx->moments.p,
                              sp_b * sizeof(double), s_b * sizeof(double), p,
                              hipMemcpyDeviceToDevice, ctx->stream));
      TRY(check_flags_and_finish(ctx, n_events));
      first = false;
    }
    // the gathered moments (padding columns zero) become the context's moments
    pb.restore();
    std::swap(ctx->moments, mom_all);
    HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                              ctx->sp, obs, ctx->stream));
  }
  HIPCHK(rfo::launch_mirror(P<int64_t>(ctx->nz_low), ctx->n_low, P<int64_t>(ctx->tpos), ctx->bd,
                            P<double>(ctx->G), ctx->stream));
  if (ctx->has_s)
    HIPCHK(rfo::launch_mirror(P<int64_t>(ctx->nz_low), ctx->n_low, P<int64_t>(ctx->tpos), ctx->bd,
                              P<double>(ctx->GQ), ctx->stream));
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  TRY(copy_out(ctx, dFdH_out, ctx->G.p, gbytes));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  ctx->has_grad = true;
  ctx->grad_s = ctx->has_s;
  ctx->has_q = false;  // with an overlap GQ now holds dF/dS
  ctx->has_dens = false;
  ctx->mom_p = p;
  return RFO_OK;
}

int rfo_hf_forces(rfo_ctx *ctx, const double *dHdR, double *forces_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_grad) return fail(ctx, RFO_E_STATE, "no gradient: call rfo_energy_and_dEdH first");
  if (ctx->grad_s)
    return fail(ctx, RFO_E_STATE, "the gradient has an overlap term: use rfo_hf_forces_overlap");
  return rfo_hf_forces_overlap(ctx, dHdR, nullptr, forces_out);
}

int rfo_hf_forces_overlap(rfo_ctx *ctx, const double *dHdR, const double *dSdR, double *forces_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_grad) return fail(ctx, RFO_E_STATE, "no gradient: call rfo_energy_and_dEdH first");
  if (!dHdR || !forces_out) return fail(ctx, RFO_E_INVALID, "NULL argument");
  if (ctx->grad_s && !dSdR) return fail(ctx, RFO_E_INVALID, "the gradient has an overlap term: dSdR is NULL");
  if (!ctx->grad_s && dSdR) return fail(ctx, RFO_E_STATE, "the last gradient has no overlap term");
  HIPCHK(hipSetDevice(ctx->device));
  const size_t dbytes = (size_t)ctx->nnzb * 3 * ctx->bd * ctx->bd * sizeof(double);
  TRY(ensure(ctx, ctx->dHdR, dbytes));
  TRY(ensure(ctx, ctx->forces, (size_t)ctx->nb * 3 * sizeof(double)));
  HIPCHK(hipMemcpyAsync(ctx->dHdR.p, dHdR, dbytes, hipMemcpyDefault, ctx->stream));
  // force_a = -(sum <dF/dH, dH/dR_a> + sum <dF/dS, dS/dR_a>) over the stored blocks
  HIPCHK(rfo::launch_forces(P<int64_t>(ctx->row_ptr), P<int64_t>(ctx->tpos), P<double>(ctx->G),
                            P<double>(ctx->dHdR), ctx->nb, ctx->bd, P<double>(ctx->forces), 1.0, 0,
                            ctx->stream));
  if (dSdR) {
    HIPCHK(hipMemcpyAsync(ctx->dHdR.p, dSdR, dbytes, hipMemcpyDefault, ctx->stream));
    HIPCHK(rfo::launch_forces(P<int64_t>(ctx->row_ptr), P<int64_t>(ctx->tpos), P<double>(ctx->GQ),
                              P<double>(ctx->dHdR), ctx->nb, ctx->bd, P<double>(ctx->forces), 1.0, 1,
                              ctx->stream));
  }
  TRY(copy_out(ctx, forces_out, ctx->forces.p, (size_t)ctx->nb * 3 * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RFO_OK;
}

int rfo_get_dFdS(rfo_ctx *ctx, double *dFdS_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  if (!ctx->has_grad || !ctx->grad_s)
    return fail(ctx, RFO_E_STATE, "no overlap gradient: call rfo_energy_and_dEdH with an overlap first");
  if (!dFdS_out) return fail(ctx, RFO_E_INVALID, "dFdS_out is NULL");
  HIPCHK(hipSetDevice(ctx->device));
  TRY(copy_out(ctx, dFdS_out, ctx->GQ.p, (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double)));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  return RFO_OK;
}

}  // extern "C"
