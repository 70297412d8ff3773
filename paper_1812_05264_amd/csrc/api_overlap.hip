// C ABI: the overlap S of a nonorthogonal basis, the Q blocks and the density forces.
#include "api_internal.h"

using namespace rfo_api;

extern "C" {
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

}  // extern "C"
