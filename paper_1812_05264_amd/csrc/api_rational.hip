// C ABI: the rational (pole) estimate, complex shifted solves by CGLS.
#include "api_internal.h"

using namespace rfo_api;

namespace {

// ---------------------------------------------------------------------------
// Rational expansion (Rational approximation, Eq. rational_PQ; the rational
// free-energy derivative, Eq. rational_derivative with dS = 0).  The solves run on
// the mapped H_hat (and S) already on the device:
//   H - z S = c (H_hat - z_hat S),  c = (e_max - e_min)/2,  z_hat = (z - d)/c,
//   d = (e_max + e_min)/2,  so (H - z S)^{-1} y = x / c  with  (H_hat - z_hat S) x = y.
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
               bool first, int64_t *iters, const double *rhs = nullptr) {
  const int64_t n = ctx->n;
  const int sp = ctx->sp;
  const int G = rfo::cg_nparts(n), grid = w.ca.grid;
  // right-hand side: the probes, or a dense real [n][sp] block when rhs is given
  const uint64_t *sgn = rhs ? nullptr : ctx->signs ? P<uint64_t>(ctx->sgn) : nullptr;
  const double *rden = rhs ? rhs : ctx->signs ? nullptr : P<double>(ctx->rden);
  double *sc = w.sc;
  double *yy = sc, *ssn = sc + 3 * sp, *rr = sc + 4 * sp, *al = sc + 5 * sp, *be = sc + 6 * sp,
         *res_d = sc + 7 * sp;
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
    HIPCHK(rfo::launch_cgls_reduce(w.part, grid, nullptr, 0, sp, sc, 1, res_d, ctx->stream));
    HIPCHK(rfo::launch_cx_update(w.r, w.q, al, n, sp, w.part2, ctx->stream));  // |r|^2 partials
    TRY(cspmm(ctx, w, w.r, w.s, zr, -zi, w.part));  // s = A^H r
    HIPCHK(rfo::launch_cgls_reduce(w.part, grid, w.part2, G, sp, sc, 2, res_d, ctx->stream));
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

}  // namespace

extern "C" {
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
  if (ctx->has_s && dFdH_out && density_out)
    return fail(ctx, RFO_E_UNSUPPORTED,
                "with an overlap, request the density and the gradient in separate calls (the Q blocks "
                "and dF/dS share a buffer)");
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
  if (ctx->tune[RFO_TUNE_CPLX_PPL] >= 0) w.ppl = ctx->tune[RFO_TUNE_CPLX_PPL] == 2 && sp % 128 == 0 ? 2 : 1;
  w.u = ctx->bd == 1 ? 4 : 1;
  {
    const int u = (int)tuned(ctx, RFO_TUNE_CPLX_ROWS, w.u);
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
    grid = tuned(ctx, RFO_TUNE_CPLX_GRID, grid);
    const int64_t units = (int64_t)w.ca.n_pt * w.ca.n_rg;
    grid = std::min(grid, (units + 7) / 8 * 8);
    w.ca.grid = (int)std::max<int64_t>(8, grid / 8 * 8);
  }
  w.nparts = std::max(rfo::cg_nparts(n), w.ca.grid);
  // planes: x, r, p, q, s (complex), the P r accumulator, and S r with an overlap; for the
  // gradient with an overlap also the second solution (complex) and r
  const bool grad_s = grad && ctx->has_s;
  TRY(ensure(ctx, ctx->rat, (size_t)(grad_s ? 15 : ctx->has_s ? 12 : 11) * plane * sizeof(double)));
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
  sa.s_live = (int)ctx->s;
  const size_t gbytes = (size_t)ctx->nnzb * ctx->bd * ctx->bd * sizeof(double);
  ctx->has_grad = ctx->has_dens = ctx->has_q = false;
  ctx->grad_s = false;
  // with an overlap: the second solves h_k = (H_hat - z_hat S)^{-1} S r (warm-started from
  // the previous pole's, in X2) and r as a plane; the gradient terms are symmetric parts
  // summed on the blocks on and above the diagonal (then mirrored)
  double *X1 = w.x, *X2 = grad_s ? base + 12 * plane : nullptr, *Rp = grad_s ? base + 14 * plane : nullptr;
  auto sym_term = [&](const double *X, const double *Y, double coef, double *G, int acc) -> int {
    rfo::SddmmArgs b = sa;
    b.nzlist = P<int64_t>(ctx->nz_up);
    b.nlist = ctx->n_up;
    b.sym = 1;
    b.xbase = X;
    b.ybase = Y;
    b.first = 0.5 * coef;  // the symmetric kernel adds X Y^T + Y X^T
    b.G = G;
    b.accumulate = acc;
    HIPCHK(rfo::launch_sddmm(0, b, ctx->stream));
    return RFO_OK;
  };
  if (grad_s) {
    TRY(ensure(ctx, ctx->G, gbytes));
    TRY(ensure(ctx, ctx->GQ, gbytes));
    HIPCHK(rfo::launch_cx_fill(sgn, rden, n, sp, 1.0, Rp, nullptr, ctx->stream));
    // dF/dH starts at g1 r (S^{-1} r)^T; dF/dS at -g1 (S^{-1} H r)(S^{-1} r)^T, with
    // S^{-1} H r by CG from H r = c q (in the real planes of r and s, free before the poles)
    TRY(sym_term(Rp, SiR, poly[2], P<double>(ctx->G), 0));
    HIPCHK(rfo::launch_cx_scale(w.q, w.r, plane, c, ctx->stream));
    TRY(cg_solve(ctx, pl, ctx->vec, w.r, w.s));
    TRY(sym_term(w.s, SiR, -poly[2], P<double>(ctx->GQ), 0));
    HIPCHK(rfo::launch_cx_fill(sgn, rden, n, sp, 0.0, X2, X2 + plane, ctx->stream));  // h = 0
  } else if (grad) {
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
    w.x = X1;
    TRY(cgls_solve(ctx, w, zr, zi, tol, max_iter, t == 0, &iters[k]));
    // rho_k = (S r) . x_k, and P r += 2 Re[(w_k / c) x_k]
    const double wr = 2.0 * res_f[2 * k] / c, wi = 2.0 * res_f[2 * k + 1] / c;
    HIPCHK(rfo::launch_cx_pdot(sgn, rden, Sr, w.x, w.x + plane, n, sp, dens ? w.acc : nullptr, wr, wi,
                               w.part, w.part2, ctx->stream));
    HIPCHK(rfo::launch_colreduce(w.part, rfo::cg_nparts(n), sp, rho + (size_t)2 * k * sp, ctx->stream));
    HIPCHK(rfo::launch_colreduce(w.part2, rfo::cg_nparts(n), sp, rho + (size_t)(2 * k + 1) * sp,
                                 ctx->stream));
    if (grad_s) {
      // h_k c = x2 = (H_hat - z_hat S)^{-1} S r; with g_k = x1 / c, h_k = x2 / c, z_k the pole:
      //   dF/dH += -2 Re[tau_k h_k g_k^T],  dF/dS += 2 Re[tau_k (r g_k^T + z_k h_k g_k^T)],
      // Re[t x2 x1^T] = tr (a2 a1^T - b2 b1^T) - ti (a2 b1^T + b2 a1^T)  (x = a + i b)
      int64_t it2 = 0;  // counted in rfo_rational_stats; iterations_out keeps the solves with r
      w.x = X2;
      TRY(cgls_solve(ctx, w, zr, zi, tol, max_iter, t == 0, &it2, Sr));
      w.x = X1;
      const double *a1 = X1, *b1 = X1 + plane, *a2 = X2, *b2 = X2 + plane;
      const double tr = res_g[2 * k], ti = res_g[2 * k + 1];
      const double pr = poles[2 * k], pi = poles[2 * k + 1];
      const double ur = tr * pr - ti * pi, ui = tr * pi + ti * pr;  // tau_k z_k
      const double c2 = 2.0 / (c * c), c1 = 2.0 / c;
      double *GH = P<double>(ctx->G), *GS = P<double>(ctx->GQ);
      TRY(sym_term(a2, a1, -c2 * tr, GH, 1));
      TRY(sym_term(b2, b1, c2 * tr, GH, 1));
      TRY(sym_term(a2, b1, c2 * ti, GH, 1));
      TRY(sym_term(b2, a1, c2 * ti, GH, 1));
      TRY(sym_term(Rp, a1, c1 * tr, GS, 1));
      TRY(sym_term(Rp, b1, -c1 * ti, GS, 1));
      TRY(sym_term(a2, a1, c2 * ur, GS, 1));
      TRY(sym_term(b2, b1, -c2 * ur, GS, 1));
      TRY(sym_term(a2, b1, -c2 * ui, GS, 1));
      TRY(sym_term(b2, a1, -c2 * ui, GS, 1));
    } else if (grad) {
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
  if (grad_s) {
    HIPCHK(rfo::launch_mirror(P<int64_t>(ctx->nz_low), ctx->n_low, P<int64_t>(ctx->tpos), ctx->bd,
                              P<double>(ctx->G), ctx->stream));
    HIPCHK(rfo::launch_mirror(P<int64_t>(ctx->nz_low), ctx->n_low, P<int64_t>(ctx->tpos), ctx->bd,
                              P<double>(ctx->GQ), ctx->stream));
  }
  if (grad) {
    TRY(copy_out(ctx, dFdH_out, ctx->G.p, gbytes));
    ctx->has_grad = true;
    ctx->grad_s = grad_s;
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

}  // extern "C"
