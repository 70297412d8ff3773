// Internal declarations shared by the host orchestration (api.hip) and the
// kernel translation units.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfo {

constexpr int kWG = 256;            // threads per workgroup (4 wave64)
constexpr int kWaves = kWG / 64;
// Column-index and H_hat value arrays are allocated with kStepPad extra zero
// blocks after nnzb so that the step kernel may read whole chunks of blocks.
constexpr int kStepPad = 8;

// ---------------------------------------------------------------------------
// Chebyshev step: out = c1 * H_hat x + c2 * prev + beta * r, fused with
//   moment partials   part[rg][c] += r_c . out        (when mom != 0)
//   density accumulator acc += sum_i alpha[i] y_{k+2-m+i}, i < m (when acc != nullptr
//     and m = acc_terms > 0): the pass holds y_{k-1} (prev), y_k (the row of x)
//     and y_{k+1} (out), so the accumulator is read and written once per up to
//     three terms; the terms are added oldest first, as one at a time would be.
// Vectors are [n][sp] row-major (n = nb * bd scalar rows, sp = padded probes).
// The work is n_pt * n_rg units of `rows_per_wg` block rows of one probe tile of
// 64*ppl probes, swept by a resident grid of `grid` workgroups.
// ---------------------------------------------------------------------------
struct StepArgs {
  const int64_t *row_ptr;
  const int32_t *col;
  const void *hval;        // H_hat blocks in the matrix type
  const void *x;           // y_k (gathered)
  const void *prev;        // y_{k-1} (may alias out)
  void *out;               // y_{k+1}
  const void *xb;          // BF16 steps: BF16 copy of y_k, the operand that is gathered
  void *outb;              // BF16 steps: BF16 copy of y_{k+1}, written with it
  const int64_t *kc_ptr;   // BF16 steps: first K chunk of each block row [nb + 1]
  const int32_t *kc_idx;   // BF16 steps: per chunk, the kKChunk gathered rows J*9 + c (-1: zero row)
  const uint64_t *sgn;     // [n][sp/64] sign bits (bit 1 = +1), or nullptr
  const double *rden;      // [n][sp] dense probes, or nullptr
  double c1, c2;
  const double *beta;      // device scalar: adds beta * r when non-null
  void *acc;               // density accumulator or nullptr
  const double *alpha;     // device array: alpha^f of the acc_terms newest terms, oldest first
  int acc_terms;           // 0..3; 3 needs prev (c2 != 0)
  double *part;            // [grid][sp] moment partials (ring slot) or nullptr
  double *part2;           // doubling moments: part gets <y_{k+1}, y_{k+1}>, part2
                           // <y_{k+1}, y_k> (instead of r . y_{k+1}); nullptr = off
  // vector sources: out += sum_{t < nsrc} srcw[t] * src[t] (same layout as out)
  const void *src[3];
  double srcw[3];
  int nsrc;
  int64_t nb;              // block rows
  int sp;
  int rows_per_wg;
  int n_rg, n_pt;
  int rpi;                 // 1x1 blocks: rows per wave iteration (1 or 2, 8 neighbours per
                           // chunk) or 7 (one row, 7 neighbours per chunk); 9x9: blocks per chunk
  int grid;                // workgroups (multiple of 8); part has [grid][sp]
  int reverse;             // sweep each XCD's range of units from its end
  int hsplit;              // BF16 steps: the pack holds hi and lo BF16 parts of H_hat
  // probe columns at or past s_live are zero in every input vector (dense probes,
  // whose padding columns are zero): a lane whose probes all lie there loads
  // nothing and stores zeros.  0 = every column is live.
  int s_live;
};

// Kernel variant of a step: 1 = density accumulator terms, 2 = doubling
// moments, 3 = vector sources, 0 = none (they are not combined).
inline int step_mode(const StepArgs &a) {
  if (a.acc != nullptr && a.acc_terms > 0) return 1;
  if (a.part2 != nullptr) return 2;
  return a.nsrc > 0 ? 3 : 0;
}

// precision: 0 = fp64 (double vectors, double H), 1 = fp32 (float vectors, float H)
hipError_t launch_step(int bd, int precision, int ppl, const StepArgs &a, hipStream_t s);

// y = scale * r (+ acc = alpha * r, + part = r . y) with the step kernel's decomposition
struct InitArgs {
  void *out;
  void *outb;              // FP32 vectors: BF16 copy of out, or nullptr
  const uint64_t *sgn;
  const double *rden;
  const double *scale;     // device scalar, nullptr = 1
  void *acc;
  const double *alpha;     // device scalar used with acc
  double *part;
  int64_t nb;
  int bd;
  int sp;
  int rows_per_wg;
  int n_rg, n_pt;
  int ppl;
  int grid;                // same grid as the step kernel
};
hipError_t launch_init(int precision, const InitArgs &a, hipStream_t s);
// Resident workgroups per CU of the step kernel variant (0 on error).
int step_blocks_per_cu(int bd, int precision, int ppl, int rpi);
// K rows per chunk of the BF16 MFMA step (the K of v_mfma_f32_16x16x32_bf16)
constexpr int kKChunk = 32;
// BF16 MFMA step for 9x9 blocks; a.hval holds the packed A operands
// ([n_chunks][36] uint4, two with split), a.n_pt counts tiles of 16 * nt_tiles probes.
hipError_t launch_step_bf16(int nt_tiles, const StepArgs &a, hipStream_t s);
int step_bf16_blocks_per_cu(int nt_tiles, int u, int split);  // u = K chunks per iteration (a.rpi)
// A operands of the K-packed BF16 step: chunk q, lane group g, output row m holds
// H_hat[nz][m][c] for the eight K rows 8g..8g+7 of the chunk, whose source codes
// kc_src[kKChunk q + k] = nz * 9 + c (-1: zero) list the block and column of each K row.
// split: each entry is followed by the low BF16 parts bf16(h - bf16(h)).
hipError_t launch_pack_bf16(const double *hhat, const int32_t *kc_src, int64_t n_chunks, int split,
                            void *apack, hipStream_t s);

// ---------------------------------------------------------------------------
// Setup kernels
// ---------------------------------------------------------------------------
// Spectral map H_hat = (2H - (a+b)I)/(b-a) plus validity checks (finite values,
// symmetric values via the transpose map); writes fp64 and (optionally) fp32.
hipError_t launch_map(const double *h, const int64_t *brow, const int32_t *col,
                      const int64_t *tpos, int64_t nnzb, int bd, double e_min,
                      double e_max, double *hhat64, float *hhat32, int *flags,
                      hipStream_t s);
// Gershgorin interval: per-workgroup partial min/max, then a final reduction.
hipError_t launch_gershgorin(const double *h, const int64_t *row_ptr,
                             const int32_t *col, int64_t nb, int bd,
                             double *scratch, double *out2, hipStream_t s);
// Probe classification (all +-1?) and packing to sign bits.
hipError_t launch_probe_pack(const double *rden, int64_t n, int s_real, int sp,
                             uint64_t *sgn, int *flags, hipStream_t st);
// Chebyshev coefficients of f, x f, g by Chebyshev-Gauss quadrature.
hipError_t launch_coefficients(double e_min, double e_max, double T, double mu,
                               int64_t p, int64_t nq, double *samples,
                               double *costab, double *coef, hipStream_t s);
// Fixed-order reduction of moment partials: moments[k][c] for k in
// [k0, k0 + count), ring slot of index k is k % ring.  Flags a moment that
// exceeds (1 + tol) * moments[0][c].  dbl: the partials are the doubling inner
// products and moment k >= 2 is 2 * sum - moments[k mod 2] (moments 0 and 1
// must be final before the launch).
hipError_t launch_moment_reduce(const double *part, int ring, int64_t k0,
                                int count, int n_rg, int sp, double *moments,
                                int check, double tol, int *flags, int dbl,
                                hipStream_t s);
// N, E, F from moments and coefficients.
hipError_t launch_traces(const double *moments, const double *w,
                         const double *coef, int64_t p, int sp, double *out3,
                         hipStream_t s);
// Masked outer products on the block pattern:
//   G[nz] (+)= sum_t coef_t sum_c w_c X_t[I-block][c] Y_t[J-block][c]
// X_t = xbase + t*xstride (precision-typed), Y_t = ybase + t*ystride, or the
// probes when ybase == nullptr.  coef_t = scale * (j0 + t == 0 ? first : rest).
struct SddmmArgs {
  const int64_t *brow;
  const int32_t *col;
  int64_t nnzb;
  int bd;
  int sp;
  const void *xbase;
  int64_t xstride;
  const void *ybase;
  int64_t ystride;
  const uint64_t *sgn;
  const double *rden;
  const double *w;
  int count;
  int64_t j0;
  double scale, first, rest;
  double *G;
  int accumulate;
  const int64_t *nzlist;   // blocks to compute (nullptr = all nnzb)
  int64_t nlist;
  int ppl;                 // probes per lane per load (1 or 2)
  int sym;                 // G[nz] (+)= sum_t coef_t sum_c w_c (X_I Y_J^T + Y_I X_J^T)
  int s_live;              // columns at or past s_live have weight zero and are skipped
                           // (0 = none)
};
hipError_t launch_sddmm(int precision, const SddmmArgs &a, hipStream_t s);

// Symmetric segment gradient of the BF16 steps on the matrix cores, from the
// vectors' BF16 copies, with one weight w0 for the first s_real probes and zero
// for the padding:
//   G[nz] (+)= sum_t coef_t w0 sum_{c < s_real} (X_I Y_J^T + Y_I X_J^T)[:, c],
// coef_t = scale * (j0 + t == 0 ? first : rest), for the upper blocks nzlist[q],
// q in [grp[g], grp[g+1]): every group lies in one block row and holds at most
// kSddmmGroup blocks.  The partial sums of one t (FP32 on the matrix cores) are
// added in FP64.
constexpr int kSddmmGroup = 6;  // measured best (10: 22% slower)
struct SddmmMfmaArgs {
  const int64_t *grp;      // [n_grp + 1]
  int64_t n_grp;
  const int64_t *nzlist;
  const int64_t *brow;
  const int32_t *col;
  int sp, s_real;
  const void *xbase, *ybase;  // BF16 (unsigned short) copies
  int64_t xstride, ystride;   // elements between the vectors of consecutive t
  int count;
  int64_t j0;
  double scale, first, rest, w0;
  double *G;
  int accumulate;
};
hipError_t launch_sddmm_bf16(const SddmmMfmaArgs &a, hipStream_t s);
// G[nz] = G[tpos[nz]]^T for the listed blocks (completes a symmetric gradient).
hipError_t launch_mirror(const int64_t *nzlist, int64_t nlist, const int64_t *tpos, int bd,
                         double *G, hipStream_t s);
// Hellmann-Feynman forces from G and d H_IJ / d R_I blocks: F (+)= sign * force.
hipError_t launch_forces(const int64_t *row_ptr, const int64_t *tpos,
                         const double *G, const double *D, int64_t nb, int bd,
                         double *F, double sign, int accumulate, hipStream_t s);

// ---------------------------------------------------------------------------
// Nonorthogonal basis: H_hat with S, and conjugate gradients for S t = y per
// probe column.  sc holds [yy | rr | pq | rrn | alpha | beta] (sp each), part
// [cg_nparts(n)][sp] column partials, resmax the largest rrn / yy after an update.
// sp must be a positive multiple of 64 (hipErrorInvalidValue otherwise).
// ---------------------------------------------------------------------------
hipError_t launch_map_overlap(const double *h, const double *s, const int64_t *tpos, int64_t nnzb,
                              int bd, double e_min, double e_max, double *hhat, int *flags,
                              hipStream_t st);
int cg_nparts(int64_t n);
// t = 0, r = p = y, yy = rr = |y_c|^2
hipError_t launch_cg_init(const double *y, double *t, double *r, double *p, int64_t n, int sp,
                          double *part, double *sc, hipStream_t s);
// alpha_c = rr_c / (p_c . q_c) from the column partials of p . q that the product
// q = S p left in part [nparts][sp] (its moment partials with p as the probe block);
// sets *resmax = 0 for the update that follows
hipError_t launch_cg_alpha(const double *part, int nparts, int sp, double *sc, double *resmax,
                           hipStream_t s);
// t += alpha p, r -= alpha q, beta = |r|^2 / rr, rr = |r|^2, p = r + beta p, *resmax
hipError_t launch_cg_update(double *t, double *r, double *p, const double *q, int64_t n, int sp,
                            double *part, double *sc, double *resmax, hipStream_t s);

// ---------------------------------------------------------------------------
// Rational expansion with S = I: CGLS for (H_hat - z) x = y per probe column on
// complex vectors stored as two real [n][sp] planes (re, then im, `plane`
// elements apart).  Column partials are [nparts][sp]; launch_colreduce sums
// them in a fixed order.  CGLS scalars sc = [yy | gam | qq | ssn | rr | alpha |
// beta] (sp each).
// ---------------------------------------------------------------------------
hipError_t launch_colreduce(const double *part, int nparts, int sp, double *out, hipStream_t s);
// out = ca A + cb B + cc C + cr r over n rows of sp FP64 columns (null operands add nothing;
// r from sgn or rden as in the step kernels)
hipError_t launch_combine(double *out, double ca, const double *A, double cb, const double *B, double cc,
                          const double *C, double cr, const uint64_t *sgn, const double *rden, int64_t n,
                          int sp, hipStream_t s);

// out = (H_hat - z) x, with the column partials of |out_c|^2 when part != nullptr
// ([grid][sp]); same unit decomposition as the Chebyshev step (the value and
// column arrays carry kStepPad zero entries past nnzb).
struct CspArgs {
  const int64_t *row_ptr;
  const int32_t *col;
  const double *hval;      // H_hat blocks (FP64)
  const double *sval;      // overlap S blocks (out = H_hat x - z S x), or nullptr (S = I)
  const double *x;         // complex input (two planes)
  double *out;             // complex output (two planes), not aliasing x
  double zr, zi;           // the shift z
  double *part;            // [grid][sp] partials or nullptr
  int64_t nb;              // block rows
  int64_t plane;           // n * sp
  int sp;
  int rows_per_wg;
  int n_rg, n_pt;          // n_pt probe tiles of 64 * ppl
  int grid;                // multiple of 8
};
// u: neighbours per chunk (1x1: 4 or 8; 9x9: blocks per chunk, 1 or 2)
hipError_t launch_cspmm(int bd, int ppl, int u, const CspArgs &a, hipStream_t s);
int cspmm_blocks_per_cu(int bd, int ppl, int u, bool hs);
// dre = scale * y (probes), dim = 0 when non-null
hipError_t launch_cx_fill(const uint64_t *sgn, const double *rden, int64_t n, int sp, double scale,
                          double *dre, double *dim, hipStream_t s);
// r = y - q (q == nullptr: r = y); partials |r_c|^2 and |y_c|^2 ([cg_nparts(n)][sp] each)
hipError_t launch_cx_resid(const uint64_t *sgn, const double *rden, const double *q, double *r,
                           int64_t n, int sp, double *part_rr, double *part_yy, hipStream_t s);
// r -= alpha_c q; partials |r_c|^2
hipError_t launch_cx_update(double *r, const double *q, const double *alpha, int64_t n, int sp,
                            double *part, hipStream_t s);
// x += alpha_c p, then p = s + beta_c p
hipError_t launch_cx_dir(const double *sv, double *p, double *x, const double *alpha,
                         const double *beta, int64_t n, int sp, hipStream_t s);
// partials y_c . a_c, y_c . b_c with y the probes (yd == nullptr) or the plane yd;
// acc += wr a - wi b when acc != nullptr
hipError_t launch_cx_pdot(const uint64_t *sgn, const double *rden, const double *yd, const double *a,
                          const double *b, int64_t n, int sp, double *acc, double wr, double wi,
                          double *part_a, double *part_b, hipStream_t s);
// dst = alpha * src (n elements)
hipError_t launch_cx_scale(const double *src, double *dst, int64_t n, double alpha, hipStream_t s);
// mode 0: gam = ssn, *resmax;  1: alpha = gam / qq;  2: beta = ssn / gam, gam = ssn, *resmax
hipError_t launch_cgls_scalars(double *sc, int sp, int mode, double *resmax, hipStream_t s);
// the column sums and scalars of one half-iteration in one kernel: mode 1 reduces pa
// [na][sp] into qq and forms alpha (and zeroes *resmax); mode 2 reduces pa into ssn and
// pb [nb][sp] into rr and forms beta, gam and *resmax (the values of launch_colreduce
// followed by launch_cgls_scalars)
hipError_t launch_cgls_reduce(const double *pa, int na, const double *pb, int nb, int sp, double *sc,
                              int mode, double *resmax, hipStream_t s);
struct RationalScalars {
  double f0, ew, g0, g1;   // constant of f, 2 Re sum_k w_k, constant and slope of g
};
// N, E, F from rho [n_poles][2][sp] ((S r_c) . x_kc), m01 [2][sp] (r.r, (H r).(S^{-1} r)),
// weights and coef [3][n_poles] complex (N, E, F coefficients of rho).
hipError_t launch_rational_traces(const double *rho, const double *m01, const double *w,
                                  const double *coef, int n_poles, int sp,
                                  const RationalScalars &k, double *out3, hipStream_t s);

}  // namespace rfo
