/*
 * rfo.h -- randomized Fermi-operator expansion on one MI355X (gfx950).
 *
 * C ABI of the hot path of the randomized Chebyshev method assessed in
 * Moussa & Baczewski, "Assessment of localized and randomized algorithms for
 * electronic structure" (arXiv:1812.05264).  For an orthogonal (S = I) sparse
 * tight-binding Hamiltonian H, a temperature T and a chemical potential mu the
 * library evaluates, from a block of probe vectors R = [r_1 ... r_s]:
 *
 *   moments   mu_{k,c} = r_c^T T_k(H_hat) r_c, k < p, with the spectral map
 *             H_hat = (2H - (e_max + e_min) I)/(e_max - e_min)
 *             (Polynomial approximation; Chebyshev recursion with S = I);
 *   traces    N = tr f(H), E = tr[H f(H)], F = tr g(H), each as
 *             sum_c w_c sum_k c_k mu_{k,c} with the Chebyshev coefficients c_k
 *             of f, x f(x) or g (Methods: free-energy function g, Fermi
 *             function f = g', free energy, electron count and band energy);
 *   density   M (.) P~ = sum_c w_c M (.) (f(H) r_c r_c^T) on H's block
 *             pattern M (Random approximation, random density estimator);
 *   gradient  dF~/dH on H's block pattern for the probe estimate
 *             F~ = sum_c w_c r_c^T g_p(H) r_c, by the reverse (Clenshaw)
 *             form of the polynomial free-energy derivative (Analytical
 *             free-energy derivatives), and from it Hellmann-Feynman forces
 *             (Observable response, dF/dlambda = tr[P dH/dlambda]).
 *
 * Conventions shared by every call:
 *   - All functions return an rfo_status.  Nothing is thrown across the ABI.
 *     On failure rfo_last_error() describes the cause.
 *   - A context is not thread-safe; distinct contexts are independent.
 *   - Every pointer belongs to the caller.  set_* calls copy their inputs, so
 *     the caller may free them on return.  Output pointers may be host memory
 *     or device memory of the context's GPU (unified addressing decides the
 *     copy direction); a call returns only once its outputs are complete.
 *   - Work is issued on the stream given to rfo_create (NULL = the null
 *     stream), so the library interoperates with a PyTorch stream.
 *   - Block-sparse row (BSR) layout, used by every H-shaped array:
 *       row_ptr int64 [n_block_rows + 1], row_ptr[0] = 0, non-decreasing;
 *       col_idx int32 [nnzb], strictly increasing inside a block row;
 *       blocks  [nnzb][block_dim][block_dim] row-major;
 *     block_dim is 1 or 9, every block row stores its diagonal block, the
 *     pattern is symmetric and H_JI = H_IJ^T.
 *   - Probe layout: R [n][s] row-major, n = n_block_rows * block_dim.
 *   - The library reads no environment variables.  Launch geometry and schedule
 *     choices are context state (rfo_set_tuning); their defaults are the measured best.
 */
#ifndef RFO_H
#define RFO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The library is built with hidden symbols by default; these are its exports. */
#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility push(default)
#endif

typedef struct rfo_ctx rfo_ctx;

typedef enum {
  RFO_OK = 0,
  RFO_E_INVALID = -1,     /* bad argument, layout or pattern */
  RFO_E_STATE = -2,       /* call out of order (e.g. moments before probes) */
  RFO_E_NOMEM = -3,       /* device allocation failed */
  RFO_E_DEVICE = -4,      /* HIP runtime error */
  RFO_E_NUMERIC = -5,     /* non-finite input, or |mu_{k,c}| > ||r_c||^2:
                             the spectrum left [e_min, e_max] */
  RFO_E_UNSUPPORTED = -6  /* valid request the library does not implement */
} rfo_status;

/* Arithmetic of the H.V products (Chebyshev steps).  Spectral map, moments,
 * traces and Chebyshev coefficients are always FP64. */
typedef enum {
  RFO_FP64 = 0,           /* FP64 vectors and H */
  RFO_FP32 = 1,           /* FP32 vectors and H, FP64 moments */
  RFO_BF16 = 2,           /* BF16 H and vector operands on MFMA, FP32
                             accumulation and FP32 vectors, FP64 moments */
  RFO_BF16X2 = 3          /* as RFO_BF16 with H_hat as a pair of BF16 values
                             hi + lo (two MFMAs per K chunk): the rounding of
                             H_hat falls from 2^-9 to about 2^-17 relative */
} rfo_precision;

/* Creates a context on HIP device `device`; `hip_stream` is a hipStream_t or
 * NULL.  *out receives the context (NULL on failure). */
int rfo_create(rfo_ctx **out, int device, void *hip_stream);

/* Frees all device memory of the context.  NULL is ignored. */
void rfo_destroy(rfo_ctx *ctx);

/* Message of the last failed call on ctx ("" if none); valid until the next
 * call on ctx.  With ctx == NULL: the message of the calling thread's last failed
 * rfo_create. */
const char *rfo_last_error(const rfo_ctx *ctx);

/* Sets H (paper: Methods, orthogonal basis S = I; Polynomial approximation,
 * spectral interval [e_min, e_max]).  The library stores the mapped
 * Hamiltonian H_hat = (2H - (e_max + e_min) I)/(e_max - e_min) in the
 * requested precision.  If e_min >= e_max the interval is Gershgorin's,
 * widened by 1% about its centre.
 *   row_ptr, col_idx: host memory; values: host or device memory, FP64.
 *   row_ptr == NULL && col_idx == NULL keeps the previous pattern and replaces
 *   the values only (n_block_rows and block_dim must repeat).
 * Errors: RFO_E_INVALID for a bad layout, a missing diagonal block, an
 * asymmetric pattern or asymmetric values; RFO_E_NUMERIC for non-finite
 * values. */
int rfo_set_hamiltonian(rfo_ctx *ctx, int64_t n_block_rows, int block_dim,
                        const int64_t *row_ptr, const int32_t *col_idx,
                        const double *values, double e_min, double e_max,
                        int precision);

/* Returns the spectral interval in use (after a Gershgorin fallback). */
int rfo_get_interval(const rfo_ctx *ctx, double *e_min, double *e_max);

/* Sets the probe block R [n][s] (host memory, FP64) and weights w [s]
 * (host memory; NULL = 1/s each), so that sum_c w_c r_c r_c^T estimates the
 * identity (Random approximation: mean of R R^dagger is I).  Probes whose
 * entries are all +-1 (Rademacher) are stored as sign bits; any other real
 * probes are stored in FP64.  Must follow rfo_set_hamiltonian (n must match);
 * setting a new Hamiltonian of another size clears the probes. */
int rfo_set_probes(rfo_ctx *ctx, int64_t n_probes, const double *R,
                   const double *weights);

/* Chebyshev moments, traces and density blocks (paper: Polynomial
 * approximation, Eq. poly_PQ with S = I: the three-term recurrence
 * y_0 = r, y_1 = H_hat r, y_{k+1} = 2 H_hat y_k - y_{k-1}, and P r ~ sum_k
 * alpha^f_k y_k; Random approximation, Eq. random_density: M (.) P~ =
 * sum_c w_c M (.) (P r_c) r_c^T; traces as in the file header).
 * Runs p = n_terms Chebyshev terms (p - 1 H.V steps) on every probe.
 *   moments_out [s][p]  per-probe mu_{k,c} (nullable)
 *   NEF_out     [3]     N, E, F (nullable)
 *   density_out [nnzb][bd][bd]  M (.) P~, unsymmetrized (nullable; when NULL
 *               the density accumulator is not run)
 * Without density and with moment doubling on (the default), the moments come
 * from floor(p/2) steps instead: mu_2j = 2 y_j.y_j - mu_0 and
 * mu_2j-1 = 2 y_j.y_j-1 - mu_1 (T_2j = 2 T_j^2 - T_0, T_2j-1 = 2 T_j T_j-1 - T_1),
 * the same values up to rounding.
 * In FP64 and FP32 without an overlap, a last probe tile of 128 columns holding at most
 * 64 real probes runs as a batch of its own, 64 columns wide (the same values up to the
 * order of FP64 sums).
 * Requires T > 0, finite mu, 1 <= n_terms <= 1048576.
 * Errors: RFO_E_STATE without H or probes; RFO_E_NUMERIC when a moment
 * exceeds ||r_c||^2 (relative slack 1e-6 in FP64, 1e-3 in FP32/BF16). */
int rfo_fermi_moments(rfo_ctx *ctx, double T, double mu, int64_t n_terms,
                      double *moments_out, double *NEF_out,
                      double *density_out);

/* rfo_fermi_moments without density and without any device allocation, for
 * callers that cannot allocate (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  The same kernels in the same order:
 * the results equal those of rfo_fermi_moments with density_out = NULL, except
 * when that call runs a mostly-padding last probe tile as a batch of its own
 * (more than 128 probes, s mod 128 in 1..64): this call keeps one block, and the
 * two agree to rounding.  Like the other calls it waits for its work before it
 * returns (it reads the status flag and copies N, E, F out), so it allocates
 * nothing but is not itself recorded into a HIP graph.  The
 * work memory comes from a fixed device array of the library, 128 MiB per device
 * (held from the first such call on a device until the process ends), shared by
 * every call on that device: calls that overlap on one device race.  It must
 * hold two probe vectors (n * sp * 8 bytes each in FP64; 4 in FP32; 6 in BF16,
 * sp = s rounded up to 64, or to 128 above 64 probes), the moment partials and
 * moments, the coefficient tables (about 270 * n_terms bytes) and the moments in
 * the caller's layout (s * n_terms * 8 bytes).
 *   moments_out [s][p], NEF_out [3]: as for rfo_fermi_moments (nullable; host
 *   or device memory).
 * H and probes are those of the last rfo_set_hamiltonian / rfo_set_probes.
 * Afterwards rfo_traces_at has no moments (RFO_E_STATE): they stay in the shared
 * array.
 * Errors: those of rfo_fermi_moments; RFO_E_INVALID when the work memory would
 * exceed the array (nothing is launched); RFO_E_UNSUPPORTED with an overlap. */
int rfo_fermi_moments_noalloc(rfo_ctx *ctx, double T, double mu, int64_t n_terms,
                              double *moments_out, double *NEF_out);

/* N, E, F at another (T, mu) from the moments of the last rfo_fermi_moments or
 * rfo_energy_and_dEdH call (the moments do not depend on T or mu; only the
 * coefficients are recomputed, paper: Polynomial approximation).  Used for
 * scans of mu at fixed electron count.  NEF_out [3] host or device memory.
 * Errors: RFO_E_STATE before any call, or after rfo_set_hamiltonian /
 * rfo_set_probes invalidated the moments. */
int rfo_traces_at(rfo_ctx *ctx, double T, double mu, double *NEF_out);

/* Free energy F~ and its gradient dF~/dH on H's block pattern (paper:
 * Analytical free-energy derivatives, polynomial form; the interval is held
 * fixed, so dF/dH = 2/(e_max - e_min) dF/dH_hat).  The forward pass keeps
 * checkpoints every ceil(sqrt(steps)) steps and the backward pass replays one
 * segment at a time, so memory grows with sqrt(p) vectors, not p.  With moment
 * doubling on (rfo_set_moment_doubling, the default) F~ is taken through the
 * doubled moments of floor(p/2) steps and the backward recurrence carries
 * their vector sources; the result is the same gradient up to rounding.
 *   NEF_out   [3]  N, E, F of the forward pass (nullable)
 *   dFdH_out  [nnzb][bd][bd]  raw gradient G (nullable)
 * The gradient also stays on the device for rfo_hf_forces.
 * Probe columns run in batches, each adding its sums to G, when the vectors of all
 * probes exceed the memory budget (RFO_TUNE_ADJOINT_BYTES), and, in FP64 and FP32, when
 * the last probe tile of 128 columns holds at most 64 real ones (that tile then runs
 * 64 columns wide); batches change only the order of the FP64 sums.
 * With an overlap S (rfo_set_overlap) the derivative is that of F~ = sum_k beta_k
 * r^T T_k(H_hat S^{-1}) r (paper: Eq. polynomial_response), taken by the direct
 * recurrence (no moment doubling) with one conjugate-gradient solve per forward,
 * replayed and reverse step: dFdH_out then holds the symmetric part of dF~/dH
 * ((G_IJ + G_JI^T)/2, what symmetric variations of H see; with S != I the two halves
 * differ), and dF~/dS, likewise symmetrized, stays on the device for
 * rfo_get_dFdS and rfo_hf_forces_overlap.  Probe batches are not taken with an
 * overlap: RFO_E_NOMEM when the vectors of all probes exceed the budget. */
int rfo_energy_and_dEdH(rfo_ctx *ctx, double T, double mu, int64_t n_terms,
                        double *NEF_out, double *dFdH_out);

/* dF~/dS [nnzb][bd][bd] (symmetric part, host or device memory) of the last
 * rfo_energy_and_dEdH call with an overlap (paper: Analytical free-energy
 * derivatives, Eq. polynomial_response).  RFO_E_STATE without one. */
int rfo_get_dFdS(rfo_ctx *ctx, double *dFdS_out);

/* Forces from the last gradient with an overlap (paper: Observable response): for
 * a two-centre model with dHdR, dSdR [nnzb][3][bd][bd] = d H_IJ / d R_I and
 * d S_IJ / d R_I, force_a = -(sum <dF~/dH, dH/dR_a> + sum <dF~/dS, dS/dR_a>) over
 * the stored blocks.  dSdR must be NULL exactly when the gradient has no overlap
 * term (then this is rfo_hf_forces).  forces_out [n_block_rows][3].
 * Errors: RFO_E_STATE before rfo_energy_and_dEdH or for dSdR without an overlap
 * gradient; RFO_E_INVALID for a missing dSdR. */
int rfo_hf_forces_overlap(rfo_ctx *ctx, const double *dHdR, const double *dSdR,
                          double *forces_out);

/* Hellmann-Feynman forces from the last gradient (paper: Observable
 * response with S = I): for a two-centre model with
 * dHdR [nnzb][3][bd][bd] = d H_IJ / d R_I for every stored block (host or
 * device memory), force_a = -(sum_J <G_aJ, D_aJ> - sum_I <G_Ia, D_Ia>).
 *   forces_out [n_block_rows][3].
 * Errors: RFO_E_STATE before rfo_energy_and_dEdH, or when that gradient has an
 * overlap term (use rfo_hf_forces_overlap). */
int rfo_hf_forces(rfo_ctx *ctx, const double *dHdR, double *forces_out);

/* Nonorthogonal basis (paper: Polynomial approximation with S, Eq. poly_PQ).
 * values [nnzb][bd][bd] FP64 (host or device): the overlap S on H's block
 * pattern, symmetric positive definite; NULL clears it (S = I).  With S set,
 * H_hat = [2H - (e_max + e_min) S]/(e_max - e_min) and every step forms
 * y_{k+1} = 2 H_hat S^{-1} y_k - y_{k-1}, applying S^{-1} to every probe column
 * by conjugate gradients to |residual| <= cg_tol |y| (cg_tol <= 0: 1e-13).  The
 * moments stay mu_k = r . y_k (N = tr[P S]); with density output the library
 * also forms the Q blocks (Q y = S^{-1} H S^{-1} sum_k alpha_k y_k).  Moment
 * doubling is not used (T_k(H_hat S^{-1}) is not symmetric); rfo_energy_and_dEdH
 * then gives dF~/dH and dF~/dS (see there).
 * Requires FP64 precision and an interval passed to rfo_set_hamiltonian that
 * contains the spectrum of the pencil (H, S) (RFO_E_UNSUPPORTED / RFO_E_STATE
 * otherwise).  rfo_set_hamiltonian clears S.
 * Errors: RFO_E_NUMERIC for non-finite values or a CG that breaks down or does
 * not converge (S not positive definite), RFO_E_INVALID for S_JI != S_IJ^T. */
int rfo_set_overlap(rfo_ctx *ctx, const double *values, double cg_tol);

/* Q blocks [nnzb][bd][bd] of the last rfo_fermi_moments call with density and
 * an overlap (host or device memory).  RFO_E_STATE otherwise. */
int rfo_get_density_q(rfo_ctx *ctx, double *q_out);

/* Forces from the density blocks of the last rfo_fermi_moments call with
 * density (paper: Observable response): for a two-centre model with
 * dHdR, dSdR [nnzb][3][bd][bd] = d H_IJ / d R_I, d S_IJ / d R_I,
 *   force_a = -(tr[P dH/dR_a] - tr[Q dS/dR_a])
 * with the estimated P and Q blocks (dSdR NULL: no overlap term).
 * forces_out [n_block_rows][3].  Unlike rfo_hf_forces these are the forces of
 * the density estimate, not the gradient of F~.
 * Errors: RFO_E_STATE without density blocks, or dSdR without Q blocks. */
int rfo_density_forces(rfo_ctx *ctx, const double *dHdR, const double *dSdR,
                       double *forces_out);

/* Multi-color probe ensemble (paper: Hybrid approximation, the multi-color
 * vector ensemble; Implementation details, Welsh-Powell coloring).  Host-only:
 * needs no context and no GPU.  Colours the atoms so that two atoms closer than
 * r_max (strictly) never share a colour: the atoms are visited in order of
 * decreasing number of neighbours within r_max (ties by index), each taking the
 * smallest colour none of its already coloured neighbours holds.
 *   positions [n_atoms][3] (host), colours_out [n_atoms] (0 .. q-1),
 *   n_colours_out: q.
 * Errors: RFO_E_INVALID for n_atoms < 1, r_max <= 0, non-finite input or NULL;
 * RFO_E_UNSUPPORTED when the cell list would exceed 4e9 cells. */
int rfo_color_atoms(int64_t n_atoms, const double *positions, double r_max, int32_t *colours_out,
                    int32_t *n_colours_out);

/* Sets the probes to one sample of the multi-color ensemble, built on the
 * device: with q = 1 + max colour, column k * n_orb + o (k < q, o < n_orb) holds
 * signs[a][o] on orbital o of every atom a of colour k (row a * n_orb + o) and
 * zero elsewhere; every column has weight one.  The orbitals of an atom are
 * consecutive rows: n_orb must divide the number of rows n.  Replaces
 * rfo_set_probes with the block it would be given (stored in FP64).
 *   colours [n / n_orb] (host, >= 0), signs [n / n_orb][n_orb] (host, +-1).
 * Errors: RFO_E_STATE without a Hamiltonian; RFO_E_INVALID for bad arguments. */
int rfo_set_colored_probes(rfo_ctx *ctx, const int32_t *colours, int n_orb, const double *signs);

/* Rational (pole) expansion, pole fit (paper: Rational approximation, Eq.
 * rational_fit).  Host-only: needs no context and no GPU.  The paper's fastest
 * fit is numerical and unprinted; this is the analytical kind it names for a
 * finite spectral interval, applicable to both f and g: a trapezoid rule for a
 * Cauchy integral on a conformal map of an annulus (Hale, Higham and Trefethen
 * 2008), applied to the even parts of f and g as functions of (x - mu)^2.
 * With n = n_nodes it returns 2n poles z_k, all with Im z_k > 0, shared by
 *   f(x) ~ poly[0] + 2 Re sum_k res_f_k / (x - z_k),
 *   g(x) ~ poly[1] + poly[2] x + 2 Re sum_k res_g_k / (x - z_k)
 * on [e_min, e_max] (f = 2/(1 + exp((x - mu)/T)), g = -2T ln(1 + exp(-(x - mu)/T))).
 * The error falls geometrically in n at a rate set by ln((e - mu)^2 / (pi T)^2).
 *   poles, res_f, res_g: caller arrays of 2n complex numbers as (re, im) pairs
 *   [2n][2]; poly: [3] = (f0, g0, g1).
 * Errors: RFO_E_INVALID for n_nodes outside [1, 1024], T <= 0, e_max <= e_min,
 * non-finite input or NULL; RFO_E_NUMERIC if a node evaluates to non-finite. */
int rfo_rational_fit(int n_nodes, double T, double mu, double e_min, double e_max,
                     double *poles, double *res_f, double *res_g, double *poly);

/* Rational estimate (paper: Rational approximation, Eq. rational_PQ;
 * rational free-energy primitive and its derivative, Eq. rational_derivative
 * with dS = 0).  For every probe column the library solves the shifted systems
 * (H - z_k) g_k = r_c by CGLS (conjugate gradients on the normal equations)
 * to |r_c - (H - z_k) g_k| <= tol |r_c|, poles ordered by decreasing |z_k - mu|
 * and each solve started from the previous pole's solution, and forms
 *   P r = f0 r + 2 Re sum_k w_k g_k,
 *   N = sum_c w_c r_c.P r_c,
 *   E = sum_c w_c [f0 r_c.H r_c + 2 Re(sum_k w_k) r_c.r_c + 2 Re sum_k w_k z_k r_c.g_k],
 *   F = sum_c w_c [g0 r_c.r_c + g1 r_c.H r_c + 2 Re sum_k tau_k r_c.g_k],
 *   density  M (.) sum_c w_c (P r_c) r_c^T on H's block pattern,
 *   dF/dH    g1 sum_c w_c r_c r_c^T - 2 Re sum_k tau_k sum_c w_c g_k g_k^T on the
 *            pattern (G(z)^T = G(z) for symmetric H; no conjugation),
 * with w_k = res_f, tau_k = res_g, (f0, g0, g1) = poly and w_c the probe weights.
 *   mu: only orders the poles.  n_poles >= 1; poles, res_f, res_g [n_poles][2]
 *   (re, im), host memory; every pole must have Im z_k > 0.
 *   tol in (0, 1); max_iter >= 1 CGLS iterations per pole.
 *   NEF_out [3] (N, E, F), density_out, dFdH_out [nnzb][bd][bd]: NULL skips;
 *   host or device memory.  iterations_out [n_poles] (NULL skips): CGLS
 *   iterations per pole, in the caller's pole order.
 * With an overlap S set (rfo_set_overlap) the systems are (H - z_k S) g_k = r_c
 * (Eq. rational_PQ as printed) and
 *   P r = f0 S^{-1} r + 2 Re sum_k w_k g_k,   Q r = S^{-1} H P r,
 *   N = sum_c w_c (S r_c).(P r_c),  E = sum_c w_c (H r_c).(P r_c),
 *   F = sum_c w_c [g0 r_c.r_c + g1 (H r_c).(S^{-1} r_c) + 2 Re sum_k tau_k (S r_c).g_k],
 * with S^{-1} by conjugate gradients (the overlap's cg_tol); the density call
 * then also forms the Q blocks (rfo_get_density_q).  The gradient with an overlap
 * (Eq. rational_derivative with dS, and the linear part of g) takes a second solve
 * per pole, h_k = (H - z_k S)^{-1} S r_c: dFdH_out holds the symmetric part of
 *   dF/dH = sum_c w_c [g1 r_c (S^{-1} r_c)^T - 2 Re sum_k tau_k h_k g_k^T]
 * and dF/dS, likewise symmetrized,
 *   dF/dS = sum_c w_c [-g1 (S^{-1} H r_c)(S^{-1} r_c)^T + 2 Re sum_k tau_k (r_c g_k^T + z_k h_k g_k^T)],
 * stays on the device for rfo_get_dFdS and rfo_hf_forces_overlap; density and
 * gradient are then requested in separate calls (RFO_E_UNSUPPORTED otherwise).
 * After the call rfo_hf_forces (S = I) or rfo_hf_forces_overlap uses this
 * gradient (if requested), and rfo_density_forces this density (if requested
 * without the gradient).
 * Requires FP64 precision (RFO_E_UNSUPPORTED otherwise).
 * Errors: RFO_E_STATE before H and probes; RFO_E_INVALID for bad arguments;
 * RFO_E_NUMERIC if CGLS breaks down or does not converge within max_iter. */
int rfo_rational_estimate(rfo_ctx *ctx, double mu, int64_t n_poles, const double *poles,
                          const double *res_f, const double *res_g, const double *poly,
                          double tol, int64_t max_iter, double *NEF_out, double *density_out,
                          double *dFdH_out, int64_t *iterations_out);

/* CGLS iterations and solves (one per pole) since the context was created. */
int rfo_rational_stats(const rfo_ctx *ctx, int64_t *iterations, int64_t *solves);

/* Conjugate-gradient iterations and solves since the context was created. */
int rfo_cg_stats(const rfo_ctx *ctx, int64_t *iterations, int64_t *solves);

/* Moment doubling for calls without density output (see rfo_fermi_moments):
 * enabled != 0 turns it on (the default), 0 makes every moment a direct
 * r . y_k over p - 1 steps. */
int rfo_set_moment_doubling(rfo_ctx *ctx, int enabled);

/* Launch geometry and schedule of a context (for measurement; the defaults are the
 * measured best).  value = -1 restores the default.  Keys and accepted values:
 *   RFO_TUNE_PPL            probes per lane of the step kernels: 1, 2, 4
 *   RFO_TUNE_RPI            1x1: rows per wave iteration (1, 2, 7); 9x9: blocks per chunk (1, 2)
 *   RFO_TUNE_ROWS_PER_WG    block rows per scheduling unit of the step kernels (>= 1)
 *   RFO_TUNE_GRID           resident workgroups of the step kernels (>= 8, rounded to 8)
 *   RFO_TUNE_BF16_CHUNKS    BF16 steps: K chunks of 32 rows per iteration (1, 2)
 *   RFO_TUNE_SDDMM_PPL      probes per lane of the vector-unit outer products (1, 2)
 *   RFO_TUNE_SDDMM_MFMA     0 keeps the BF16 segment gradient on the vector units (it then
 *                           reads the FP32 vectors instead of their BF16 copies)
 *   RFO_TUNE_SDDMM_STEPS    steps per launch of the segment gradient on the vector units
 *                           (default 32; 0 = one launch per segment)
 *   RFO_TUNE_SDDMM_STEPS_BF16  the same for the matrix-core segment gradient (default 8)
 *   RFO_TUNE_OVERLAP        1: each segment's gradient of the doubled adjoint runs on a
 *                           second stream beside the next segment's steps (default 0; the
 *                           result is bitwise the serial one)
 *   RFO_TUNE_CPLX_PPL, RFO_TUNE_CPLX_ROWS, RFO_TUNE_CPLX_GRID  probes per lane (1, 2), rows
 *                           (1x1: 4, 8) or blocks (9x9: 1, 2) per chunk, and workgroups of
 *                           the complex shifted product of the rational estimate
 *   RFO_TUNE_ADJOINT_BYTES  memory budget (bytes) of rfo_energy_and_dEdH's vector slots
 *                           (default: 85% of the device memory free at the call plus what
 *                           the slots already hold); above it the probe columns run in
 *                           batches, each adding its sums to the gradient
 *   RFO_TUNE_ALT_SWEEP      1 (default): every other Chebyshev-step launch sweeps its rows
 *                           in the opposite order, so it first reads what the previous
 *                           launch touched last (0: always forward)
 *   RFO_TUNE_ADJOINT_TAIL   1: rfo_energy_and_dEdH with the doubled moments keeps, within the
 *                           memory budget above, the last vectors of its forward pass, so the
 *                           top checkpoint segments are not replayed (the same gradient, bitwise;
 *                           the context then holds up to the whole budget).  0 (default)
 * Geometry changes only the order of FP64 sums (rounding).  The segment gradient's step
 * groups, its matrix-core switch and the adjoint's probe batches change how G is summed
 * and so its rounding (and, for RFO_TUNE_SDDMM_MFMA = 0, which operands the BF16
 * gradient reads).
 * Errors: RFO_E_INVALID for an unknown key or a value out of range. */
typedef enum {
  RFO_TUNE_PPL = 0,
  RFO_TUNE_RPI = 1,
  RFO_TUNE_ROWS_PER_WG = 2,
  RFO_TUNE_GRID = 3,
  RFO_TUNE_BF16_CHUNKS = 4,
  RFO_TUNE_SDDMM_PPL = 5,
  RFO_TUNE_SDDMM_MFMA = 6,
  RFO_TUNE_SDDMM_STEPS = 7,
  RFO_TUNE_SDDMM_STEPS_BF16 = 8,
  RFO_TUNE_OVERLAP = 9,
  RFO_TUNE_CPLX_PPL = 10,
  RFO_TUNE_CPLX_ROWS = 11,
  RFO_TUNE_CPLX_GRID = 12,
  RFO_TUNE_ADJOINT_BYTES = 13,
  RFO_TUNE_ALT_SWEEP = 14,
  RFO_TUNE_ADJOINT_TAIL = 15,
  RFO_TUNE_COUNT = 16
} rfo_tuning;
int rfo_set_tuning(rfo_ctx *ctx, int key, int64_t value);

/* Instrumentation: when enabled, the library records HIP events around each
 * run of consecutive Chebyshev-step launches on its stream.  rfo_step_timing
 * returns the mean step-kernel time (ms) over the steps recorded since the
 * last reset, and their count. */
int rfo_set_timing(rfo_ctx *ctx, int enabled);
int rfo_step_timing(rfo_ctx *ctx, double *mean_ms, int64_t *n_steps);

#if defined(__GNUC__) || defined(__clang__)
#pragma GCC visibility pop
#endif

#ifdef __cplusplus
}
#endif

#endif /* RFO_H */
