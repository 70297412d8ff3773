// Chebyshev step kernels: one fused pass per term of the three-term recurrence
//   y_{k+1} = 2 H_hat y_k - y_{k-1}   (y_1 = H_hat y_0)
// with the moment partials r_c . y_{k+1} and the density accumulator
// acc = sum_k alpha_k y_k folded into the same pass (paper: Polynomial
// approximation, Chebyshev recursion with S = I; Random approximation).  A pass
// holds y_{k-1}, y_k and y_{k+1}, so the accumulator is updated on every third
// pass only, with three terms at once.
// The reverse recurrence of the free-energy gradient uses the same kernel with
// an added beta_j r term.
//
// Mapping: lanes run along probes (64*PPL probes per wave, PPL consecutive per
// lane), waves along block rows.  Block indices and H_hat entries are
// wave-uniform and come through the scalar cache; each neighbour's vector rows
// are read as whole coalesced segments.
//
// Schedule: the grid is one resident wave of G workgroups (G a multiple of 8)
// sweeping n_pt * n_rg units (probe tile, group of rows_per_wg block rows) in
// XCD-aware bands (Sched in device_util.h).
//
// Moment partials: workgroup b owns row b of a [G][sp] array.  Its units visit
// the probe tiles in increasing order; when it leaves a tile it sums its four
// waves' partials for that tile (fixed order) and stores them; tiles it never
// visits get zeros.  The reduction over b runs in a separate kernel in a fixed
// order, so moments are bitwise reproducible.
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

namespace {

template <int PPL>
__device__ __forceinline__ void flush_tile(double (&mom)[PPL], double (*red)[64 * PPL], int wave,
                                           int lane, double *prow, int pt) {
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    red[wave][lane * PPL + q] = mom[q];
    mom[q] = 0.0;
  }
  __syncthreads();
  if (wave == 0) {
#pragma unroll
    for (int q = 0; q < PPL; ++q) {
      double t = red[0][lane * PPL + q];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) t += red[w][lane * PPL + q];
      prow[pt * (64 * PPL) + lane * PPL + q] = t;
    }
  }
  __syncthreads();
}

// Zero this workgroup's partial row for every tile before the sweep: the tiles
// it never meets (with a stride above the units per tile it may skip some)
// must read as zero, and those it meets are overwritten by flush_tile.
template <int PPL>
__device__ __forceinline__ void zero_partials(double *prow, int n_pt, int wave, int lane) {
  if (wave != 0) return;
  for (int t = 0; t < n_pt; ++t)
#pragma unroll
    for (int q = 0; q < PPL; ++q) prow[t * (64 * PPL) + lane * PPL + q] = 0.0;
}

}  // namespace

// ---------------------------------------------------------------------------
// 1x1 blocks.  Gathers of U neighbours are issued together before their FMAs,
// for RPI rows at once, so each wave keeps RPI * U vector loads in flight; the
// streamed rows of y_{k-1} and the probe signs are requested before the
// gathers.  The column and value arrays carry kStepPad zero entries past nnzb,
// so a chunk may read indices past the end of the last row; slots past a row's
// end load nothing and get zero weight (U = 7 fits a 7-point stencil row in one
// chunk).  NT selects non-temporal hints for the streamed arrays.
// ---------------------------------------------------------------------------
template <typename VT, typename MT, int PPL, int U, int RPI, bool NT, int MODE, bool PAD>
__global__ __launch_bounds__(kWG) void k_step1(StepArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sp = a.sp;
  const int nw = sp >> 6;
  const int s_live = a.s_live > 0 ? a.s_live : sp;
  const VT *__restrict__ x = static_cast<const VT *>(a.x);
  const VT *prev = static_cast<const VT *>(a.prev);
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const MT *hval = static_cast<const MT *>(a.hval);
  const bool has_prev = a.c2 != 0.0;
  const bool add_r = a.beta != nullptr;
  const bool mom_on = a.part != nullptr;
  // MODE 1: density accumulator terms; MODE 2: doubling moments <y,y>, <y,y_k>
  // instead of r.y (the MODE 0 variants carry no code for either)
  constexpr bool DBL = MODE == 2;
  const bool need_r = add_r || (mom_on && !DBL);
  const double beta = add_r ? sld(a.beta) : 0.0;
  const int m = MODE == 1 ? a.acc_terms : 0;
  // MODE 3: vector sources added to the output (reverse recurrence with doubling)
  constexpr bool SRC = MODE == 3;
  const int nsrc = SRC ? a.nsrc : 0;
  const VT *srcp[3];
  VT srw[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    srcp[t] = t < nsrc ? static_cast<const VT *>(a.src[t]) : nullptr;
    srw[t] = t < nsrc ? (VT)a.srcw[t] : (VT)0;
  }
  VT al[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) al[i] = i < m ? (VT)sld(a.alpha + i) : (VT)0;
  const VT c1 = (VT)a.c1, c2 = (VT)a.c2;
  __shared__ double red[kWaves][64 * PPL];
  double *prow = mom_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;

  double mom[PPL], mom2[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = mom2[q] = 0.0;
  int cur_pt = -1;
  double *prow2 = DBL && mom_on ? a.part2 + (int64_t)blockIdx.x * sp : nullptr;
  if (mom_on) zero_partials<PPL>(prow, a.n_pt, wave, lane);
  if (DBL && mom_on) zero_partials<PPL>(prow2, a.n_pt, wave, lane);

  for (Sched sc(a.n_pt, a.n_rg, a.reverse != 0); sc.more(); sc.next()) {
    const int pt = sc.pt();
    const int64_t rg = sc.rg();
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) {
        flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
        if (DBL) flush_tile<PPL>(mom2, red, wave, lane, prow2, cur_pt);
      }
      cur_pt = pt;
    }
    const int c0 = pt * (64 * PPL) + lane * PPL;
    // PAD: a lane whose probes are all zero padding loads nothing (its inputs are
    // zero); without padding columns the predicate is compiled out
    const bool live = !PAD || c0 < s_live;
    const int64_t r0 = rg * a.rows_per_wg;
    const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
    for (int64_t I0 = r0 + wave * RPI; I0 < r1; I0 += kWaves * RPI) {
      int64_t Ir[RPI], beg[RPI], end[RPI];
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        Ir[r] = min(I0 + r, r1 - 1);  // a clamped row is computed but not stored
        beg[r] = sld(a.row_ptr + Ir[r]);
        end[r] = sld(a.row_ptr + Ir[r] + 1);
      }
      VecN<VT, PPL> pv[RPI], xs[RPI], sv[3][RPI];
      uint64_t sw[RPI];
      VecN<double, PPL> rv[RPI];
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        const int64_t off = Ir[r] * sp + c0;
        if (has_prev)
          pv[r] = !live ? zerov<VT, PPL>() : NT ? ldv_nt<VT, PPL>(prev + off) : ldv<VT, PPL>(prev + off);
        if (SRC) {
#pragma unroll
          for (int t = 0; t < 3; ++t)
            if (t < nsrc) sv[t][r] = live ? ldv_nt<VT, PPL>(srcp[t] + off) : zerov<VT, PPL>();
        }
        if (need_r) {
          if (a.sgn) sw[r] = a.sgn[Ir[r] * nw + (c0 >> 6)];
          else rv[r] = live ? ldv<double, PPL>(a.rden + off) : zerov<double, PPL>();
        }
      }
      VT s[RPI][PPL];
#pragma unroll
      for (int r = 0; r < RPI; ++r)
#pragma unroll
        for (int q = 0; q < PPL; ++q) s[r][q] = (VT)0;
      {
        int64_t J[RPI][U];
        VecN<VT, PPL> xv[RPI][U];
#pragma unroll
        for (int r = 0; r < RPI; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            // slots past the row's end issue no load (the L2 request rate is the
            // step's limit) and get zero weight
            const int64_t Jc = sld(a.col + beg[r] + u);
            J[r][u] = beg[r] + u < end[r] ? Jc : Ir[r];
          }
#pragma unroll
        for (int r = 0; r < RPI; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (beg[r] + u < end[r] && live) xv[r][u] = ldv<VT, PPL>(x + J[r][u] * sp + c0);
            else {
#pragma unroll
              for (int q = 0; q < PPL; ++q) xv[r][u].v[q] = (VT)0;
            }
          }
#pragma unroll
        for (int r = 0; r < RPI; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t nz = beg[r] + u;
            const VT h = nz < end[r] ? (VT)sld(hval + nz) : (VT)0;
#pragma unroll
            for (int q = 0; q < PPL; ++q) s[r][q] = fma(h, xv[r][u].v[q], s[r][q]);
            // y_k of the row itself for the accumulator: every row stores its
            // diagonal, so one of the gathered rows is it
            if ((m >= 2 || DBL) && nz < end[r] && J[r][u] == Ir[r]) xs[r] = xv[r][u];
          }
      }
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        for (int64_t nz0 = beg[r] + U; nz0 < end[r]; nz0 += U) {
          int64_t J[U];
          VecN<VT, PPL> xv[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t Jc = sld(a.col + nz0 + u);
            J[u] = nz0 + u < end[r] ? Jc : Ir[r];
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            if (nz0 + u < end[r] && live) xv[u] = ldv<VT, PPL>(x + J[u] * sp + c0);
            else {
#pragma unroll
              for (int q = 0; q < PPL; ++q) xv[u].v[q] = (VT)0;
            }
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t nz = nz0 + u;
            const VT h = nz < end[r] ? (VT)sld(hval + nz) : (VT)0;
#pragma unroll
            for (int q = 0; q < PPL; ++q) s[r][q] = fma(h, xv[u].v[q], s[r][q]);
            if ((m >= 2 || DBL) && nz < end[r] && J[u] == Ir[r]) xs[r] = xv[u];
          }
        }
      }
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        if (I0 + r >= r1) continue;
        const int64_t off = Ir[r] * sp + c0;
        VecN<VT, PPL> o;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          double rq = 0.0;
          if (need_r) rq = a.sgn ? (((sw[r] >> ((c0 + q) & 63)) & 1ull) ? 1.0 : -1.0) : rv[r].v[q];
          VT v = c1 * s[r][q];
          if (has_prev) v = fma(c2, pv[r].v[q], v);
          if (add_r) v = (VT)((double)v + beta * rq);
          if (SRC) {
#pragma unroll
            for (int t = 0; t < 3; ++t)
              if (t < nsrc) v = fma(srw[t], sv[t][r].v[q], v);
          }
          o.v[q] = v;
          if (mom_on) {
            if (DBL) {
              mom[q] = fma((double)v, (double)v, mom[q]);
              mom2[q] = fma((double)v, (double)xs[r].v[q], mom2[q]);
            } else {
              mom[q] = fma(rq, (double)v, mom[q]);
            }
          }
        }
        if (NT) stv_nt<VT, PPL>(out + off, o);
        else stv<VT, PPL>(out + off, o);
        if (m > 0) {
          VecN<VT, PPL> av = !live ? zerov<VT, PPL>() : NT ? ldv_nt<VT, PPL>(acc + off) : ldv<VT, PPL>(acc + off);
          av = add_terms<VT, PPL>(av, m, al, pv[r], xs[r], o);
          if (NT) stv_nt<VT, PPL>(acc + off, av);
          else stv<VT, PPL>(acc + off, av);
        }
      }
    }
  }
  if (mom_on && cur_pt >= 0) {
    flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
    if (DBL) flush_tile<PPL>(mom2, red, wave, lane, prow2, cur_pt);
  }
}

// ---------------------------------------------------------------------------
// 9x9 blocks.  Each wave takes one block row at a time.  Per chunk of U blocks
// it loads the U H_hat blocks (U * 81 values, contiguous) with coalesced vector
// loads into its own LDS slice and issues the U * 9 neighbour-row gathers; the
// 81 * U * PPL FMAs then read the H_hat entries back as LDS broadcasts.  (Going
// through the scalar cache instead serializes: sixteen waves per CU on
// different block rows overflow it.)
// ---------------------------------------------------------------------------
template <typename VT, typename MT, int PPL, int U, bool NT, int MODE, bool PAD>
__global__ __launch_bounds__(kWG) void k_step9(StepArgs a) {
  constexpr int BD = 9, BB = 81;
  constexpr int CH = U * BB;                       // H_hat values per chunk
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sp = a.sp;
  const int nw = sp >> 6;
  const int s_live = a.s_live > 0 ? a.s_live : sp;
  const VT *__restrict__ x = static_cast<const VT *>(a.x);
  const VT *prev = static_cast<const VT *>(a.prev);
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const MT *hval = static_cast<const MT *>(a.hval);
  const bool has_prev = a.c2 != 0.0;
  const bool add_r = a.beta != nullptr;
  const bool mom_on = a.part != nullptr;
  // MODE 1: density accumulator terms; MODE 2: doubling moments <y,y>, <y,y_k>
  // instead of r.y (the MODE 0 variants carry no code for either)
  constexpr bool DBL = MODE == 2;
  const bool need_r = add_r || (mom_on && !DBL);
  const double beta = add_r ? sld(a.beta) : 0.0;
  const int m = MODE == 1 ? a.acc_terms : 0;
  // MODE 3: vector sources added to the output (reverse recurrence with doubling)
  constexpr bool SRC = MODE == 3;
  const int nsrc = SRC ? a.nsrc : 0;
  const VT *srcp[3];
  VT srw[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    srcp[t] = t < nsrc ? static_cast<const VT *>(a.src[t]) : nullptr;
    srw[t] = t < nsrc ? (VT)a.srcw[t] : (VT)0;
  }
  VT al[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) al[i] = i < m ? (VT)sld(a.alpha + i) : (VT)0;
  const VT c1 = (VT)a.c1, c2 = (VT)a.c2;
  __shared__ double red[kWaves][64 * PPL];
  __shared__ MT hs[kWaves][CH];
  MT *hw = hs[wave];
  double *prow = mom_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;

  double mom[PPL], mom2[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = mom2[q] = 0.0;
  int cur_pt = -1;
  double *prow2 = DBL && mom_on ? a.part2 + (int64_t)blockIdx.x * sp : nullptr;
  if (mom_on) zero_partials<PPL>(prow, a.n_pt, wave, lane);
  if (DBL && mom_on) zero_partials<PPL>(prow2, a.n_pt, wave, lane);

  for (Sched sc(a.n_pt, a.n_rg, a.reverse != 0); sc.more(); sc.next()) {
    const int pt = sc.pt();
    const int64_t rg = sc.rg();
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) {
        flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
        if (DBL) flush_tile<PPL>(mom2, red, wave, lane, prow2, cur_pt);
      }
      cur_pt = pt;
    }
    const int c0 = pt * (64 * PPL) + lane * PPL;
    // PAD: a lane whose probes are all zero padding loads nothing (its inputs are
    // zero); without padding columns the predicate is compiled out
    const bool live = !PAD || c0 < s_live;
    const int64_t r0 = rg * a.rows_per_wg;
    const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
    // one scalar row of the output: shift, sources, moments, store, accumulator
    auto finish_row = [&](int64_t I, int i, const VT(&si)[PPL]) {
        const int64_t row = I * BD + i;
        const int64_t off = row * sp + c0;
        VecN<VT, PPL> pv, xs;
        if (has_prev)
          pv = !live ? zerov<VT, PPL>() : NT ? ldv_nt<VT, PPL>(prev + off) : ldv<VT, PPL>(prev + off);
        VecN<VT, PPL> sv[3];
        if (SRC) {
#pragma unroll
          for (int t = 0; t < 3; ++t)
            if (t < nsrc) sv[t] = live ? ldv_nt<VT, PPL>(srcp[t] + off) : zerov<VT, PPL>();
        }
        if (m >= 2 || DBL) xs = live ? ldv<VT, PPL>(x + off) : zerov<VT, PPL>();
        double r[PPL];
        if (need_r) {
          if (a.sgn) {
            const uint64_t w = a.sgn[row * nw + (c0 >> 6)];
#pragma unroll
            for (int q = 0; q < PPL; ++q) r[q] = ((w >> ((c0 + q) & 63)) & 1ull) ? 1.0 : -1.0;
          } else {
            const VecN<double, PPL> rv = live ? ldv<double, PPL>(a.rden + off) : zerov<double, PPL>();
#pragma unroll
            for (int q = 0; q < PPL; ++q) r[q] = rv.v[q];
          }
        }
        VecN<VT, PPL> o;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          VT v = c1 * si[q];
          if (has_prev) v = fma(c2, pv.v[q], v);
          if (add_r) v = (VT)((double)v + beta * r[q]);
          if (SRC) {
#pragma unroll
            for (int t = 0; t < 3; ++t)
              if (t < nsrc) v = fma(srw[t], sv[t].v[q], v);
          }
          o.v[q] = v;
          if (mom_on) {
            if (DBL) {
              mom[q] = fma((double)v, (double)v, mom[q]);
              mom2[q] = fma((double)v, (double)xs.v[q], mom2[q]);
            } else {
              mom[q] = fma(r[q], (double)v, mom[q]);
            }
          }
        }
        if (NT) stv_nt<VT, PPL>(out + off, o);
        else stv<VT, PPL>(out + off, o);
        if (m > 0) {
          VecN<VT, PPL> av = !live ? zerov<VT, PPL>() : NT ? ldv_nt<VT, PPL>(acc + off) : ldv<VT, PPL>(acc + off);
          av = add_terms<VT, PPL>(av, m, al, pv, xs, o);
          if (NT) stv_nt<VT, PPL>(acc + off, av);
          else stv<VT, PPL>(acc + off, av);
        }
    };
    for (int64_t I = r0 + wave; I < r1; I += kWaves) {
      const int64_t beg = sld(a.row_ptr + I), end = sld(a.row_ptr + I + 1);
      VT s[BD][PPL];
#pragma unroll
      for (int i = 0; i < BD; ++i)
#pragma unroll
        for (int q = 0; q < PPL; ++q) s[i][q] = (VT)0;
      constexpr int NH = (CH + 63) / 64;
      // H_hat chunk -> registers (coalesced) and the neighbour gathers
      auto load_chunk = [&](int64_t nz, MT(&hv)[NH], VecN<VT, PPL>(&xv)[U][BD]) {
        const MT *hsrc = hval + nz * BB;
#pragma unroll
        for (int k = 0; k < NH; ++k) {
          const int e = k * 64 + lane;
          if (e < CH) hv[k] = hsrc[e];
        }
        int64_t J[U];
#pragma unroll
        for (int u = 0; u < U; ++u) J[u] = sld(a.col + nz + u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          // a chunk slot past the row's end gathers nothing (its FMAs are skipped)
          if (u == 0 || nz + u < end) {
#pragma unroll
            for (int j = 0; j < BD; ++j)
              xv[u][j] = live ? ldv<VT, PPL>(x + (J[u] * BD + j) * sp + c0) : zerov<VT, PPL>();
          }
        }
      };
      // H_hat chunk -> LDS, then the FMAs with LDS broadcasts
      auto use_chunk = [&](int64_t nz, const MT(&hv)[NH], const VecN<VT, PPL>(&xv)[U][BD]) {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < NH; ++k) {
          const int e = k * 64 + lane;
          if (e < CH) hw[e] = hv[k];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (nz + u < end) {
#pragma unroll
            for (int i = 0; i < BD; ++i)
#pragma unroll
              for (int j = 0; j < BD; ++j) {
                const VT h = (VT)hw[u * BB + i * BD + j];
#pragma unroll
                for (int q = 0; q < PPL; ++q) s[i][q] = fma(h, xv[u][j].v[q], s[i][q]);
              }
          }
        }
      };
      for (int64_t nz = beg; nz < end; nz += U) {
        MT hv[NH];
        VecN<VT, PPL> xv[U][BD];
        load_chunk(nz, hv, xv);
        use_chunk(nz, hv, xv);
      }
#pragma unroll
      for (int i = 0; i < BD; ++i) finish_row(I, i, s[i]);
    }
  }
  if (mom_on && cur_pt >= 0) {
    flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
    if (DBL) flush_tile<PPL>(mom2, red, wave, lane, prow2, cur_pt);
  }
}

// ---------------------------------------------------------------------------
// y = scale * r, optional acc = alpha * y and moment partials r . y, with the
// step kernels' schedule so that the partials line up.
// ---------------------------------------------------------------------------
template <typename VT, int PPL>
__global__ __launch_bounds__(kWG) void k_init(InitArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sp = a.sp;
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const double scale = a.scale ? sld(a.scale) : 1.0;
  const double alpha = acc ? sld(a.alpha) : 0.0;
  const bool mom_on = a.part != nullptr;
  __shared__ double red[kWaves][64 * PPL];
  double *prow = mom_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;
  double mom[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = 0.0;
  int cur_pt = -1;
  if (mom_on) zero_partials<PPL>(prow, a.n_pt, wave, lane);
  for (Sched sc(a.n_pt, a.n_rg); sc.more(); sc.next()) {
    const int pt = sc.pt();
    const int64_t rg = sc.rg();
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
      cur_pt = pt;
    }
    const int c0 = pt * (64 * PPL) + lane * PPL;
    const int64_t r0 = rg * a.rows_per_wg;
    const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
    for (int64_t I = r0 + wave; I < r1; I += kWaves) {
      for (int i = 0; i < a.bd; ++i) {
        const int64_t row = I * a.bd + i;
        const int64_t off = row * sp + c0;
        VecN<VT, PPL> o, av;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          const double r = probe_value(a.sgn, a.rden, row, sp, c0 + q);
          o.v[q] = (VT)(scale * r);
          av.v[q] = (VT)(alpha * (double)o.v[q]);
          mom[q] = fma(r, (double)o.v[q], mom[q]);
        }
        stv<VT, PPL>(out + off, o);
        if (acc) stv<VT, PPL>(acc + off, av);
        if constexpr (sizeof(VT) == 4) {
          if (a.outb) {
            VecN<unsigned short, PPL> ob;
#pragma unroll
            for (int q = 0; q < PPL; ++q) ob.v[q] = bf16_bits((float)o.v[q]);
            stv<unsigned short, PPL>(static_cast<unsigned short *>(a.outb) + off, ob);
          }
        }
      }
    }
  }
  if (mom_on) {
    if (cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <typename VT, typename MT, int PPL, int MODE, bool PAD>
const void *step_fn(int bd, int rpi) {
  // 1x1: rpi = rows per wave iteration with 8 neighbours per chunk, or 7: one
  // row per iteration with 7 neighbours per chunk; 9x9: rpi = blocks per chunk
  if (bd == 1) {
    if (rpi == 7) return (const void *)k_step1<VT, MT, PPL, 7, 1, true, MODE, PAD>;
    return rpi == 2 ? (const void *)k_step1<VT, MT, PPL, 8, 2, true, MODE, PAD>
                    : (const void *)k_step1<VT, MT, PPL, 8, 1, true, MODE, PAD>;
  }
  return rpi == 2 ? (const void *)k_step9<VT, MT, PPL, 2, true, MODE, PAD>
                  : (const void *)k_step9<VT, MT, PPL, 1, true, MODE, PAD>;
}

template <typename VT, typename MT, int MODE, bool PAD>
const void *step_fn_t(int bd, int ppl, int rpi) {
  switch (ppl) {
    case 1: return step_fn<VT, MT, 1, MODE, PAD>(bd, rpi);
    case 2: return step_fn<VT, MT, 2, MODE, PAD>(bd, rpi);
    case 4: return step_fn<VT, MT, 4, MODE, PAD>(bd, rpi);
    default: return nullptr;
  }
}

template <typename VT, typename MT, bool PAD>
const void *step_fn_m(int bd, int ppl, int rpi, int mode) {
  switch (mode) {
    case 0: return step_fn_t<VT, MT, 0, PAD>(bd, ppl, rpi);
    case 1: return step_fn_t<VT, MT, 1, PAD>(bd, ppl, rpi);
    case 2: return step_fn_t<VT, MT, 2, PAD>(bd, ppl, rpi);
    case 3: return step_fn_t<VT, MT, 3, PAD>(bd, ppl, rpi);
    default: return nullptr;
  }
}

// mode: 0 plain, 1 density accumulator, 2 doubling moments, 3 vector sources;
// pad: some probe columns are zero padding (StepArgs::s_live)
const void *select_step(int bd, int precision, int ppl, int rpi, int mode, bool pad) {
  if ((bd != 1 && bd != 9) || rpi < 1 || (rpi > 2 && !(bd == 1 && rpi == 7))) return nullptr;
  if (pad)
    return precision == 0 ? step_fn_m<double, double, true>(bd, ppl, rpi, mode)
                          : step_fn_m<float, float, true>(bd, ppl, rpi, mode);
  return precision == 0 ? step_fn_m<double, double, false>(bd, ppl, rpi, mode)
                        : step_fn_m<float, float, false>(bd, ppl, rpi, mode);
}

const void *select_init(int precision, int ppl) {
  if (precision == 0) {
    switch (ppl) {
      case 1: return (const void *)k_init<double, 1>;
      case 2: return (const void *)k_init<double, 2>;
      case 4: return (const void *)k_init<double, 4>;
    }
  } else {
    switch (ppl) {
      case 1: return (const void *)k_init<float, 1>;
      case 2: return (const void *)k_init<float, 2>;
      case 4: return (const void *)k_init<float, 4>;
    }
  }
  return nullptr;
}

}  // namespace

int step_blocks_per_cu(int bd, int precision, int ppl, int rpi) {
  const void *f = select_step(bd, precision, ppl, rpi, 0, false);
  if (!f) return 0;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, f, kWG, 0) != hipSuccess) return 0;
  return nblk;
}

hipError_t launch_step(int bd, int precision, int ppl, const StepArgs &a, hipStream_t s) {
  const void *f = select_step(bd, precision, ppl, a.rpi, step_mode(a), a.s_live > 0 && a.s_live < a.sp);
  if (!f || a.grid < 8 || (a.grid & 7)) return hipErrorInvalidValue;
  void *args[] = {const_cast<StepArgs *>(&a)};
  return hipLaunchKernel(f, dim3((unsigned)a.grid), dim3(kWG), args, 0, s);
}

hipError_t launch_init(int precision, const InitArgs &a, hipStream_t s) {
  const void *f = select_init(precision, a.ppl);
  if (!f || a.grid < 8 || (a.grid & 7)) return hipErrorInvalidValue;
  void *args[] = {const_cast<InitArgs *>(&a)};
  return hipLaunchKernel(f, dim3((unsigned)a.grid), dim3(kWG), args, 0, s);
}

}  // namespace rfo
