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
// Schedule: the grid is one resident wave of G workgroups (G a multiple of 8).
// The work is U = n_pt * n_rg units (probe tile, group of rows_per_wg block
// rows), ordered tile-major.  XCD x (hardware workgroups b with b mod 8 = x)
// owns the contiguous units [U x/8, U (x+1)/8) and its G/8 workgroups sweep
// them together, unit lo + b/8 + i G/8 at sweep i.  The rows in flight on an
// XCD therefore form a narrow band that moves through the matrix, and the
// neighbour rows it gathers are still in that XCD's L2.
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

struct Sched {
  int64_t u, hi;
  int stride;
  __device__ Sched(int64_t U) {
    const int b = blockIdx.x, G = gridDim.x;
    const int x = b & 7;
    stride = G >> 3;
    const int64_t lo = U * x / 8;
    hi = U * (x + 1) / 8;
    u = lo + (b >> 3);
  }
};

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

template <int PPL>
__device__ __forceinline__ void zero_other_tiles(double *prow, int first, int last, int n_pt,
                                                 int wave, int lane) {
  if (wave != 0) return;
  for (int t = 0; t < n_pt; ++t) {
    if (t >= first && t <= last) continue;
#pragma unroll
    for (int q = 0; q < PPL; ++q) prow[t * (64 * PPL) + lane * PPL + q] = 0.0;
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// 1x1 blocks.  Gathers of U neighbours are issued together before their FMAs,
// for RPI rows at once, so each wave keeps RPI * U vector loads in flight; the
// streamed rows of y_{k-1} and the probe signs are requested before the
// gathers.  The column and value arrays carry kStepPad zero entries past nnzb,
// so a chunk may read past the end of the last row; entries past a row's end
// get zero weight.  NT selects non-temporal hints for the streamed arrays.
// ---------------------------------------------------------------------------
template <typename VT, typename MT, int PPL, int U, int RPI, bool NT>
__global__ __launch_bounds__(kWG) void k_step1(StepArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sp = a.sp;
  const int nw = sp >> 6;
  const VT *__restrict__ x = static_cast<const VT *>(a.x);
  const VT *prev = static_cast<const VT *>(a.prev);
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const MT *hval = static_cast<const MT *>(a.hval);
  const bool has_prev = a.c2 != 0.0;
  const bool add_r = a.beta != nullptr;
  const bool mom_on = a.part != nullptr;
  const bool need_r = add_r || mom_on;
  const double beta = add_r ? sld(a.beta) : 0.0;
  const int m = acc ? a.acc_terms : 0;
  VT al[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) al[i] = i < m ? (VT)sld(a.alpha + i) : (VT)0;
  const VT c1 = (VT)a.c1, c2 = (VT)a.c2;
  __shared__ double red[kWaves][64 * PPL];
  double *prow = mom_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;

  double mom[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = 0.0;
  int first_pt = -1, cur_pt = -1;

  for (Sched sc((int64_t)a.n_pt * a.n_rg); sc.u < sc.hi; sc.u += sc.stride) {
    const int pt = (int)(sc.u / a.n_rg);
    const int64_t rg = sc.u - (int64_t)pt * a.n_rg;
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
      if (first_pt < 0) first_pt = pt;
      cur_pt = pt;
    }
    const int c0 = pt * (64 * PPL) + lane * PPL;
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
      VecN<VT, PPL> pv[RPI], xs[RPI];
      uint64_t sw[RPI];
      VecN<double, PPL> rv[RPI];
#pragma unroll
      for (int r = 0; r < RPI; ++r) {
        const int64_t off = Ir[r] * sp + c0;
        if (has_prev) pv[r] = NT ? ldv_nt<VT, PPL>(prev + off) : ldv<VT, PPL>(prev + off);
        if (m >= 2) xs[r] = ldv<VT, PPL>(x + off);
        if (need_r) {
          if (a.sgn) sw[r] = a.sgn[Ir[r] * nw + (c0 >> 6)];
          else rv[r] = ldv<double, PPL>(a.rden + off);
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
            // slots past the row's end re-read the row's own vector (a cache hit)
            const int64_t Jc = sld(a.col + beg[r] + u);
            J[r][u] = beg[r] + u < end[r] ? Jc : Ir[r];
          }
#pragma unroll
        for (int r = 0; r < RPI; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) xv[r][u] = ldv<VT, PPL>(x + J[r][u] * sp + c0);
#pragma unroll
        for (int r = 0; r < RPI; ++r)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t nz = beg[r] + u;
            const VT h = nz < end[r] ? (VT)sld(hval + nz) : (VT)0;
#pragma unroll
            for (int q = 0; q < PPL; ++q) s[r][q] = fma(h, xv[r][u].v[q], s[r][q]);
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
          for (int u = 0; u < U; ++u) xv[u] = ldv<VT, PPL>(x + J[u] * sp + c0);
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int64_t nz = nz0 + u;
            const VT h = nz < end[r] ? (VT)sld(hval + nz) : (VT)0;
#pragma unroll
            for (int q = 0; q < PPL; ++q) s[r][q] = fma(h, xv[u].v[q], s[r][q]);
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
          o.v[q] = v;
          if (mom_on) mom[q] = fma(rq, (double)v, mom[q]);
        }
        if (NT) stv_nt<VT, PPL>(out + off, o);
        else stv<VT, PPL>(out + off, o);
        if (m > 0) {
          VecN<VT, PPL> av = NT ? ldv_nt<VT, PPL>(acc + off) : ldv<VT, PPL>(acc + off);
          av = add_terms<VT, PPL>(av, m, al, pv[r], xs[r], o);
          if (NT) stv_nt<VT, PPL>(acc + off, av);
          else stv<VT, PPL>(acc + off, av);
        }
      }
    }
  }
  if (mom_on) {
    if (cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
    zero_other_tiles<PPL>(prow, first_pt, cur_pt, a.n_pt, wave, lane);
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
template <typename VT, typename MT, int PPL, int U, bool NT>
__global__ __launch_bounds__(kWG) void k_step9(StepArgs a) {
  constexpr int BD = 9, BB = 81;
  constexpr int CH = U * BB;                       // H_hat values per chunk
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sp = a.sp;
  const int nw = sp >> 6;
  const VT *__restrict__ x = static_cast<const VT *>(a.x);
  const VT *prev = static_cast<const VT *>(a.prev);
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const MT *hval = static_cast<const MT *>(a.hval);
  const bool has_prev = a.c2 != 0.0;
  const bool add_r = a.beta != nullptr;
  const bool mom_on = a.part != nullptr;
  const bool need_r = add_r || mom_on;
  const double beta = add_r ? sld(a.beta) : 0.0;
  const int m = acc ? a.acc_terms : 0;
  VT al[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) al[i] = i < m ? (VT)sld(a.alpha + i) : (VT)0;
  const VT c1 = (VT)a.c1, c2 = (VT)a.c2;
  __shared__ double red[kWaves][64 * PPL];
  __shared__ MT hs[kWaves][CH];
  MT *hw = hs[wave];
  double *prow = mom_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;

  double mom[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = 0.0;
  int first_pt = -1, cur_pt = -1;

  for (Sched sc((int64_t)a.n_pt * a.n_rg); sc.u < sc.hi; sc.u += sc.stride) {
    const int pt = (int)(sc.u / a.n_rg);
    const int64_t rg = sc.u - (int64_t)pt * a.n_rg;
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
      if (first_pt < 0) first_pt = pt;
      cur_pt = pt;
    }
    const int c0 = pt * (64 * PPL) + lane * PPL;
    const int64_t r0 = rg * a.rows_per_wg;
    const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
    for (int64_t I = r0 + wave; I < r1; I += kWaves) {
      const int64_t beg = sld(a.row_ptr + I), end = sld(a.row_ptr + I + 1);
      VT s[BD][PPL];
#pragma unroll
      for (int i = 0; i < BD; ++i)
#pragma unroll
        for (int q = 0; q < PPL; ++q) s[i][q] = (VT)0;
      for (int64_t nz = beg; nz < end; nz += U) {
        // H_hat chunk -> registers (coalesced), neighbour gathers, then LDS
        MT hv[(CH + 63) / 64];
        const MT *hsrc = hval + nz * BB;
#pragma unroll
        for (int k = 0; k < (CH + 63) / 64; ++k) {
          const int e = k * 64 + lane;
          if (e < CH) hv[k] = hsrc[e];
        }
        int64_t J[U];
#pragma unroll
        for (int u = 0; u < U; ++u) J[u] = sld(a.col + nz + u);
        VecN<VT, PPL> xv[U][BD];
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
          for (int j = 0; j < BD; ++j) xv[u][j] = ldv<VT, PPL>(x + (J[u] * BD + j) * sp + c0);
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int k = 0; k < (CH + 63) / 64; ++k) {
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
      }
#pragma unroll
      for (int i = 0; i < BD; ++i) {
        const int64_t row = I * BD + i;
        const int64_t off = row * sp + c0;
        VecN<VT, PPL> pv, xs;
        if (has_prev) pv = NT ? ldv_nt<VT, PPL>(prev + off) : ldv<VT, PPL>(prev + off);
        if (m >= 2) xs = ldv<VT, PPL>(x + off);
        double r[PPL];
        if (need_r) {
          if (a.sgn) {
            const uint64_t w = a.sgn[row * nw + (c0 >> 6)];
#pragma unroll
            for (int q = 0; q < PPL; ++q) r[q] = ((w >> ((c0 + q) & 63)) & 1ull) ? 1.0 : -1.0;
          } else {
            const VecN<double, PPL> rv = ldv<double, PPL>(a.rden + off);
#pragma unroll
            for (int q = 0; q < PPL; ++q) r[q] = rv.v[q];
          }
        }
        VecN<VT, PPL> o;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          VT v = c1 * s[i][q];
          if (has_prev) v = fma(c2, pv.v[q], v);
          if (add_r) v = (VT)((double)v + beta * r[q]);
          o.v[q] = v;
          if (mom_on) mom[q] = fma(r[q], (double)v, mom[q]);
        }
        if (NT) stv_nt<VT, PPL>(out + off, o);
        else stv<VT, PPL>(out + off, o);
        if (m > 0) {
          VecN<VT, PPL> av = NT ? ldv_nt<VT, PPL>(acc + off) : ldv<VT, PPL>(acc + off);
          av = add_terms<VT, PPL>(av, m, al, pv, xs, o);
          if (NT) stv_nt<VT, PPL>(acc + off, av);
          else stv<VT, PPL>(acc + off, av);
        }
      }
    }
  }
  if (mom_on) {
    if (cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
    zero_other_tiles<PPL>(prow, first_pt, cur_pt, a.n_pt, wave, lane);
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
  int first_pt = -1, cur_pt = -1;
  for (Sched sc((int64_t)a.n_pt * a.n_rg); sc.u < sc.hi; sc.u += sc.stride) {
    const int pt = (int)(sc.u / a.n_rg);
    const int64_t rg = sc.u - (int64_t)pt * a.n_rg;
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
      if (first_pt < 0) first_pt = pt;
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
      }
    }
  }
  if (mom_on) {
    if (cur_pt >= 0) flush_tile<PPL>(mom, red, wave, lane, prow, cur_pt);
    zero_other_tiles<PPL>(prow, first_pt, cur_pt, a.n_pt, wave, lane);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <typename VT, typename MT, int PPL>
const void *step_fn(int bd, int rpi, int nt) {
  if (bd == 1) {
    if (rpi == 2)
      return nt ? (const void *)k_step1<VT, MT, PPL, 8, 2, true>
                : (const void *)k_step1<VT, MT, PPL, 8, 2, false>;
    return nt ? (const void *)k_step1<VT, MT, PPL, 8, 1, true>
              : (const void *)k_step1<VT, MT, PPL, 8, 1, false>;
  }
  if (rpi == 1)
    return nt ? (const void *)k_step9<VT, MT, PPL, 1, true> : (const void *)k_step9<VT, MT, PPL, 1, false>;
  return nt ? (const void *)k_step9<VT, MT, PPL, 2, true> : (const void *)k_step9<VT, MT, PPL, 2, false>;
}

template <typename VT, typename MT>
const void *step_fn_t(int bd, int ppl, int rpi, int nt) {
  switch (ppl) {
    case 1: return step_fn<VT, MT, 1>(bd, rpi, nt);
    case 2: return step_fn<VT, MT, 2>(bd, rpi, nt);
    case 4: return step_fn<VT, MT, 4>(bd, rpi, nt);
    default: return nullptr;
  }
}

const void *select_step(int bd, int precision, int ppl, int rpi, int nt) {
  if (bd != 1 && bd != 9) return nullptr;
  return precision == 0 ? step_fn_t<double, double>(bd, ppl, rpi, nt)
                        : step_fn_t<float, float>(bd, ppl, rpi, nt);
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

int step_blocks_per_cu(int bd, int precision, int ppl, int rpi, int nt) {
  const void *f = select_step(bd, precision, ppl, rpi, nt);
  if (!f) return 0;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, f, kWG, 0) != hipSuccess) return 0;
  return nblk;
}

hipError_t launch_step(int bd, int precision, int ppl, const StepArgs &a, hipStream_t s) {
  const void *f = select_step(bd, precision, ppl, a.rpi, a.nt);
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
