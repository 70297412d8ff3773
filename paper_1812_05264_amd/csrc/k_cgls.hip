// Rational expansion (paper: Rational approximation, Eq. rational_PQ with S = I):
// the shifted systems (H_hat - z) x = y for every probe column, solved by CGLS
// (conjugate gradients on the normal equations, the solver the paper applies to
// the indefinite complex-shifted matrices), and the per-pole accumulations.
//
// Complex block vectors are two real planes, re then im, each [n][sp] like the
// Chebyshev vectors, so the real H_hat multiplies both planes with the same
// gathers and block values.  Column sums (norms, inner products with the
// probes) are written as per-workgroup partials and reduced in a fixed order
// (launch_colreduce, or k_cgls_reduce with the CGLS scalars), so every scalar is
// bitwise reproducible.
#include "colsum.h"
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

namespace {

template <int PPL>
__device__ __forceinline__ void flush_norm(double (&nrm)[PPL], double (*red)[64 * PPL], int wave,
                                           int lane, double *prow, int pt) {
#pragma unroll
  for (int q = 0; q < PPL; ++q) {
    red[wave][lane * PPL + q] = nrm[q];
    nrm[q] = 0.0;
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

}  // namespace

// out = (H_hat - z) x on complex planes, with the column partials of |out_c|^2;
// HS: out = H_hat x - z (S x) with the overlap S on the same pattern (H_hat then
// maps H with S).  Same persistent XCD-banded schedule as the Chebyshev step
// (Sched).  1x1 blocks: U neighbours per chunk, entries through the scalar cache;
// 9x9 blocks: U blocks per chunk, their entries staged in the wave's LDS slice.
template <int BD, int PPL, int U, bool HS>
__global__ __launch_bounds__(kWG) void k_cspmm(CspArgs a) {
  constexpr int BB = BD * BD;
  constexpr int NM = HS ? 2 : 1;  // matrices applied to x: H_hat (and S)
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int sp = a.sp;
  const double *__restrict__ xr = a.x;
  const double *__restrict__ xi = a.x + a.plane;
  double *orr = a.out;
  double *oi = a.out + a.plane;
  const double zr = a.zr, zi = a.zi;
  const bool nrm_on = a.part != nullptr;
  __shared__ double red[kWaves][64 * PPL];
  __shared__ double hs[BD == 1 ? 1 : kWaves][BD == 1 ? 1 : NM * U * BB];
  double *prow = nrm_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;
  if (nrm_on && wave == 0)
    for (int t = 0; t < a.n_pt; ++t)
#pragma unroll
      for (int q = 0; q < PPL; ++q) prow[t * (64 * PPL) + lane * PPL + q] = 0.0;
  double nrm[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) nrm[q] = 0.0;
  int cur_pt = -1;

  for (Sched sc(a.n_pt, a.n_rg); sc.more(); sc.next()) {
    const int pt = sc.pt();
    const int64_t rg = sc.rg();
    if (pt != cur_pt) {
      if (nrm_on && cur_pt >= 0) flush_norm<PPL>(nrm, red, wave, lane, prow, cur_pt);
      cur_pt = pt;
    }
    const int c0 = pt * (64 * PPL) + lane * PPL;
    const int64_t r0 = rg * a.rows_per_wg;
    const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
    for (int64_t I = r0 + wave; I < r1; I += kWaves) {
      const int64_t beg = sld(a.row_ptr + I), end = sld(a.row_ptr + I + 1);
      double sr[BD][PPL], si[BD][PPL];        // H_hat x
      double tr[HS ? BD : 1][PPL], ti[HS ? BD : 1][PPL];  // S x
#pragma unroll
      for (int i = 0; i < BD; ++i)
#pragma unroll
        for (int q = 0; q < PPL; ++q) sr[i][q] = si[i][q] = 0.0;
#pragma unroll
      for (int i = 0; i < (HS ? BD : 1); ++i)
#pragma unroll
        for (int q = 0; q < PPL; ++q) tr[i][q] = ti[i][q] = 0.0;
      if constexpr (BD == 1) {
        for (int64_t nz0 = beg; nz0 < end; nz0 += U) {
          int64_t J[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            // slots past the row's end re-read the row itself with weight zero
            const int64_t Jc = sld(a.col + nz0 + u);
            J[u] = nz0 + u < end ? Jc : I;
          }
          VecN<double, PPL> vr[U], vi[U];
#pragma unroll
          for (int u = 0; u < U; ++u) {
            vr[u] = ldv<double, PPL>(xr + J[u] * sp + c0);
            vi[u] = ldv<double, PPL>(xi + J[u] * sp + c0);
          }
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const double h = nz0 + u < end ? sld(a.hval + nz0 + u) : 0.0;
#pragma unroll
            for (int q = 0; q < PPL; ++q) {
              sr[0][q] = fma(h, vr[u].v[q], sr[0][q]);
              si[0][q] = fma(h, vi[u].v[q], si[0][q]);
            }
            if constexpr (HS) {
              const double sv = nz0 + u < end ? sld(a.sval + nz0 + u) : 0.0;
#pragma unroll
              for (int q = 0; q < PPL; ++q) {
                tr[0][q] = fma(sv, vr[u].v[q], tr[0][q]);
                ti[0][q] = fma(sv, vi[u].v[q], ti[0][q]);
              }
            }
          }
        }
      } else {
        double *hw = hs[wave];
        constexpr int CH = U * BB;               // H_hat entries per chunk (then as many of S)
        constexpr int NH = (NM * CH + 63) / 64;
        for (int64_t nz = beg; nz < end; nz += U) {
          // U blocks per chunk; the value and column arrays carry kStepPad zero
          // blocks past nnzb, and blocks past the row's end get no FMAs
          double hv[NH];
#pragma unroll
          for (int k = 0; k < NH; ++k) {
            const int e = k * 64 + lane;
            if (e < CH) hv[k] = a.hval[nz * BB + e];
            else if (HS && e < NM * CH) hv[k] = a.sval[nz * BB + (e - CH)];
          }
          int64_t J[U];
#pragma unroll
          for (int u = 0; u < U; ++u) J[u] = sld(a.col + nz + u);
          VecN<double, PPL> vr[U][BD], vi[U][BD];
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int j = 0; j < BD; ++j) {
              vr[u][j] = ldv<double, PPL>(xr + (J[u] * BD + j) * sp + c0);
              vi[u][j] = ldv<double, PPL>(xi + (J[u] * BD + j) * sp + c0);
            }
          __builtin_amdgcn_wave_barrier();
#pragma unroll
          for (int k = 0; k < NH; ++k) {
            const int e = k * 64 + lane;
            if (e < NM * CH) hw[e] = hv[k];
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
                  const double h = hw[u * BB + i * BD + j];
#pragma unroll
                  for (int q = 0; q < PPL; ++q) {
                    sr[i][q] = fma(h, vr[u][j].v[q], sr[i][q]);
                    si[i][q] = fma(h, vi[u][j].v[q], si[i][q]);
                  }
                  if constexpr (HS) {
                    const double sv = hw[CH + u * BB + i * BD + j];
#pragma unroll
                    for (int q = 0; q < PPL; ++q) {
                      tr[i][q] = fma(sv, vr[u][j].v[q], tr[i][q]);
                      ti[i][q] = fma(sv, vi[u][j].v[q], ti[i][q]);
                    }
                  }
                }
            }
          }
        }
      }
#pragma unroll
      for (int i = 0; i < BD; ++i) {
        const int64_t off = (I * BD + i) * sp + c0;
        VecN<double, PPL> ar, ai;
        if constexpr (HS) {
#pragma unroll
          for (int q = 0; q < PPL; ++q) {
            ar.v[q] = tr[i][q];
            ai.v[q] = ti[i][q];
          }
        } else {
          ar = ldv<double, PPL>(xr + off);
          ai = ldv<double, PPL>(xi + off);
        }
        VecN<double, PPL> o_r, o_i;
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          // (h - z m) x with m x = (ar, ai) = x (S = I) or S x:
          //   re = h xr - zr ar + zi ai,  im = h xi - zr ai - zi ar
          const double vr = fma(zi, ai.v[q], fma(-zr, ar.v[q], sr[i][q]));
          const double vi = fma(-zi, ar.v[q], fma(-zr, ai.v[q], si[i][q]));
          o_r.v[q] = vr;
          o_i.v[q] = vi;
          if (nrm_on) nrm[q] = fma(vi, vi, fma(vr, vr, nrm[q]));
        }
        stv<double, PPL>(orr + off, o_r);
        stv<double, PPL>(oi + off, o_i);
      }
    }
  }
  if (nrm_on && cur_pt >= 0) flush_norm<PPL>(nrm, red, wave, lane, prow, cur_pt);
}

namespace {

template <bool HS>
const void *select_cspmm_t(int bd, int ppl, int u) {
  if (bd == 1) {
    if (u == 8) return ppl == 2 ? (const void *)k_cspmm<1, 2, 8, HS> : (const void *)k_cspmm<1, 1, 8, HS>;
    return ppl == 2 ? (const void *)k_cspmm<1, 2, 4, HS> : (const void *)k_cspmm<1, 1, 4, HS>;
  }
  if (bd == 9) {
    if (u == 2) return ppl == 2 ? (const void *)k_cspmm<9, 2, 2, HS> : (const void *)k_cspmm<9, 1, 2, HS>;
    return ppl == 2 ? (const void *)k_cspmm<9, 2, 1, HS> : (const void *)k_cspmm<9, 1, 1, HS>;
  }
  return nullptr;
}

// u: neighbours per chunk (1x1: 4 or 8; 9x9: blocks per chunk, 1 or 2); hs: with S
const void *select_cspmm(int bd, int ppl, int u, bool hs) {
  return hs ? select_cspmm_t<true>(bd, ppl, u) : select_cspmm_t<false>(bd, ppl, u);
}

// rows [lo, hi) of workgroup b when n rows are split over gridDim.x workgroups
__device__ __forceinline__ void row_range(int64_t n, int64_t &lo, int64_t &hi) {
  const int64_t G = gridDim.x, b = blockIdx.x;
  lo = n * b / G;
  hi = n * (b + 1) / G;
}

// Thread layout of the row-range kernels: with sp < kWG (and kWG a multiple of
// sp) the kWG / sp row lanes of a column take every (kWG / sp)-th row and their
// sums are combined in lane order (ColLanes::finish); otherwise one thread per
// column (a loop over columns when sp > kWG).
struct ColLanes {
  int nl, lr, c0, cstep;
  __device__ ColLanes(int sp) {
    nl = (sp < kWG && kWG % sp == 0) ? kWG / sp : 1;
    lr = nl > 1 ? (int)threadIdx.x / sp : 0;
    c0 = nl > 1 ? (int)threadIdx.x % sp : (int)threadIdx.x;
    cstep = nl > 1 ? sp : kWG;
  }
  // stores the column sum v of column c into out[c] (row lane 0 after combining)
  __device__ void finish(double v, int c, int sp, double *red, double *out) const {
    if (nl == 1) {
      out[c] = v;
      return;
    }
    red[threadIdx.x] = v;
    __syncthreads();
    if (lr == 0) {
      double t = red[c];
      for (int l = 1; l < nl; ++l) t += red[l * sp + c];
      out[c] = t;
    }
    __syncthreads();
  }
};

}  // namespace

int cspmm_blocks_per_cu(int bd, int ppl, int u, bool hs) {
  const void *f = select_cspmm(bd, ppl, u, hs);
  if (!f) return 0;
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, f, kWG, 0) != hipSuccess) return 0;
  return nb;
}

hipError_t launch_cspmm(int bd, int ppl, int u, const CspArgs &a, hipStream_t s) {
  const void *f = select_cspmm(bd, ppl, u, a.sval != nullptr);
  if (!f || a.sp % (64 * ppl) != 0 || a.grid % 8 != 0 || a.grid <= 0) return hipErrorInvalidValue;
  CspArgs args = a;
  void *kargs[] = {&args};
  return hipLaunchKernel(f, dim3(a.grid), dim3(kWG), kargs, 0, s);
}

// dst_re = scale * y, dst_im = 0 (dst_im may be null)
__global__ __launch_bounds__(kWG) void k_cx_fill(const uint64_t *sgn, const double *rden,
                                                 int64_t n, int sp, double scale,
                                                 double *__restrict__ dre,
                                                 double *__restrict__ dim) {
  const int64_t total = n * sp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = e / sp;
    const int c = (int)(e - row * sp);
    dre[e] = scale * probe_value(sgn, rden, row, sp, c);
    if (dim) dim[e] = 0.0;
  }
}

// r = y - q (q null: r = y); partials: part_rr = |r_c|^2, part_yy = y_c . y_c
__global__ __launch_bounds__(kWG) void k_cx_resid(const uint64_t *sgn, const double *rden,
                                                  const double *__restrict__ q, double *__restrict__ r,
                                                  int64_t n, int sp, int64_t plane,
                                                  double *__restrict__ part_rr,
                                                  double *__restrict__ part_yy) {
  int64_t lo, hi;
  row_range(n, lo, hi);
  const ColLanes cl(sp);
  __shared__ double red[kWG];
  for (int c = cl.c0; c < sp; c += cl.cstep) {
    double rr = 0.0, yy = 0.0;
    for (int64_t i = lo + cl.lr; i < hi; i += cl.nl) {
      const int64_t e = i * sp + c;
      const double y = probe_value(sgn, rden, i, sp, c);
      const double a = q ? y - q[e] : y;
      const double b = q ? -q[plane + e] : 0.0;
      r[e] = a;
      r[plane + e] = b;
      rr = fma(b, b, fma(a, a, rr));
      yy = fma(y, y, yy);
    }
    cl.finish(rr, c, sp, red, part_rr + (int64_t)blockIdx.x * sp);
    cl.finish(yy, c, sp, red, part_yy + (int64_t)blockIdx.x * sp);
  }
}

// r -= alpha_c q (complex planes, real alpha); partials of |r_c|^2
__global__ __launch_bounds__(kWG) void k_cx_update(double *__restrict__ r,
                                                   const double *__restrict__ q,
                                                   const double *__restrict__ alpha, int64_t n,
                                                   int sp, int64_t plane,
                                                   double *__restrict__ part) {
  int64_t lo, hi;
  row_range(n, lo, hi);
  const ColLanes cl(sp);
  __shared__ double red[kWG];
  for (int c = cl.c0; c < sp; c += cl.cstep) {
    const double al = alpha[c];
    double rr = 0.0;
    for (int64_t i = lo + cl.lr; i < hi; i += cl.nl) {
      const int64_t e = i * sp + c;
      const double a = fma(-al, q[e], r[e]);
      const double b = fma(-al, q[plane + e], r[plane + e]);
      r[e] = a;
      r[plane + e] = b;
      rr = fma(b, b, fma(a, a, rr));
    }
    cl.finish(rr, c, sp, red, part + (int64_t)blockIdx.x * sp);
  }
}

// x += alpha_c p, then p = s + beta_c p (both planes): the step of the solution
// along the direction of this iteration, and the next direction
__global__ __launch_bounds__(kWG) void k_cx_dir(const double *__restrict__ sv, double *__restrict__ p,
                                                double *__restrict__ x,
                                                const double *__restrict__ alpha,
                                                const double *__restrict__ beta, int64_t n2,
                                                int sp) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n2;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e % sp);
    const double pv = p[e];
    x[e] = fma(alpha[c], pv, x[e]);
    p[e] = fma(beta[c], pv, sv[e]);
  }
}

// partials of y_c . a_c and y_c . b_c; with acc: acc += wr a - wi b (= Re[(wr + i wi)(a + i b)])
__global__ __launch_bounds__(kWG) void k_cx_pdot(const uint64_t *sgn, const double *rden,
                                                 const double *__restrict__ yd,
                                                 const double *__restrict__ av,
                                                 const double *__restrict__ bv, int64_t n, int sp,
                                                 double *__restrict__ acc, double wr, double wi,
                                                 double *__restrict__ part_a,
                                                 double *__restrict__ part_b) {
  int64_t lo, hi;
  row_range(n, lo, hi);
  const ColLanes cl(sp);
  __shared__ double red[kWG];
  for (int c = cl.c0; c < sp; c += cl.cstep) {
    double sa = 0.0, sb = 0.0;
    for (int64_t i = lo + cl.lr; i < hi; i += cl.nl) {
      const int64_t e = i * sp + c;
      const double y = yd ? yd[e] : probe_value(sgn, rden, i, sp, c);
      const double a = av[e], b = bv[e];
      sa = fma(y, a, sa);
      sb = fma(y, b, sb);
      if (acc) acc[e] = fma(-wi, b, fma(wr, a, acc[e]));
    }
    cl.finish(sa, c, sp, red, part_a + (int64_t)blockIdx.x * sp);
    cl.finish(sb, c, sp, red, part_b + (int64_t)blockIdx.x * sp);
  }
}

// Per-column CGLS scalars (one workgroup), sc = [yy | gam | qq | ssn | rr | alpha | beta]:
// mode 0 (start): gam = ssn;  mode 1: alpha = gam / qq;  mode 2: beta = ssn / gam,
// gam = ssn.  Modes 0 and 2 write *resmax = max_c rr / yy over columns with yy > 0.
__global__ __launch_bounds__(kWG) void k_cgls_scalars(double *__restrict__ sc, int sp, int mode,
                                                      double *__restrict__ resmax) {
  double *yy = sc, *gam = sc + sp, *qq = sc + 2 * sp, *ssn = sc + 3 * sp, *rr = sc + 4 * sp,
         *al = sc + 5 * sp, *be = sc + 6 * sp;
  double m = 0.0;
  for (int c = threadIdx.x; c < sp; c += blockDim.x) {
    if (mode == 1) {
      al[c] = (gam[c] > 0.0 && qq[c] > 0.0) ? gam[c] / qq[c] : 0.0;
    } else {
      if (mode == 2) be[c] = gam[c] > 0.0 ? ssn[c] / gam[c] : 0.0;
      gam[c] = ssn[c];
      if (yy[c] > 0.0) m = fmax(m, rr[c] / yy[c]);
      // a non-finite residual must reach the host check (fmax drops NaN)
      if (!isfinite(rr[c]) || !isfinite(ssn[c])) m = HUGE_VAL;
    }
  }
  if (mode == 1) return;
  m = wave_max(m);
  __shared__ double red[kWaves];
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = red[0];
    for (int w = 1; w < kWaves; ++w) t = fmax(t, red[w]);
    *resmax = t;
  }
}

// One CGLS half-iteration's column sums (colsum's fixed order, as launch_colreduce) and
// scalars in one kernel, on sc = [yy | gam | qq | ssn | rr | alpha | beta]:
//   mode 1: qq = sums of pa [na][sp]; alpha = gam / qq; *resmax = 0 for mode 2.
//   mode 2: ssn = sums of pa [na][sp], rr = sums of pb [nb][sp]; beta = ssn / gam,
//           gam = ssn, *resmax = max_c rr / yy over columns with yy > 0 (an integer max
//           on the bit patterns of non-negative doubles), +inf for a non-finite rr or ssn.
__global__ __launch_bounds__(64 * kColWaves) void k_cgls_reduce(const double *__restrict__ pa, int na,
                                                                const double *__restrict__ pb, int nb,
                                                                int sp, double *__restrict__ sc,
                                                                int mode,
                                                                double *__restrict__ resmax) {
  __shared__ double red_a[kColPh][kColCols], red_b[kColPh][kColCols];
  int c;
  const double va = colsum(pa, na, sp, red_a, c);
  const double vb = mode == 2 ? colsum(pb, nb, sp, red_b, c) : 0.0;
  if (threadIdx.x >= kColCols) return;
  double *yy = sc, *gam = sc + sp, *qq = sc + 2 * sp, *ssn = sc + 3 * sp, *rr = sc + 4 * sp,
         *al = sc + 5 * sp, *be = sc + 6 * sp;
  if (mode == 1 && blockIdx.x == 0 && threadIdx.x == 0) *resmax = 0.0;
  if (c >= sp) return;
  if (mode == 1) {
    qq[c] = va;
    al[c] = (gam[c] > 0.0 && va > 0.0) ? gam[c] / va : 0.0;
    return;
  }
  ssn[c] = va;
  rr[c] = vb;
  be[c] = gam[c] > 0.0 ? va / gam[c] : 0.0;
  gam[c] = va;
  double m = -1.0;
  if (yy[c] > 0.0) m = vb / yy[c];
  if (!isfinite(vb) || !isfinite(va)) m = HUGE_VAL;
  if (m >= 0.0)
    atomicMax(reinterpret_cast<unsigned long long *>(resmax),
              (unsigned long long)__double_as_longlong(m));
}

// N, E, F of the rational estimate (one workgroup, fixed order):
//   per column c:  N_c = f0 m0 + 2 Re sum_k cn_k rho_kc
//                  E_c = f0 h + ew m0 + 2 Re sum_k ce_k rho_kc
//                  F_c = g1 h + g0 m0 + 2 Re sum_k cf_k rho_kc
// with m0 = r.r, h = (H r).(S^{-1} r) (S = I: r.H r), rho_kc = (S r_c) . x_kc and
// coef = [cn | ce | cf] complex per pole; out3 = sum_c w_c (N_c, E_c, F_c).
__global__ __launch_bounds__(kWG) void k_rational_traces(const double *__restrict__ rho,
                                                         const double *__restrict__ m01,
                                                         const double *__restrict__ w,
                                                         const double *__restrict__ coef,
                                                         int n_poles, int sp, RationalScalars k,
                                                         double *__restrict__ out3) {
  double acc[3] = {0.0, 0.0, 0.0};
  for (int c = threadIdx.x; c < sp; c += blockDim.x) {
    const double m0 = m01[c], rhr = m01[sp + c];
    double sn = 0.0, se = 0.0, sf = 0.0;
    for (int p = 0; p < n_poles; ++p) {
      const double pr = rho[(int64_t)p * 2 * sp + c], pi = rho[(int64_t)p * 2 * sp + sp + c];
      const double *cn = coef + 2 * p, *ce = coef + 2 * (n_poles + p), *cf = coef + 2 * (2 * n_poles + p);
      sn += cn[0] * pr - cn[1] * pi;
      se += ce[0] * pr - ce[1] * pi;
      sf += cf[0] * pr - cf[1] * pi;
    }
    const double wc = w[c];
    acc[0] = fma(wc, k.f0 * m0 + 2.0 * sn, acc[0]);
    acc[1] = fma(wc, k.f0 * rhr + k.ew * m0 + 2.0 * se, acc[1]);
    acc[2] = fma(wc, k.g1 * rhr + k.g0 * m0 + 2.0 * sf, acc[2]);
  }
  __shared__ double red[3][kWaves];
  for (int t = 0; t < 3; ++t) {
    const double v = wave_sum(acc[t]);
    if ((threadIdx.x & 63) == 0) red[t][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int wv = 0; wv < kWaves; ++wv) s += red[threadIdx.x][wv];
    out3[threadIdx.x] = s;
  }
}

namespace {
int ew_blocks(int64_t total) {
  int64_t b = (total + kWG - 1) / kWG;
  if (b > 65536) b = 65536;
  return (int)std::max<int64_t>(1, b);
}
}  // namespace

hipError_t launch_cx_fill(const uint64_t *sgn, const double *rden, int64_t n, int sp, double scale,
                          double *dre, double *dim, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_fill, dim3(ew_blocks(n * sp)), dim3(kWG), 0, s, sgn, rden, n, sp, scale,
                     dre, dim);
  return hipGetLastError();
}

hipError_t launch_cx_resid(const uint64_t *sgn, const double *rden, const double *q, double *r,
                           int64_t n, int sp, double *part_rr, double *part_yy, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_resid, dim3(cg_nparts(n)), dim3(kWG), 0, s, sgn, rden, q, r, n, sp,
                     n * sp, part_rr, part_yy);
  return hipGetLastError();
}

hipError_t launch_cx_update(double *r, const double *q, const double *alpha, int64_t n, int sp,
                            double *part, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_update, dim3(cg_nparts(n)), dim3(kWG), 0, s, r, q, alpha, n, sp, n * sp,
                     part);
  return hipGetLastError();
}

hipError_t launch_cx_dir(const double *sv, double *p, double *x, const double *alpha,
                         const double *beta, int64_t n, int sp, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_dir, dim3(ew_blocks(2 * n * sp)), dim3(kWG), 0, s, sv, p, x, alpha, beta,
                     2 * n * sp, sp);
  return hipGetLastError();
}

hipError_t launch_cx_pdot(const uint64_t *sgn, const double *rden, const double *yd, const double *a,
                          const double *b, int64_t n, int sp, double *acc, double wr, double wi,
                          double *part_a, double *part_b, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_pdot, dim3(cg_nparts(n)), dim3(kWG), 0, s, sgn, rden, yd, a, b, n, sp,
                     acc, wr, wi, part_a, part_b);
  return hipGetLastError();
}

// dst = alpha * src over n elements
__global__ __launch_bounds__(kWG) void k_cx_scale(const double *__restrict__ src,
                                                  double *__restrict__ dst, int64_t n,
                                                  double alpha) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (int64_t)gridDim.x * blockDim.x)
    dst[e] = alpha * src[e];
}

hipError_t launch_cx_scale(const double *src, double *dst, int64_t n, double alpha, hipStream_t s) {
  hipLaunchKernelGGL(k_cx_scale, dim3(ew_blocks(n)), dim3(kWG), 0, s, src, dst, n, alpha);
  return hipGetLastError();
}

hipError_t launch_cgls_scalars(double *sc, int sp, int mode, double *resmax, hipStream_t s) {
  hipLaunchKernelGGL(k_cgls_scalars, dim3(1), dim3(kWG), 0, s, sc, sp, mode, resmax);
  return hipGetLastError();
}

hipError_t launch_cgls_reduce(const double *pa, int na, const double *pb, int nb, int sp, double *sc,
                              int mode, double *resmax, hipStream_t s) {
  if (sp <= 0 || (mode != 1 && mode != 2) || (mode == 2 && !pb)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cgls_reduce, dim3((sp + kColCols - 1) / kColCols), dim3(64 * kColWaves), 0, s,
                     pa, na, pb, nb, sp, sc, mode, resmax);
  return hipGetLastError();
}

hipError_t launch_rational_traces(const double *rho, const double *m01, const double *w,
                                  const double *coef, int n_poles, int sp,
                                  const RationalScalars &k, double *out3, hipStream_t s) {
  hipLaunchKernelGGL(k_rational_traces, dim3(1), dim3(kWG), 0, s, rho, m01, w, coef, n_poles, sp,
                     k, out3);
  return hipGetLastError();
}

}  // namespace rfo
