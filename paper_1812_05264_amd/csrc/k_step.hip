// Chebyshev step kernels: one fused pass per term of the three-term recurrence
//   y_{k+1} = 2 H_hat y_k - y_{k-1}   (y_1 = H_hat y_0)
// with the moment partials r_c . y_{k+1} and the density accumulator
// acc += alpha_{k+1} y_{k+1} folded into the same pass (paper: Polynomial
// approximation, Chebyshev recursion with S = I; Random approximation).
// The reverse recurrence of the free-energy gradient uses the same kernel with
// an added beta_j r term.
//
// Mapping: lanes run along probes (64*PPL probes per wave, PPL consecutive per
// lane, one 16-byte or 8-byte access per lane), waves along block rows.  Block
// indices and H_hat entries are wave-uniform and come through the scalar
// cache; each neighbour's vector rows are read as whole coalesced segments.
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

template <int BD, typename VT, typename MT, int PPL>
__global__ __launch_bounds__(kWG) void k_step(StepArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int rg = L / a.n_pt;
  const int pt = L - rg * a.n_pt;
  const int64_t r0 = (int64_t)rg * a.rows_per_wg;
  const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
  const int sp = a.sp;
  const int c0 = pt * (64 * PPL) + lane * PPL;
  const VT *__restrict__ x = static_cast<const VT *>(a.x);
  const VT *prev = static_cast<const VT *>(a.prev);
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const MT *__restrict__ hval = static_cast<const MT *>(a.hval);
  const bool has_prev = a.c2 != 0.0;
  const bool add_r = a.beta != nullptr;
  const double beta = add_r ? *a.beta : 0.0;
  const VT alpha = acc ? (VT)*a.alpha : (VT)0;
  const bool mom_on = a.part != nullptr;
  const VT c1 = (VT)a.c1, c2 = (VT)a.c2;

  double mom[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = 0.0;

  for (int64_t I = r0 + wave; I < r1; I += kWaves) {
    const int64_t beg = a.row_ptr[I], end = a.row_ptr[I + 1];
    VT s[BD][PPL];
#pragma unroll
    for (int i = 0; i < BD; ++i)
#pragma unroll
      for (int q = 0; q < PPL; ++q) s[i][q] = (VT)0;
    for (int64_t nz = beg; nz < end; ++nz) {
      const int64_t J = a.col[nz];
      const MT *hb = hval + nz * (BD * BD);
      VecN<VT, PPL> xv[BD];
#pragma unroll
      for (int j = 0; j < BD; ++j) xv[j] = ldv<VT, PPL>(x + (J * BD + j) * sp + c0);
#pragma unroll
      for (int i = 0; i < BD; ++i) {
#pragma unroll
        for (int j = 0; j < BD; ++j) {
          const VT h = (VT)hb[i * BD + j];
#pragma unroll
          for (int q = 0; q < PPL; ++q) s[i][q] = fma(h, xv[j].v[q], s[i][q]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < BD; ++i) {
      const int64_t row = I * BD + i;
      const int64_t off = row * sp + c0;
      VecN<VT, PPL> o;
      VecN<VT, PPL> pv;
      if (has_prev) pv = ldv<VT, PPL>(prev + off);
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        VT v = c1 * s[i][q];
        if (has_prev) v = fma(c2, pv.v[q], v);
        o.v[q] = v;
      }
      if (add_r || mom_on) {
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          const double r = probe_value(a.sgn, a.rden, row, sp, c0 + q);
          if (add_r) o.v[q] = (VT)((double)o.v[q] + beta * r);
          mom[q] = fma(r, (double)o.v[q], mom[q]);
        }
      }
      stv<VT, PPL>(out + off, o);
      if (acc) {
        VecN<VT, PPL> av = ldv<VT, PPL>(acc + off);
#pragma unroll
        for (int q = 0; q < PPL; ++q) av.v[q] = fma(alpha, o.v[q], av.v[q]);
        stv<VT, PPL>(acc + off, av);
      }
    }
  }

  if (mom_on) {
    __shared__ double red[kWaves][64 * PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) red[wave][lane * PPL + q] = mom[q];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        double t = red[0][lane * PPL + q];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += red[w][lane * PPL + q];
        a.part[(int64_t)rg * sp + c0 + q] = t;
      }
    }
  }
}

// y = scale * r, optional acc = alpha * y and moment partials r . y, with the
// same workgroup decomposition as k_step so that the partials line up.
template <typename VT, int PPL>
__global__ __launch_bounds__(kWG) void k_init(InitArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int L = xcd_logical(blockIdx.x, gridDim.x);
  const int rg = L / a.n_pt;
  const int pt = L - rg * a.n_pt;
  const int64_t r0 = (int64_t)rg * a.rows_per_wg;
  const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
  const int sp = a.sp;
  const int c0 = pt * (64 * PPL) + lane * PPL;
  VT *out = static_cast<VT *>(a.out);
  VT *acc = static_cast<VT *>(a.acc);
  const double scale = a.scale ? *a.scale : 1.0;
  const double alpha = acc ? *a.alpha : 0.0;
  double mom[PPL];
#pragma unroll
  for (int q = 0; q < PPL; ++q) mom[q] = 0.0;
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
  if (a.part) {
    __shared__ double red[kWaves][64 * PPL];
#pragma unroll
    for (int q = 0; q < PPL; ++q) red[wave][lane * PPL + q] = mom[q];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
      for (int q = 0; q < PPL; ++q) {
        double t = red[0][lane * PPL + q];
#pragma unroll
        for (int w = 1; w < kWaves; ++w) t += red[w][lane * PPL + q];
        a.part[(int64_t)rg * sp + c0 + q] = t;
      }
    }
  }
}

template <int BD, typename VT, typename MT>
static hipError_t launch_step_t(int ppl, const StepArgs &a, hipStream_t s) {
  const dim3 grid((unsigned)((int64_t)a.n_rg * a.n_pt)), block(kWG);
  switch (ppl) {
    case 1: hipLaunchKernelGGL((k_step<BD, VT, MT, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_step<BD, VT, MT, 2>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_step<BD, VT, MT, 4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_step(int bd, int precision, int ppl, const StepArgs &a, hipStream_t s) {
  if (bd == 1) {
    return precision == 0 ? launch_step_t<1, double, double>(ppl, a, s)
                          : launch_step_t<1, float, float>(ppl, a, s);
  }
  if (bd == 9) {
    return precision == 0 ? launch_step_t<9, double, double>(ppl, a, s)
                          : launch_step_t<9, float, float>(ppl, a, s);
  }
  return hipErrorInvalidValue;
}

template <typename VT>
static hipError_t launch_init_t(const InitArgs &a, hipStream_t s) {
  const dim3 grid((unsigned)((int64_t)a.n_rg * a.n_pt)), block(kWG);
  switch (a.ppl) {
    case 1: hipLaunchKernelGGL((k_init<VT, 1>), grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL((k_init<VT, 2>), grid, block, 0, s, a); break;
    case 4: hipLaunchKernelGGL((k_init<VT, 4>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_init(int precision, const InitArgs &a, hipStream_t s) {
  return precision == 0 ? launch_init_t<double>(a, s) : launch_init_t<float>(a, s);
}

}  // namespace rfo
