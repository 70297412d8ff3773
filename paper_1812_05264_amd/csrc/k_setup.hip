// Setup and reduction kernels of the randomized Fermi-operator path:
//   spectral map of H (Polynomial approximation: H_hat = (2H - (e_max+e_min)I)/(e_max-e_min)),
//   Gershgorin interval fallback, probe packing, Chebyshev coefficients of the
//   Fermi, energy-weighted and free-energy functions by Chebyshev-Gauss
//   quadrature, fixed-order moment reduction and the traces N, E, F
//   (Methods: free-energy function, electron count and band energy).
// Every reduction here runs in a fixed order: results are bitwise reproducible.
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

// ---- spectral map -----------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_map(const double *__restrict__ h,
                                             const int64_t *__restrict__ brow,
                                             const int32_t *__restrict__ col,
                                             const int64_t *__restrict__ tpos, int64_t nnzb,
                                             int bd, double e_min, double e_max,
                                             double *__restrict__ hhat64,
                                             float *__restrict__ hhat32, int *flags) {
  const int bb = bd * bd;
  const int64_t total = nnzb * bb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t nz = e / bb;
    const int rem = (int)(e - nz * bb);
    const int i = rem / bd, j = rem - (rem / bd) * bd;
    const double v = h[e];
    if (!isfinite(v)) atomicOr(flags, 1);
    const double vt = h[tpos[nz] * bb + j * bd + i];
    if (!(fabs(v - vt) <= 1e-10 * (fabs(v) + fabs(vt)))) atomicOr(flags, 2);
    const bool diag = (brow[nz] == (int64_t)col[nz]) && (i == j);
    const double shifted = diag ? 2.0 * v - (e_max + e_min) : 2.0 * v;
    const double hh = shifted / (e_max - e_min);
    hhat64[e] = hh;
    if (hhat32) hhat32[e] = (float)hh;
  }
}

hipError_t launch_map(const double *h, const int64_t *brow, const int32_t *col,
                      const int64_t *tpos, int64_t nnzb, int bd, double e_min,
                      double e_max, double *hhat64, float *hhat32, int *flags,
                      hipStream_t s) {
  const int64_t total = nnzb * bd * bd;
  int64_t blocks = (total + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_map, dim3((unsigned)blocks), dim3(kWG), 0, s, h, brow, col, tpos,
                     nnzb, bd, e_min, e_max, hhat64, hhat32, flags);
  return hipGetLastError();
}

// ---- Gershgorin interval ----------------------------------------------------
__global__ __launch_bounds__(kWG) void k_gersh_rows(const double *__restrict__ h,
                                                    const int64_t *__restrict__ row_ptr,
                                                    const int32_t *__restrict__ col, int64_t nb,
                                                    int bd, double *__restrict__ scratch) {
  const int64_t row = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double lo = INFINITY, hi = -INFINITY;
  if (row < nb * bd) {
    const int64_t I = row / bd;
    const int i = (int)(row - I * bd);
    double center = 0.0, rad = 0.0;
    for (int64_t nz = row_ptr[I]; nz < row_ptr[I + 1]; ++nz) {
      for (int j = 0; j < bd; ++j) {
        const double v = h[(nz * bd + i) * bd + j];
        if ((int64_t)col[nz] == I && j == i) center = v;
        else rad += fabs(v);
      }
    }
    lo = center - rad;
    hi = center + rad;
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  __shared__ double slo[kWaves], shi[kWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    slo[wave] = lo;
    shi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWaves; ++w) {
      lo = fmin(lo, slo[w]);
      hi = fmax(hi, shi[w]);
    }
    scratch[2 * blockIdx.x] = fmin(lo, slo[0]);
    scratch[2 * blockIdx.x + 1] = fmax(hi, shi[0]);
  }
}

__global__ __launch_bounds__(kWG) void k_gersh_final(const double *__restrict__ scratch,
                                                     int nblk, double *out2) {
  double lo = INFINITY, hi = -INFINITY;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    lo = fmin(lo, scratch[2 * b]);
    hi = fmax(hi, scratch[2 * b + 1]);
  }
  lo = wave_min(lo);
  hi = wave_max(hi);
  __shared__ double slo[kWaves], shi[kWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    slo[wave] = lo;
    shi[wave] = hi;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 0; w < kWaves; ++w) {
      lo = fmin(lo, slo[w]);
      hi = fmax(hi, shi[w]);
    }
    out2[0] = lo;
    out2[1] = hi;
  }
}

hipError_t launch_gershgorin(const double *h, const int64_t *row_ptr, const int32_t *col,
                             int64_t nb, int bd, double *scratch, double *out2,
                             hipStream_t s) {
  const int64_t rows = nb * bd;
  const int nblk = (int)((rows + kWG - 1) / kWG);
  hipLaunchKernelGGL(k_gersh_rows, dim3(nblk), dim3(kWG), 0, s, h, row_ptr, col, nb, bd,
                     scratch);
  hipLaunchKernelGGL(k_gersh_final, dim3(1), dim3(kWG), 0, s, scratch, nblk, out2);
  return hipGetLastError();
}

// ---- probes -------------------------------------------------------------------
// flags bit 0: some real entry is not +-1 (dense storage needed); bit 1: non-finite
__global__ __launch_bounds__(kWG) void k_probe_pack(const double *__restrict__ rden, int64_t n,
                                                    int s_real, int sp, uint64_t *__restrict__ sgn,
                                                    int *flags) {
  const int nw = sp >> 6;
  const int64_t total = n * nw;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t row = t / nw;
    const int w = (int)(t - row * nw);
    uint64_t bits = 0;
    for (int b = 0; b < 64; ++b) {
      const int c = w * 64 + b;
      const double v = rden[row * sp + c];
      if (c < s_real) {
        if (!isfinite(v)) atomicOr(flags, 2);
        if (v != 1.0 && v != -1.0) atomicOr(flags, 1);
      }
      if (v > 0.0) bits |= (1ull << b);
    }
    sgn[t] = bits;
  }
}

hipError_t launch_probe_pack(const double *rden, int64_t n, int s_real, int sp, uint64_t *sgn,
                             int *flags, hipStream_t st) {
  const int64_t total = n * (sp >> 6);
  int64_t blocks = (total + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_probe_pack, dim3((unsigned)blocks), dim3(kWG), 0, st, rden, n, s_real,
                     sp, sgn, flags);
  return hipGetLastError();
}

// ---- Chebyshev coefficients -----------------------------------------------------
// Node j of the nq-point Chebyshev-Gauss rule: x_j = cos(pi (j + 1/2)/nq), energy
// e_j = e_min (1 - x_j)/2 + e_max (1 + x_j)/2.  Samples of
//   f(e) = 2/(1 + exp((e - mu)/T)) = 1 - tanh((e - mu)/(2T)),  e f(e),
//   g(e) = -2T ln(1 + exp(-(e - mu)/T)) (stable softplus form),
// and the table cos(pi m/(2 nq)), m < 4 nq, so that cos(pi k (j + 1/2)/nq) is
// entry (k (2j + 1)) mod 4nq: exact argument reduction for every k.
__global__ __launch_bounds__(kWG) void k_coef_samples(double e_min, double e_max, double T,
                                                      double mu, int64_t nq,
                                                      double *__restrict__ samples,
                                                      double *__restrict__ costab) {
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < 4 * nq;
       m += (int64_t)gridDim.x * blockDim.x) {
    costab[m] = cospi((double)m / (double)(2 * nq));
    if (m < nq) {
      const double x = cos(M_PI * ((double)m + 0.5) / (double)nq);
      const double e = 0.5 * e_min * (1.0 - x) + 0.5 * e_max * (1.0 + x);
      const double f = 1.0 - tanh((e - mu) / (2.0 * T));
      const double z = -(e - mu) / T;
      const double softplus = fmax(z, 0.0) + log1p(exp(-fabs(z)));
      samples[m] = f;
      samples[nq + m] = e * f;
      samples[2 * nq + m] = -2.0 * T * softplus;
    }
  }
}

// c_k = (2 - delta_k0)/nq sum_j h(e_j) cos(pi k (j + 1/2)/nq), one workgroup per k
__global__ __launch_bounds__(kWG) void k_coefs(const double *__restrict__ samples,
                                               const double *__restrict__ costab, int64_t nq,
                                               int64_t p, double *__restrict__ coef) {
  const int64_t k = blockIdx.x;
  const int64_t M = 4 * nq;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t j = threadIdx.x; j < nq; j += blockDim.x) {
    const double cv = costab[(k * (2 * j + 1)) % M];
    s0 = fma(samples[j], cv, s0);
    s1 = fma(samples[nq + j], cv, s1);
    s2 = fma(samples[2 * nq + j], cv, s2);
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  __shared__ double red[3][kWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += red[threadIdx.x][w];
    coef[threadIdx.x * p + k] = (k == 0 ? 1.0 : 2.0) / (double)nq * t;
  }
}

hipError_t launch_coefficients(double e_min, double e_max, double T, double mu, int64_t p,
                               int64_t nq, double *samples, double *costab, double *coef,
                               hipStream_t s) {
  int64_t blocks = (4 * nq + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_coef_samples, dim3((unsigned)blocks), dim3(kWG), 0, s, e_min, e_max, T,
                     mu, nq, samples, costab);
  hipLaunchKernelGGL(k_coefs, dim3((unsigned)p), dim3(kWG), 0, s, samples, costab, nq, p,
                     coef);
  return hipGetLastError();
}

// ---- moments ---------------------------------------------------------------------
// flags bit 2: a moment exceeded its bound or is not finite.
// One workgroup of 16 waves per (moment index, 64-probe chunk): wave w sums the
// partial rows g = w, w + 16, ... into four interleaved accumulators (so that
// each lane keeps four loads in flight), adds them as (s0 + s1) + (s2 + s3), and
// wave 0 adds the 16 wave sums in order.  The order is fixed, so the moments are
// bitwise reproducible.
constexpr int kRedWaves = 16;

__global__ __launch_bounds__(64 * kRedWaves) void k_moment_reduce(const double *__restrict__ part, int ring,
                                                                  int64_t k0, int count, int n_rg, int sp,
                                                                  double *__restrict__ moments, int check,
                                                                  double tol, int *flags, int dbl) {
  const int chunks = sp >> 6;
  const int d = blockIdx.x / chunks;
  const int lane = threadIdx.x & 63;
  const int c = (blockIdx.x - d * chunks) * 64 + lane;
  const int wave = threadIdx.x >> 6;
  const int64_t k = k0 + d;
  const double *src = part + (int64_t)(k % ring) * n_rg * sp + c;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  int g = wave;
  for (; g + 3 * kRedWaves < n_rg; g += 4 * kRedWaves) {
#pragma unroll
    for (int u = 0; u < 4; ++u) s[u] += src[(int64_t)(g + u * kRedWaves) * sp];
  }
#pragma unroll
  for (int u = 0; u < 3; ++u)
    if (g + u * kRedWaves < n_rg) s[u] += src[(int64_t)(g + u * kRedWaves) * sp];
  __shared__ double red[kRedWaves][64];
  red[wave][lane] = (s[0] + s[1]) + (s[2] + s[3]);
  __syncthreads();
  if (wave == 0) {
    double sum = red[0][lane];
    for (int w = 1; w < kRedWaves; ++w) sum += red[w][lane];
    // doubling: the partials hold <y_j, y_j> (k = 2j) or <y_j, y_{j-1}> (k = 2j-1);
    // T_2j = 2 T_j^2 - T_0 and T_2j-1 = 2 T_j T_j-1 - T_1 give the moment
    if (dbl && k >= 2) sum = 2.0 * sum - moments[(k & 1) * sp + c];
    moments[k * sp + c] = sum;
    if (check) {
      const double bound = moments[c] * (1.0 + tol) + 1e-300;
      if (!(fabs(sum) <= bound)) atomicOr(flags, 4);
    }
  }
}

hipError_t launch_moment_reduce(const double *part, int ring, int64_t k0, int count, int n_rg,
                                int sp, double *moments, int check, double tol, int *flags,
                                int dbl, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_moment_reduce, dim3((unsigned)(count * (sp >> 6))), dim3(64 * kRedWaves), 0, s, part,
                     ring, k0, count, n_rg, sp, moments, check, tol, flags, dbl);
  return hipGetLastError();
}

// ---- traces ----------------------------------------------------------------------
// out = [N, E, F] = sum_k c_k sum_c w_c mu[k][c] for the three coefficient sets
__global__ __launch_bounds__(kWG) void k_traces(const double *__restrict__ moments,
                                                const double *__restrict__ w,
                                                const double *__restrict__ coef, int64_t p, int sp,
                                                double *out3) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t k = threadIdx.x; k < p; k += blockDim.x) {
    double m = 0.0;
    for (int c = 0; c < sp; ++c) m = fma(w[c], moments[k * sp + c], m);
    s0 = fma(coef[k], m, s0);
    s1 = fma(coef[p + k], m, s1);
    s2 = fma(coef[2 * p + k], m, s2);
  }
  s0 = wave_sum(s0);
  s1 = wave_sum(s1);
  s2 = wave_sum(s2);
  __shared__ double red[3][kWaves];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    red[0][wave] = s0;
    red[1][wave] = s1;
    red[2][wave] = s2;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int q = 0; q < kWaves; ++q) t += red[threadIdx.x][q];
    out3[threadIdx.x] = t;
  }
}

hipError_t launch_traces(const double *moments, const double *w, const double *coef, int64_t p,
                         int sp, double *out3, hipStream_t s) {
  hipLaunchKernelGGL(k_traces, dim3(1), dim3(kWG), 0, s, moments, w, coef, p, sp, out3);
  return hipGetLastError();
}

}  // namespace rfo
