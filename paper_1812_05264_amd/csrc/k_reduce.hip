// Masked outer-product kernels (density blocks and free-energy gradient) and the
// Hellmann-Feynman force contraction.
//
// Density (Random approximation, random density estimator):
//   D_IJ = sum_c w_c acc_{I,c} r_{J,c}^T  on H's block pattern, acc_c ~ f(H) r_c.
// Gradient (Analytical free-energy derivatives, polynomial form, reverse order):
//   G_IJ += sum_t coef_t sum_c w_c z_{j+1,I,c} y_{j,J,c}^T  over one checkpoint segment.
// Forces (Observable response with S = I):
//   force_a = -(sum_J <G_aJ, D_aJ> - sum_I <G_Ia, D_Ia>),  D_IJ = dH_IJ/dR_I.
//
// One wave owns one block: lanes run along the contraction index (probes), each
// lane keeps all bd*bd partial sums in registers over the whole contraction, and
// a fixed butterfly reduces them at the end (bitwise reproducible).
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

template <int BD, typename VT>
__global__ __launch_bounds__(kWG) void k_sddmm(SddmmArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t nz = (int64_t)blockIdx.x * kWaves + wave;
  if (nz >= a.nnzb) return;
  const int64_t I = a.brow[nz];
  const int64_t J = a.col[nz];
  const int sp = a.sp;
  double s[BD][BD];
#pragma unroll
  for (int i = 0; i < BD; ++i)
#pragma unroll
    for (int j = 0; j < BD; ++j) s[i][j] = 0.0;

  for (int t = 0; t < a.count; ++t) {
    const double coef = a.scale * ((a.j0 + t == 0) ? a.first : a.rest);
    const VT *X = static_cast<const VT *>(a.xbase) + (int64_t)t * a.xstride;
    const VT *Y = a.ybase ? static_cast<const VT *>(a.ybase) + (int64_t)t * a.ystride : nullptr;
    for (int c = lane; c < sp; c += 64) {
      const double wc = a.w[c] * coef;
      double xa[BD], yb[BD];
#pragma unroll
      for (int i = 0; i < BD; ++i) xa[i] = wc * (double)X[(I * BD + i) * sp + c];
#pragma unroll
      for (int j = 0; j < BD; ++j)
        yb[j] = Y ? (double)Y[(J * BD + j) * sp + c] : probe_value(a.sgn, a.rden, J * BD + j, sp, c);
#pragma unroll
      for (int i = 0; i < BD; ++i)
#pragma unroll
        for (int j = 0; j < BD; ++j) s[i][j] = fma(xa[i], yb[j], s[i][j]);
    }
  }
  double *g = a.G + nz * (BD * BD);
#pragma unroll
  for (int i = 0; i < BD; ++i) {
#pragma unroll
    for (int j = 0; j < BD; ++j) {
      const double v = wave_sum(s[i][j]);
      if (lane == 0) g[i * BD + j] = a.accumulate ? g[i * BD + j] + v : v;
    }
  }
}

hipError_t launch_sddmm(int precision, const SddmmArgs &a, hipStream_t s) {
  const dim3 grid((unsigned)((a.nnzb + kWaves - 1) / kWaves)), block(kWG);
  if (a.nnzb == 0) return hipSuccess;
  if (a.bd == 1) {
    if (precision == 0) hipLaunchKernelGGL((k_sddmm<1, double>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sddmm<1, float>), grid, block, 0, s, a);
  } else if (a.bd == 9) {
    if (precision == 0) hipLaunchKernelGGL((k_sddmm<9, double>), grid, block, 0, s, a);
    else hipLaunchKernelGGL((k_sddmm<9, float>), grid, block, 0, s, a);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_forces(const int64_t *__restrict__ row_ptr,
                                                const int64_t *__restrict__ tpos,
                                                const double *__restrict__ G,
                                                const double *__restrict__ D, int64_t nb, int bd,
                                                double *__restrict__ F) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t a = (int64_t)blockIdx.x * kWaves + wave;
  if (a >= nb) return;
  const int bb = bd * bd;
  double f[3] = {0.0, 0.0, 0.0};
  for (int64_t nz = row_ptr[a]; nz < row_ptr[a + 1]; ++nz) {
    const int64_t tz = tpos[nz];
    for (int e = lane; e < bb; e += 64) {
      const double g = G[nz * bb + e];
      const double gt = G[tz * bb + e];
#pragma unroll
      for (int d = 0; d < 3; ++d)
        f[d] += g * D[(nz * 3 + d) * bb + e] - gt * D[(tz * 3 + d) * bb + e];
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double v = wave_sum(f[d]);
    if (lane == 0) F[a * 3 + d] = -v;
  }
}

hipError_t launch_forces(const int64_t *row_ptr, const int64_t *tpos, const double *G,
                         const double *D, int64_t nb, int bd, double *F, hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_forces, dim3((unsigned)((nb + kWaves - 1) / kWaves)), dim3(kWG), 0, s,
                     row_ptr, tpos, G, D, nb, bd, F);
  return hipGetLastError();
}

}  // namespace rfo
