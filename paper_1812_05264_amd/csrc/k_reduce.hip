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
// a fixed butterfly reduces them at the end (bitwise reproducible).  The gradient's
// two outer products (X_I Y_J^T and Y_I X_J^T) load their rows one after the
// other, so that only one pair of row sets is live and two waves fit per SIMD.  Workgroups
// are remapped so that each XCD takes one contiguous range of the block list:
// the waves in flight on an XCD then read the vectors of a narrow band of block
// rows, which that XCD's L2 holds.
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

template <int BD, typename VT, int PPL, bool SYM>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(2))) void k_sddmm(SddmmArgs a) {
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t widx = (int64_t)xcd_logical(blockIdx.x, gridDim.x) * kWaves + wave;
  const int64_t total = a.nzlist ? a.nlist : a.nnzb;
  if (widx >= total) return;
  const int64_t nz = a.nzlist ? sld(a.nzlist + widx) : widx;
  const int64_t I = sld(a.brow + nz);
  const int64_t J = sld(a.col + nz);
  const int sp = a.sp;
  // zero-weight columns past s_live add nothing
  const int c_end = a.s_live > 0 ? min(a.s_live, sp) : sp;
  double s[BD][BD];
#pragma unroll
  for (int i = 0; i < BD; ++i)
#pragma unroll
    for (int j = 0; j < BD; ++j) s[i][j] = 0.0;

  for (int t = 0; t < a.count; ++t) {
    const double coef = a.scale * ((a.j0 + t == 0) ? a.first : a.rest);
    const VT *X = static_cast<const VT *>(a.xbase) + (int64_t)t * a.xstride;
    const VT *Y = a.ybase ? static_cast<const VT *>(a.ybase) + (int64_t)t * a.ystride : nullptr;
    for (int c = lane * PPL; c < c_end; c += 64 * PPL) {
      double wc[PPL];
#pragma unroll
      for (int q = 0; q < PPL; ++q) wc[q] = a.w[c + q] * coef;
      // phase 1: X_I Y_J^T (Y from the probes when there is no Y vector)
      {
        VecN<VT, PPL> xv[BD], yv[BD];
#pragma unroll
        for (int i = 0; i < BD; ++i) xv[i] = ldv<VT, PPL>(X + (I * BD + i) * sp + c);
        if (Y) {
#pragma unroll
          for (int j = 0; j < BD; ++j) yv[j] = ldv<VT, PPL>(Y + (J * BD + j) * sp + c);
        } else {
#pragma unroll
          for (int j = 0; j < BD; ++j)
#pragma unroll
            for (int q = 0; q < PPL; ++q)
              yv[j].v[q] = (VT)probe_value(a.sgn, a.rden, J * BD + j, sp, c + q);
        }
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          double xa[BD];
#pragma unroll
          for (int i = 0; i < BD; ++i) xa[i] = wc[q] * (double)xv[i].v[q];
#pragma unroll
          for (int i = 0; i < BD; ++i)
#pragma unroll
            for (int j = 0; j < BD; ++j) s[i][j] = fma(xa[i], (double)yv[j].v[q], s[i][j]);
        }
      }
      if constexpr (SYM) {
        // phase 2: + Y_I X_J^T, its rows requested only after phase 1's products
        __builtin_amdgcn_sched_barrier(0);
        VecN<VT, PPL> xj[BD], yi[BD];
#pragma unroll
        for (int i = 0; i < BD; ++i) {
          yi[i] = ldv<VT, PPL>(Y + (I * BD + i) * sp + c);
          xj[i] = ldv<VT, PPL>(X + (J * BD + i) * sp + c);
        }
#pragma unroll
        for (int q = 0; q < PPL; ++q) {
          double ya[BD];
#pragma unroll
          for (int i = 0; i < BD; ++i) ya[i] = wc[q] * (double)yi[i].v[q];
#pragma unroll
          for (int i = 0; i < BD; ++i)
#pragma unroll
            for (int j = 0; j < BD; ++j) s[i][j] = fma(ya[i], (double)xj[j].v[q], s[i][j]);
        }
      }
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

template <int BD, typename VT>
static void launch_sddmm_t(const SddmmArgs &a, dim3 grid, hipStream_t s) {
  if (a.sym) {
    if (a.ppl == 2) hipLaunchKernelGGL((k_sddmm<BD, VT, 2, true>), grid, dim3(kWG), 0, s, a);
    else hipLaunchKernelGGL((k_sddmm<BD, VT, 1, true>), grid, dim3(kWG), 0, s, a);
  } else {
    if (a.ppl == 2) hipLaunchKernelGGL((k_sddmm<BD, VT, 2, false>), grid, dim3(kWG), 0, s, a);
    else hipLaunchKernelGGL((k_sddmm<BD, VT, 1, false>), grid, dim3(kWG), 0, s, a);
  }
}

hipError_t launch_sddmm(int precision, const SddmmArgs &a, hipStream_t s) {
  const int64_t total = a.nzlist ? a.nlist : a.nnzb;
  if (total == 0) return hipSuccess;
  if (a.ppl == 2 && (a.sp % 128) != 0) return hipErrorInvalidValue;
  if (a.sym && !a.ybase) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((total + kWaves - 1) / kWaves));
  if (a.bd == 1) {
    if (precision == 0) launch_sddmm_t<1, double>(a, grid, s);
    else launch_sddmm_t<1, float>(a, grid, s);
  } else if (a.bd == 9) {
    if (precision == 0) launch_sddmm_t<9, double>(a, grid, s);
    else launch_sddmm_t<9, float>(a, grid, s);
  } else {
    return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_mirror(const int64_t *__restrict__ nzlist, int64_t nlist,
                                                const int64_t *__restrict__ tpos, int bd,
                                                double *__restrict__ G) {
  const int bb = bd * bd;
  const int64_t total = nlist * bb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = e / bb;
    const int r = (int)(e - k * bb);
    const int i = r / bd, j = r - (r / bd) * bd;
    const int64_t nz = nzlist[k];
    G[nz * bb + i * bd + j] = G[tpos[nz] * bb + j * bd + i];
  }
}

hipError_t launch_mirror(const int64_t *nzlist, int64_t nlist, const int64_t *tpos, int bd,
                         double *G, hipStream_t s) {
  if (nlist == 0) return hipSuccess;
  int64_t blocks = (nlist * bd * bd + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_mirror, dim3((unsigned)blocks), dim3(kWG), 0, s, nzlist, nlist, tpos, bd, G);
  return hipGetLastError();
}

__global__ __launch_bounds__(kWG) void k_forces(const int64_t *__restrict__ row_ptr,
                                                const int64_t *__restrict__ tpos,
                                                const double *__restrict__ G,
                                                const double *__restrict__ D, int64_t nb, int bd,
                                                double *__restrict__ F, double sign, int accumulate) {
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
    const double v = -sign * wave_sum(f[d]);
    if (lane == 0) F[a * 3 + d] = accumulate ? F[a * 3 + d] + v : v;
  }
}

hipError_t launch_forces(const int64_t *row_ptr, const int64_t *tpos, const double *G,
                         const double *D, int64_t nb, int bd, double *F, double sign, int accumulate,
                         hipStream_t s) {
  if (nb == 0) return hipSuccess;
  hipLaunchKernelGGL(k_forces, dim3((unsigned)((nb + kWaves - 1) / kWaves)), dim3(kWG), 0, s,
                     row_ptr, tpos, G, D, nb, bd, F, sign, accumulate);
  return hipGetLastError();
}

}  // namespace rfo
