// Nonorthogonal basis (paper: Polynomial approximation with S, Eq. poly_PQ):
// the mapped Hamiltonian H_hat = [2H - (e_max + e_min) S]/(e_max - e_min) and
// the pieces of a conjugate-gradient solve S t = y for a block of probe columns
// (one independent CG per column; the matrix-vector product is the step kernel
// with S as its matrix).  Column reductions are two-pass and in a fixed order.
#include "colsum.h"
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

__global__ __launch_bounds__(kWG) void k_map_overlap(const double *__restrict__ h,
                                                     const double *__restrict__ s,
                                                     const int64_t *__restrict__ tpos,
                                                     int64_t nnzb, int bd, double e_min,
                                                     double e_max, double *__restrict__ hhat,
                                                     int *flags) {
  const int bb = bd * bd;
  const int64_t total = nnzb * bb;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t nz = e / bb;
    const int rem = (int)(e - nz * bb);
    const int i = rem / bd, j = rem - (rem / bd) * bd;
    const double v = s[e];
    if (!isfinite(v)) atomicOr(flags, 1);
    const double vt = s[tpos[nz] * bb + j * bd + i];
    if (!(fabs(v - vt) <= 1e-10 * (fabs(v) + fabs(vt)))) atomicOr(flags, 2);
    hhat[e] = (2.0 * h[e] - (e_max + e_min) * v) / (e_max - e_min);
  }
}

hipError_t launch_map_overlap(const double *h, const double *s, const int64_t *tpos, int64_t nnzb,
                              int bd, double e_min, double e_max, double *hhat, int *flags,
                              hipStream_t st) {
  const int64_t total = nnzb * bd * bd;
  int64_t blocks = (total + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(k_map_overlap, dim3((unsigned)blocks), dim3(kWG), 0, st, h, s, tpos, nnzb, bd,
                     e_min, e_max, hhat, flags);
  return hipGetLastError();
}

namespace {

// rows [lo, hi) of workgroup b when n rows are split over gridDim.x workgroups
__device__ __forceinline__ void row_range(int64_t n, int64_t &lo, int64_t &hi) {
  const int64_t G = gridDim.x, b = blockIdx.x;
  lo = n * b / G;
  hi = n * (b + 1) / G;
}

}  // namespace

// out[c] = sum_b part[b][c] in the fixed order of colsum.
__global__ __launch_bounds__(64 * kColWaves) void k_colreduce(const double *__restrict__ part,
                                                              int nparts, int sp,
                                                              double *__restrict__ out) {
  __shared__ double red[kColPh][kColCols];
  int c;
  const double t = colsum(part, nparts, sp, red, c);
  if (threadIdx.x < kColCols && c < sp) out[c] = t;
}

// The row-range kernels below split a workgroup's threads into R = 256 / C row lanes of
// C columns (C = 64, 128 or 256, the widest that divides sp): rows lo + rl, lo + rl + R,
// ... for the C columns c0 + cl, column chunk by column chunk; the R row lanes of a
// column are then added in row-lane order, so the partials are bitwise reproducible.
__device__ __forceinline__ int cg_cols(int sp) {
  int C = 64;
  while (C < kWG && sp % (2 * C) == 0) C *= 2;
  return C;
}

// t = 0, r = y, p = y, part = column partials of y . y
__global__ __launch_bounds__(kWG) void k_cg_init(const double *__restrict__ y,
                                                 double *__restrict__ t, double *__restrict__ r,
                                                 double *__restrict__ p, int64_t n, int sp,
                                                 double *__restrict__ part) {
  int64_t lo, hi;
  row_range(n, lo, hi);
  const int C = cg_cols(sp), R = kWG / C;
  const int cl = threadIdx.x % C, rl = threadIdx.x / C;
  __shared__ double red[kWG];
  for (int c0 = 0; c0 < sp; c0 += C) {
    const int c = c0 + cl;
    double s = 0.0;
    for (int64_t i = lo + rl; i < hi; i += R) {
      const int64_t e = i * sp + c;
      const double v = y[e];
      t[e] = 0.0;
      r[e] = v;
      p[e] = v;
      s = fma(v, v, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (rl == 0) {
      double a = red[cl];
      for (int q = 1; q < R; ++q) a += red[q * C + cl];
      part[(int64_t)blockIdx.x * sp + c] = a;
    }
    __syncthreads();
  }
}

// t += alpha_c p, r -= alpha_c q, part = column partials of r . r
__global__ __launch_bounds__(kWG) void k_cg_update(double *__restrict__ t, double *__restrict__ r,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ q,
                                                   const double *__restrict__ alpha, int64_t n,
                                                   int sp, double *__restrict__ part) {
  int64_t lo, hi;
  row_range(n, lo, hi);
  const int C = cg_cols(sp), R = kWG / C;
  const int cl = threadIdx.x % C, rl = threadIdx.x / C;
  __shared__ double red[kWG];
  for (int c0 = 0; c0 < sp; c0 += C) {
    const int c = c0 + cl;
    const double al = alpha[c];
    double s = 0.0;
    for (int64_t i = lo + rl; i < hi; i += R) {
      const int64_t e = i * sp + c;
      t[e] = fma(al, p[e], t[e]);
      const double rn = fma(-al, q[e], r[e]);
      r[e] = rn;
      s = fma(rn, rn, s);
    }
    red[threadIdx.x] = s;
    __syncthreads();
    if (rl == 0) {
      double a = red[cl];
      for (int w = 1; w < R; ++w) a += red[w * C + cl];
      part[(int64_t)blockIdx.x * sp + c] = a;
    }
    __syncthreads();
  }
}

// p = r + beta_c p.  The grid's thread count is a multiple of sp, so a thread's column
// stays the same over its grid-stride loop.
__global__ __launch_bounds__(kWG) void k_cg_direction(const double *__restrict__ r,
                                                      double *__restrict__ p,
                                                      const double *__restrict__ beta, int64_t n,
                                                      int sp) {
  const int64_t total = n * sp;
  const int64_t e0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const double be = beta[e0 % sp];
  for (int64_t e = e0; e < total; e += (int64_t)gridDim.x * blockDim.x) p[e] = fma(be, p[e], r[e]);
}

// Column sums of part [nparts][sp], then the per-column CG scalars of `mode` on
// sc = [yy | rr | pq | rrn | alpha | beta] of sp each:
//   mode 0: yy = rr = the sums (start);
//   mode 1: pq = the sums, alpha = rr / pq, and *resmax = 0 for the coming mode 2;
//   mode 2: rrn = the sums, beta = rrn / rr, rr = rrn, and *resmax = max_c rrn / yy over
//           columns with yy > 0, by an integer max on the bit patterns (non-negative
//           doubles order as their bits, and a NaN ends above every finite value).
// Columns with rr = 0 keep alpha = beta = 0.
// The sums are formed as in k_colreduce.
__global__ __launch_bounds__(64 * kColWaves) void k_cg_reduce(const double *__restrict__ part,
                                                              int nparts, int sp,
                                                              double *__restrict__ sc, int mode,
                                                              double *__restrict__ resmax) {
  __shared__ double red[kColPh][kColCols];
  int c;
  const double v = colsum(part, nparts, sp, red, c);
  if (threadIdx.x >= kColCols) return;
  double *yy = sc, *rr = sc + sp, *pq = sc + 2 * sp, *rrn = sc + 3 * sp, *al = sc + 4 * sp,
         *be = sc + 5 * sp;
  if (mode == 1 && blockIdx.x == 0 && threadIdx.x == 0) *resmax = 0.0;
  if (c >= sp) return;
  if (mode == 0) {
    yy[c] = v;
    rr[c] = v;
  } else if (mode == 1) {
    pq[c] = v;
    al[c] = (rr[c] > 0.0 && v != 0.0) ? rr[c] / v : 0.0;
  } else {
    rrn[c] = v;
    be[c] = rr[c] > 0.0 ? v / rr[c] : 0.0;
    rr[c] = v;
    if (yy[c] > 0.0)
      atomicMax(reinterpret_cast<unsigned long long *>(resmax),
                (unsigned long long)__double_as_longlong(v / yy[c]));
  }
}

namespace {
int cg_parts(int64_t n) { return (int)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 63) / 64)); }
}  // namespace

int cg_nparts(int64_t n) { return cg_parts(n); }

hipError_t launch_colreduce(const double *part, int nparts, int sp, double *out, hipStream_t s) {
  hipLaunchKernelGGL(k_colreduce, dim3((sp + kColCols - 1) / kColCols), dim3(64 * kColWaves), 0, s, part,
                     nparts, sp, out);
  return hipGetLastError();
}

hipError_t launch_cg_init(const double *y, double *t, double *r, double *p, int64_t n, int sp,
                          double *part, double *sc, hipStream_t s) {
  if (sp <= 0 || sp % 64 != 0) return hipErrorInvalidValue;
  const int G = cg_parts(n);
  hipLaunchKernelGGL(k_cg_init, dim3(G), dim3(kWG), 0, s, y, t, r, p, n, sp, part);
  hipLaunchKernelGGL(k_cg_reduce, dim3((sp + kColCols - 1) / kColCols), dim3(64 * kColWaves), 0, s, part,
                     G, sp, sc, 0, (double *)nullptr);
  return hipGetLastError();
}

hipError_t launch_cg_alpha(const double *part, int nparts, int sp, double *sc, double *resmax,
                           hipStream_t s) {
  if (sp <= 0 || sp % 64 != 0) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_cg_reduce, dim3((sp + kColCols - 1) / kColCols), dim3(64 * kColWaves), 0, s, part,
                     nparts, sp, sc, 1, resmax);
  return hipGetLastError();
}

hipError_t launch_cg_update(double *t, double *r, double *p, const double *q, int64_t n, int sp,
                            double *part, double *sc, double *resmax, hipStream_t s) {
  if (sp <= 0 || sp % 64 != 0) return hipErrorInvalidValue;
  const int G = cg_parts(n);
  hipLaunchKernelGGL(k_cg_update, dim3(G), dim3(kWG), 0, s, t, r, p, q, sc + 4 * sp, n, sp, part);
  hipLaunchKernelGGL(k_cg_reduce, dim3((sp + kColCols - 1) / kColCols), dim3(64 * kColWaves), 0, s, part,
                     G, sp, sc, 2, resmax);
  // blocks a multiple of sp / 64, so blocks * kWG is a multiple of sp
  const int64_t unit = sp / 64;
  int64_t blocks = (n * sp + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  blocks = (blocks + unit - 1) / unit * unit;
  hipLaunchKernelGGL(k_cg_direction, dim3((unsigned)blocks), dim3(kWG), 0, s, r, p, sc + 5 * sp, n,
                     sp);
  return hipGetLastError();
}

// out = ca A + cb B + cc C + cr r (a null operand or a zero weight adds nothing; r is the
// probe block, sign bits or dense)
__global__ __launch_bounds__(kWG) void k_combine(double *__restrict__ out, double ca, const double *A,
                                                 double cb, const double *B, double cc, const double *C,
                                                 double cr, const uint64_t *__restrict__ sgn,
                                                 const double *__restrict__ rden, int64_t n, int sp) {
  const int64_t total = n * sp;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    double v = 0.0;
    if (A && ca != 0.0) v = fma(ca, A[e], v);
    if (B && cb != 0.0) v = fma(cb, B[e], v);
    if (C && cc != 0.0) v = fma(cc, C[e], v);
    if (cr != 0.0) {
      const int64_t row = e / sp;
      v = fma(cr, probe_value(sgn, rden, row, sp, (int)(e - row * sp)), v);
    }
    out[e] = v;
  }
}

hipError_t launch_combine(double *out, double ca, const double *A, double cb, const double *B, double cc,
                          const double *C, double cr, const uint64_t *sgn, const double *rden, int64_t n,
                          int sp, hipStream_t s) {
  int64_t blocks = (n * sp + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)blocks), dim3(kWG), 0, s, out, ca, A, cb, B, cc, C, cr, sgn,
                     rden, n, sp);
  return hipGetLastError();
}

}  // namespace rfo
