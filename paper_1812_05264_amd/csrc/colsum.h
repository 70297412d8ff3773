// Fixed-order column reduction shared by the conjugate-gradient (overlap) and CGLS
// (rational) kernels.
#pragma once

#include "device_util.h"

namespace rfo {

// Fixed-order column sums of part [nparts][sp] for a workgroup of 64 * kColWaves
// threads that owns the kColCols columns from blockIdx.x * kColCols: lane l of wave w
// adds, for column l % kColCols, the rows h, h + kColPh, ... of phase
// h = w * (64 / kColCols) + l / kColCols in increasing order, and the kColPh phase sums
// are then added in phase order, so the result is bitwise reproducible.  Many short
// chains rather than a few long ones: the partials come from other XCDs' caches, and
// the latency of each dependent round of loads sets the time.  Every thread of the
// workgroup must call it (it has a barrier); the sum of column c (returned in c) is
// returned to the threads with threadIdx.x < kColCols, zero to the others.
constexpr int kColWaves = 16, kColCols = 16, kColPh = kColWaves * (64 / kColCols);

__device__ __forceinline__ double colsum(const double *__restrict__ part, int nparts, int sp,
                                         double (*red)[kColCols], int &c) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int cl = lane % kColCols, ph = wave * (64 / kColCols) + lane / kColCols;
  c = blockIdx.x * kColCols + cl;
  double s = 0.0;
  if (c < sp) {
#pragma unroll 4
    for (int b = ph; b < nparts; b += kColPh) s += part[(int64_t)b * sp + c];
  }
  red[ph][cl] = s;
  __syncthreads();
  if (threadIdx.x >= kColCols) return 0.0;
  double t = red[0][cl];
  for (int h = 1; h < kColPh; ++h) t += red[h][cl];
  return t;
}

}  // namespace rfo
