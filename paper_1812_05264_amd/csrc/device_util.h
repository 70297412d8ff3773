// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rfo {

// Workgroups are dispatched round-robin over the 8 XCDs (hardware id b runs on
// XCD b % 8).  Remap so that each XCD owns one contiguous range of logical ids:
// neighbouring rows then share that XCD's L2.
__device__ __forceinline__ int xcd_logical(int b, int nwg) {
  const int per = nwg >> 3, rem = nwg & 7;
  const int xcd = b & 7, idx = b >> 3;
  return xcd < rem ? xcd * (per + 1) + idx : rem * (per + 1) + (xcd - rem) * per + idx;
}

// Persistent schedule of the step kernels over n_pt * n_rg units (probe tile
// pt, row group rg), tile-major.  Workgroup b runs on XCD x = b mod 8; XCD x
// owns the contiguous units [U x/8, U (x+1)/8) and its G/8 workgroups sweep
// them together (unit lo + b/8 + i G/8 at sweep i), so the rows in flight on an
// XCD form a narrow band that moves through the matrix and the neighbour rows
// it gathers are still in that XCD's L2.  A workgroup meets the tiles in
// increasing order, but with a stride above the units per tile it may skip
// some.
// With rev set the XCD's range is swept from its end (unit lo + hi - 1 - i): a
// step that follows one sweeping forward then first reads the rows its
// predecessor touched last, while the memory-side cache still holds them.
struct Sched {
  int64_t i, hi, lo, n_rg;
  int stride;
  bool rev;
  __device__ Sched(int n_pt, int64_t n_rg_, bool rev_ = false) : n_rg(n_rg_), rev(rev_) {
    const int b = blockIdx.x, G = gridDim.x;
    const int x = b & 7;
    const int64_t U = (int64_t)n_pt * n_rg;
    stride = G >> 3;
    lo = U * x / 8;
    i = lo + (b >> 3);
    hi = U * (x + 1) / 8;
  }
  __device__ bool more() const { return i < hi; }
  __device__ void next() { i += stride; }
  __device__ int64_t unit() const { return rev ? lo + hi - 1 - i : i; }
  __device__ int pt() const { return (int)(unit() / n_rg); }
  __device__ int64_t rg() const { return unit() - (int64_t)pt() * n_rg; }
};

template <typename T, int N>
struct alignas(sizeof(T) * N) VecN {
  T v[N];
};

template <typename T, int N>
__device__ __forceinline__ VecN<T, N> zerov() {
  VecN<T, N> r;
#pragma unroll
  for (int q = 0; q < N; ++q) r.v[q] = (T)0;
  return r;
}

template <typename T, int N>
__device__ __forceinline__ VecN<T, N> ldv(const T *p) {
  return *reinterpret_cast<const VecN<T, N> *>(p);
}

template <typename T, int N>
__device__ __forceinline__ void stv(T *p, const VecN<T, N> &v) {
  *reinterpret_cast<VecN<T, N> *>(p) = v;
}

// Streaming (non-temporal) variants for arrays read or written once per pass, so
// that they do not displace gathered rows from the L2.
template <typename T, int N>
__device__ __forceinline__ VecN<T, N> ldv_nt(const T *p) {
  VecN<T, N> r;
  if constexpr (N == 1) {
    r.v[0] = __builtin_nontemporal_load(p);
  } else {
    typedef T V __attribute__((ext_vector_type(N)));
    const V v = __builtin_nontemporal_load(reinterpret_cast<const V *>(p));
#pragma unroll
    for (int q = 0; q < N; ++q) r.v[q] = v[q];
  }
  return r;
}

template <typename T, int N>
__device__ __forceinline__ void stv_nt(T *p, const VecN<T, N> &x) {
  if constexpr (N == 1) {
    __builtin_nontemporal_store(x.v[0], p);
  } else {
    typedef T V __attribute__((ext_vector_type(N)));
    V v;
#pragma unroll
    for (int q = 0; q < N; ++q) v[q] = x.v[q];
    __builtin_nontemporal_store(v, reinterpret_cast<V *>(p));
  }
}

// Probe entry r[row][c]: sign bits (bit 1 = +1, bit 0 = -1) or dense FP64.
__device__ __forceinline__ double probe_value(const uint64_t *sgn, const double *rden,
                                              int64_t row, int sp, int c) {
  if (sgn) {
    const uint64_t w = sgn[row * (sp >> 6) + (c >> 6)];
    return ((w >> (c & 63)) & 1ull) ? 1.0 : -1.0;
  }
  return rden[row * sp + c];
}

// Butterfly sum over the 64 lanes of a wave; every lane gets the total.  The
// pairing order is fixed, so the result is deterministic.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Density accumulator update with the m (1..3) newest terms of the recurrence
// that one pass holds, oldest first: y_{k-1} (p), y_k (x), y_{k+1} (o); al[i]
// is the coefficient of the i-th of those m terms.  Adding them in this order
// gives the same rounding as adding one term per pass.
template <typename VT, int N>
__device__ __forceinline__ VecN<VT, N> add_terms(VecN<VT, N> av, int m, const VT (&al)[3],
                                                 const VecN<VT, N> &p, const VecN<VT, N> &x,
                                                 const VecN<VT, N> &o) {
  int i = 0;
  if (m >= 3) {
#pragma unroll
    for (int q = 0; q < N; ++q) av.v[q] = fma(al[0], p.v[q], av.v[q]);
    i = 1;
  }
  if (m >= 2) {
    const VT c = al[i++];
#pragma unroll
    for (int q = 0; q < N; ++q) av.v[q] = fma(c, x.v[q], av.v[q]);
  }
  const VT c = al[i];
#pragma unroll
  for (int q = 0; q < N; ++q) av.v[q] = fma(c, o.v[q], av.v[q]);
  return av;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// BF16 bits of an FP32 value, rounded to nearest even.
__device__ __forceinline__ unsigned short bf16_bits(float f) {
  __bf16 b = (__bf16)f;
  return __builtin_bit_cast(unsigned short, b);
}

// Load through the constant address space: with a wave-uniform address this
// becomes a scalar (SMEM) load.  Only for data that no kernel of the same launch
// writes.
template <typename T>
__device__ __forceinline__ T sld(const T *p) {
  return *(const __attribute__((address_space(4))) T *)(p);
}

}  // namespace rfo
