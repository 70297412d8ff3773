// BF16 Chebyshev step for 9x9 blocks on the matrix cores (gfx950 MFMA).
//
// The block product Y_I = sum_J H_hat_IJ X_J is a dense 9x9 times 9 x (probes)
// contraction per stored block (paper: block-sparse 9x9 matrix-vector work of
// the Chebyshev recursion), so it maps onto CDNA4's v_mfma_f32_16x16x32_bf16:
//   A (16 x 32, M x K) = H_hat_I* on 32 K rows, rows 9..15 zero;
//   B (32 x 16, K x N) = 32 gathered rows of the X_J for 16 probe columns;
//   D (16 x 16)        = FP32 accumulator of Y_I (rows 0..8 used).
// Lane l supplies A[l%16][8(l/16)+kk], B[8(l/16)+kk][l%16] for kk < 8 and holds
// D[4(l/16)+i][l%16] for i < 4 (checked on the device).  A wave covers 16*NT
// probes as NT MFMA tiles;
// column n of tile t is probe p0 + n*NT + t, so a lane reads and writes NT
// consecutive probes of a row with one vector access.  Operands are BF16 (round
// to nearest even); accumulation, the recurrence out = c1 D + c2 prev + beta r
// and the vectors stay FP32; moments are FP64.  Every FP32 vector has a BF16
// copy (rounded the same way) that its producer writes beside it: the gathered
// B operands come from that copy, half the bytes of the FP32 rows, and only
// the nine real rows of X_J are loaded (lanes of rows 9..15 load nothing).
//
// K is packed across the blocks of a block row: Y_I = [H_IJ1 H_IJ2 ...] [X_J1; X_J2; ...]
// is one (9) x (9 nblk) times (9 nblk) x (probes) product, cut into chunks of
// kKChunk = 32 K rows, so that every K row of an MFMA is a real row of some X_J
// (only the last chunk of a row has zero rows, which load nothing).  Per chunk,
// kc_idx lists the 32 gathered rows J*9 + c and the A operands are pre-packed:
// entry g*9 + m (m < 9) holds the eight BF16 values H_hat_IJ[m][c] of K rows
// 8g .. 8g+7; lanes with m > 8 supply zeros.
#include "device_util.h"
#include "rfo_internal.h"

namespace rfo {

namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef int i4 __attribute__((ext_vector_type(4)));

}  // namespace

// Occupancy 4 (at most 128 registers) is part of the design: the step is bound by
// the gathers each wave keeps in flight, and at occupancy 3 the same kernel is
// much slower.
template <int NT, int U, bool NTH, int MODE, bool SPLIT, bool PAD>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) void k_step9_bf16(
    StepArgs a) {
  constexpr int TW = 16 * NT;  // probes per wave (tile width)
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int g = lane >> 4, n = lane & 15;
  const int sp = a.sp;
  const int nw = sp >> 6;
  const int s_live = a.s_live > 0 ? a.s_live : sp;
  const float *__restrict__ x = static_cast<const float *>(a.x);
  const unsigned short *__restrict__ xb = static_cast<const unsigned short *>(a.xb);
  const float *prev = static_cast<const float *>(a.prev);
  float *out = static_cast<float *>(a.out);
  unsigned short *outb = static_cast<unsigned short *>(a.outb);
  float *acc = static_cast<float *>(a.acc);
  // SPLIT: each pack entry is followed by the low BF16 parts of its eight values
  const uint4 *hpack = static_cast<const uint4 *>(a.hval);
  const i4 *kidx = reinterpret_cast<const i4 *>(a.kc_idx);
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
  const float *srcp[3];
  float srw[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    srcp[t] = t < nsrc ? static_cast<const float *>(a.src[t]) : nullptr;
    srw[t] = t < nsrc ? (float)a.srcw[t] : 0.f;
  }
  float al[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) al[i] = i < m ? (float)sld(a.alpha + i) : 0.f;
  const float c1 = (float)a.c1, c2 = (float)a.c2;
  __shared__ double red[kWaves][4][TW];
  double *prow = mom_on ? a.part + (int64_t)blockIdx.x * sp : nullptr;

  double mom[NT], mom2[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) mom[t] = mom2[t] = 0.0;
  int cur_pt = -1;
  double *prow2 = DBL && mom_on ? a.part2 + (int64_t)blockIdx.x * sp : nullptr;
  // every tile's partials start at zero (a workgroup may skip tiles); the
  // tiles it meets are overwritten by flush
  if (mom_on && wave == 0)
    for (int t = 0; t < a.n_pt; ++t)
      for (int c = lane; c < TW; c += 64) {
        prow[(int64_t)t * TW + c] = 0.0;
        if (DBL) prow2[(int64_t)t * TW + c] = 0.0;
      }

  auto flush1 = [&](double(&mm)[NT], double *dst, int pt) {
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      red[wave][g][n * NT + t] = mm[t];
      mm[t] = 0.0;
    }
    __syncthreads();
    if (wave == 0) {
      for (int c = lane; c < TW; c += 64) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < kWaves; ++w)
#pragma unroll
          for (int gg = 0; gg < 4; ++gg) s += red[w][gg][c];
        dst[(int64_t)pt * TW + c] = s;
      }
    }
    __syncthreads();
  };
  auto flush = [&](int pt) {
    flush1(mom, prow, pt);
    if (DBL) flush1(mom2, prow2, pt);
  };

  for (Sched sc(a.n_pt, a.n_rg, a.reverse != 0); sc.more(); sc.next()) {
    const int pt = sc.pt();
    const int64_t rg = sc.rg();
    if (pt != cur_pt) {
      if (mom_on && cur_pt >= 0) flush(cur_pt);
      cur_pt = pt;
    }
    const int cp = pt * TW + n * NT;  // first probe column of this lane
    // PAD: a lane whose probes are all zero padding loads nothing (its inputs are
    // zero); without padding columns the predicate is compiled out
    const bool live = !PAD || cp < s_live;
    const int64_t r0 = rg * a.rows_per_wg;
    const int64_t r1 = min(a.nb, r0 + (int64_t)a.rows_per_wg);
    for (int64_t I = r0 + wave; I < r1; I += kWaves) {
      f4 d[NT];
#pragma unroll
      for (int t = 0; t < NT; ++t) d[t] = f4{0.f, 0.f, 0.f, 0.f};
      const int64_t q0 = sld(a.kc_ptr + I), q1 = sld(a.kc_ptr + I + 1);
      for (int64_t qc = q0; qc < q1; qc += U) {
        bf8 av[U], avl[U];
        VecN<unsigned short, NT> xr[U][8];
        const bool a_live = n < 9;
        const int a_idx = a_live ? g * 9 + n : 0;
        const uint4 zero4 = make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t q = min(qc + u, q1 - 1);  // a repeated chunk is not accumulated
          // every lane loads (a_idx is valid), then lanes of rows 9..15 take zeros
          const int64_t e = q * 36 + a_idx;
          const uint4 ph = hpack[SPLIT ? 2 * e : e];
          av[u] = __builtin_bit_cast(bf8, a_live ? ph : zero4);
          if constexpr (SPLIT) {
            const uint4 pl = hpack[2 * e + 1];
            avl[u] = __builtin_bit_cast(bf8, a_live ? pl : zero4);
          }
          // the chunk's 32 source rows (wave-uniform), eight per lane group
          i4 kq[8];
#pragma unroll
          for (int h = 0; h < 8; ++h) kq[h] = sld(kidx + q * 8 + h);
          const i4 ka = g == 0 ? kq[0] : (g == 1 ? kq[2] : (g == 2 ? kq[4] : kq[6]));
          const i4 kb = g == 0 ? kq[1] : (g == 1 ? kq[3] : (g == 2 ? kq[5] : kq[7]));
          const int src[8] = {ka.x, ka.y, ka.z, ka.w, kb.x, kb.y, kb.z, kb.w};
#pragma unroll
          for (int kk = 0; kk < 8; ++kk) {
            if (src[kk] >= 0 && live) {
              xr[u][kk] = ldv<unsigned short, NT>(xb + (int64_t)src[kk] * sp + cp);
            } else {
#pragma unroll
              for (int t = 0; t < NT; ++t) xr[u][kk].v[t] = 0;
            }
          }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (qc + u < q1) {
#pragma unroll
            for (int t = 0; t < NT; ++t) {
              VecN<unsigned short, 8> b;
#pragma unroll
              for (int kk = 0; kk < 8; ++kk) b.v[kk] = xr[u][kk].v[t];
              const bf8 bv = __builtin_bit_cast(bf8, b);
              // the low part first: the two products add in FP32 as (lo + hi) y
              if constexpr (SPLIT) d[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(avl[u], bv, d[t], 0, 0, 0);
              d[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[u], bv, d[t], 0, 0, 0);
            }
          }
        }
      }
      // epilogue: lane holds rows 4g+i (valid below 9) for probes cp .. cp+NT-1.
      // The streamed inputs are loaded row by row: requesting all four rows first
      // holds more registers and measured slower (occupancy 3 instead of 4).
      constexpr int NPRE = 1;
      VecN<float, NT> pv4[NPRE], xs4[NPRE];
      uint64_t sw4[NPRE];
      auto load_row = [&](int i, int slot) {
        const int64_t row = I * 9 + min(4 * g + i, 8);
        if (has_prev)
          pv4[slot] = !live ? zerov<float, NT>()
                            : NTH ? ldv_nt<float, NT>(prev + row * sp + cp) : ldv<float, NT>(prev + row * sp + cp);
        // the row's own FP32 y_k is read once: non-temporal, so that it does not
        // displace the gathered BF16 copies (measured 4% faster)
        if (m >= 2 || DBL) xs4[slot] = live ? ldv_nt<float, NT>(x + row * sp + cp) : zerov<float, NT>();
        if (need_r && a.sgn) sw4[slot] = a.sgn[row * nw + (cp >> 6)];
      };
      if constexpr (NPRE == 4) {
#pragma unroll
        for (int i = 0; i < 4; ++i) load_row(i, i);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = 4 * g + i;
        if (rr >= 9) continue;
        const int si = NPRE == 4 ? i : 0;
        if constexpr (NPRE == 1) load_row(i, 0);
        const int64_t row = I * 9 + rr;
        const int64_t off = row * sp + cp;
        const VecN<float, NT> pv = pv4[si];
        const uint64_t sw = sw4[si];
        VecN<float, NT> sv[3];
        if (SRC) {
#pragma unroll
          for (int t = 0; t < 3; ++t)
            if (t < nsrc) sv[t] = live ? ldv_nt<float, NT>(srcp[t] + off) : zerov<float, NT>();
        }
        VecN<double, NT> rv;
        if (need_r && !a.sgn) rv = live ? ldv<double, NT>(a.rden + off) : zerov<double, NT>();
        VecN<float, NT> o;
#pragma unroll
        for (int t = 0; t < NT; ++t) {
          double rq = 0.0;
          if (need_r) rq = a.sgn ? (((sw >> ((cp + t) & 63)) & 1ull) ? 1.0 : -1.0) : rv.v[t];
          float v = c1 * d[t][i];
          if (has_prev) v = fmaf(c2, pv.v[t], v);
          if (add_r) v = (float)((double)v + beta * rq);
          if (SRC) {
#pragma unroll
            for (int tt = 0; tt < 3; ++tt)
              if (tt < nsrc) v = fmaf(srw[tt], sv[tt].v[t], v);
          }
          o.v[t] = v;
          if (mom_on) {
            if (DBL) {
              mom[t] = fma((double)v, (double)v, mom[t]);
              mom2[t] = fma((double)v, (double)xs4[si].v[t], mom2[t]);
            } else {
              mom[t] = fma(rq, (double)v, mom[t]);
            }
          }
        }
        if (NTH) stv_nt<float, NT>(out + off, o);
        else stv<float, NT>(out + off, o);
        VecN<unsigned short, NT> ob;
#pragma unroll
        for (int t = 0; t < NT; ++t) ob.v[t] = bf16_bits(o.v[t]);
        stv<unsigned short, NT>(outb + off, ob);
        if (m > 0) {
          VecN<float, NT> avv = !live ? zerov<float, NT>() : NTH ? ldv_nt<float, NT>(acc + off) : ldv<float, NT>(acc + off);
          avv = add_terms<float, NT>(avv, m, al, pv, xs4[si], o);
          if (NTH) stv_nt<float, NT>(acc + off, avv);
          else stv<float, NT>(acc + off, avv);
        }
      }
    }
  }
  if (mom_on) {
    if (cur_pt >= 0) flush(cur_pt);
  }
}

// ---------------------------------------------------------------------------
// Segment gradient on the matrix cores (Analytical free-energy derivatives,
// polynomial form: G_IJ accumulates z_{j+1,I} y_{j,J}^T over the steps and the
// probes, here symmetrized), for the BF16 steps: it reads the BF16 copies of the
// segment's vectors (the operands the steps gather).  For a block (I, J) the sum
// over the probes c is a 9 x K by K x 9 contraction, K = the probes, on
// v_mfma_f32_16x16x32_bf16: A = X_I (M = the 9 rows, padded to 16), B = Y_J^T
// (N = the 9 rows of Y_J).  One wave owns a group of upper blocks of one block
// row, so X_I and Y_I are loaded once for all of them; each block keeps a 16 x 16
// FP32 tile (4 registers per lane), flushed into FP64 sums after every step t.
// Lane l supplies A[l%16][8(l/16)..+7] and B[8(l/16)..+7][l%16] and holds
// D[4(l/16)+i][l%16] (layout checked on the device); a lane loads 8 consecutive
// probes of a row with one 16-byte access, which are its eight K slots as they
// stand, the same probes in A and B.  Four waves per SIMD requested from the
// compiler (no spills; the default took three waves).
// ---------------------------------------------------------------------------
template <int GB>
__global__ __launch_bounds__(kWG) __attribute__((amdgpu_waves_per_eu(4))) void k_sddmm_bf16(SddmmMfmaArgs a) {
  constexpr int P = 8;  // probes per lane per load (16 bytes of BF16)
  const int wave = uniform(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  const int64_t gi = (int64_t)xcd_logical(blockIdx.x, gridDim.x) * kWaves + wave;
  if (gi >= a.n_grp) return;
  const int64_t q0 = sld(a.grp + gi), q1 = sld(a.grp + gi + 1);
  const int nb = (int)(q1 - q0);
  const int m = lane & 15, kq = lane >> 4;
  const bool live = m < 9;
  int64_t nzs[GB], js[GB];
#pragma unroll
  for (int g = 0; g < GB; ++g) {
    nzs[g] = sld(a.nzlist + (g < nb ? q0 + g : q0));
    js[g] = sld(a.col + nzs[g]);
  }
  const int64_t I = sld(a.brow + nzs[0]);
  const int sp = a.sp;
  double acc[GB][4];
#pragma unroll
  for (int g = 0; g < GB; ++g)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[g][r] = 0.0;

  for (int t = 0; t < a.count; ++t) {
    f4 d[GB];
#pragma unroll
    for (int g = 0; g < GB; ++g) d[g] = f4{0.f, 0.f, 0.f, 0.f};
    for (int c0 = 0; c0 < sp; c0 += 4 * P) {
      const int cp = c0 + kq * P;
      // A operands X_I, Y_I (zero rows 9..15 and zero probes past s_real)
      {
        const unsigned short *X = static_cast<const unsigned short *>(a.xbase) + (int64_t)t * a.xstride;
        const unsigned short *Y = static_cast<const unsigned short *>(a.ybase) + (int64_t)t * a.ystride;
        VecN<unsigned short, 8> xa, ya;
        if (live) {
          xa = ldv<unsigned short, 8>(X + (I * 9 + m) * sp + cp);
          ya = ldv<unsigned short, 8>(Y + (I * 9 + m) * sp + cp);
        } else {
#pragma unroll
          for (int e = 0; e < 8; ++e) xa.v[e] = ya.v[e] = 0;
        }
#pragma unroll
        for (int e = 0; e < 8; ++e)
          if (cp + e >= a.s_real) xa.v[e] = ya.v[e] = 0;
        // the blocks of the group one at a time: loading all of them before the
        // MFMAs lowers the occupancy and measured slower (11.6 against 6.4 ms per
        // 20-step cu16k segment with groups of 6)
#pragma unroll
        for (int g = 0; g < GB; ++g) {
          if (g < nb) {
            VecN<unsigned short, 8> yj, xj;
            if (live) {
              yj = ldv<unsigned short, 8>(Y + (js[g] * 9 + m) * sp + cp);
              xj = ldv<unsigned short, 8>(X + (js[g] * 9 + m) * sp + cp);
            } else {
#pragma unroll
              for (int e = 0; e < 8; ++e) yj.v[e] = xj.v[e] = 0;
            }
            d[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, xa),
                                                           __builtin_bit_cast(bf8, yj), d[g], 0, 0, 0);
            d[g] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf8, ya),
                                                           __builtin_bit_cast(bf8, xj), d[g], 0, 0, 0);
          }
        }
      }
    }
    const double coef = a.scale * a.w0 * ((a.j0 + t == 0) ? a.first : a.rest);
#pragma unroll
    for (int g = 0; g < GB; ++g)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[g][r] = fma(coef, (double)d[g][r], acc[g][r]);
  }
  // lane holds G_IJ[4 kq + r][m] of every block of the group
#pragma unroll
  for (int g = 0; g < GB; ++g) {
    if (g < nb) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = 4 * kq + r;
        if (row < 9 && live) {
          double *gp = a.G + nzs[g] * 81 + row * 9 + m;
          *gp = a.accumulate ? *gp + acc[g][r] : acc[g][r];
        }
      }
    }
  }
}

hipError_t launch_sddmm_bf16(const SddmmMfmaArgs &a, hipStream_t s) {
  if (a.n_grp == 0) return hipSuccess;
  if (a.sp % 32 != 0) return hipErrorInvalidValue;  // 32 probes per load round of a wave
  const dim3 grid((unsigned)((a.n_grp + kWaves - 1) / kWaves));
  hipLaunchKernelGGL((k_sddmm_bf16<kSddmmGroup>), grid, dim3(kWG), 0, s, a);
  return hipGetLastError();
}

// Pack H_hat (FP64 [nnzb][9][9]) into the chunked A-operand layout above: entry
// e = 36 q + 9 g + m holds the eight BF16 values of K rows 8g .. 8g+7 of chunk q
// for output row m (one uint4).  With split, entry e takes two uint4: the BF16
// values hi = bf16(h) and then lo = bf16(h - hi) (h the FP64 entry; hi + lo
// carries about 16 significant bits).
__global__ __launch_bounds__(kWG) void k_pack_bf16(const double *__restrict__ hhat,
                                                   const int32_t *__restrict__ kc_src,
                                                   int64_t n_chunks, int split,
                                                   uint4 *__restrict__ apack) {
  const int64_t total = n_chunks * 36;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t q = e / 36;
    const int r = (int)(e - q * 36);
    const int gg = r / 9, m = r - gg * 9;
    unsigned v[8], vl[8];
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int code = kc_src[q * kKChunk + 8 * gg + kk];
      const double h = code >= 0 ? hhat[(int64_t)(code / 9) * 81 + m * 9 + code % 9] : 0.0;
      v[kk] = bf16_bits((float)h);
      const double hi = (double)__builtin_bit_cast(float, v[kk] << 16);
      vl[kk] = bf16_bits((float)(h - hi));
    }
    const uint4 hi4 = make_uint4(v[0] | (v[1] << 16), v[2] | (v[3] << 16), v[4] | (v[5] << 16),
                                 v[6] | (v[7] << 16));
    if (split) {
      apack[2 * e] = hi4;
      apack[2 * e + 1] = make_uint4(vl[0] | (vl[1] << 16), vl[2] | (vl[3] << 16), vl[4] | (vl[5] << 16),
                                    vl[6] | (vl[7] << 16));
    } else {
      apack[e] = hi4;
    }
  }
}

namespace {

template <bool SPLIT, bool PAD>
const void *select_bf16_t(int nt_tiles, int u, int mode) {
#define RFO_BF16_CASE(T, UU)                                                        \
  if (nt_tiles == T && u == UU)                                                     \
    return mode == 1   ? (const void *)k_step9_bf16<T, UU, true, 1, SPLIT, PAD>     \
           : mode == 2 ? (const void *)k_step9_bf16<T, UU, true, 2, SPLIT, PAD>     \
           : mode == 3 ? (const void *)k_step9_bf16<T, UU, true, 3, SPLIT, PAD>     \
                       : (const void *)k_step9_bf16<T, UU, true, 0, SPLIT, PAD>;
  RFO_BF16_CASE(4, 1)
  RFO_BF16_CASE(4, 2)
#undef RFO_BF16_CASE
  return nullptr;
}

const void *select_bf16(int nt_tiles, int u, int mode, int split, bool pad) {
  if (pad) return split ? select_bf16_t<true, true>(nt_tiles, u, mode) : select_bf16_t<false, true>(nt_tiles, u, mode);
  return split ? select_bf16_t<true, false>(nt_tiles, u, mode) : select_bf16_t<false, false>(nt_tiles, u, mode);
}

}  // namespace

int step_bf16_blocks_per_cu(int nt_tiles, int u, int split) {
  const void *f = select_bf16(nt_tiles, u, 0, split, false);
  if (!f) return 0;
  int nblk = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nblk, f, kWG, 0) != hipSuccess) return 0;
  return nblk;
}

hipError_t launch_step_bf16(int nt_tiles, const StepArgs &a, hipStream_t s) {
  const void *f = select_bf16(nt_tiles, a.rpi, step_mode(a), a.hsplit, a.s_live > 0 && a.s_live < a.sp);
  if (!f || a.grid < 8 || (a.grid & 7)) return hipErrorInvalidValue;
  void *args[] = {const_cast<StepArgs *>(&a)};
  return hipLaunchKernel(f, dim3((unsigned)a.grid), dim3(kWG), args, 0, s);
}

hipError_t launch_pack_bf16(const double *hhat, const int32_t *kc_src, int64_t n_chunks, int split,
                            void *apack, hipStream_t s) {
  if (n_chunks == 0) return hipSuccess;
  int64_t blocks = (n_chunks * 36 + kWG - 1) / kWG;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_pack_bf16, dim3((unsigned)blocks), dim3(kWG), 0, s, hhat, kc_src, n_chunks, split,
                     static_cast<uint4 *>(apack));
  return hipGetLastError();
}

}  // namespace rfo
