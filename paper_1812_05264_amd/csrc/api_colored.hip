// C ABI: the multi-color probe ensemble (paper: Hybrid approximation, the
// multi-color vector ensemble; Implementation details, Welsh-Powell coloring).
//
// rfo_color_atoms colours the atoms so that two atoms closer than the coloring
// radius never share a colour: neighbours come from a cell list of cube side
// r_max (an atom's neighbours lie in its own and the 26 adjacent cells), and the
// Welsh-Powell greedy visits the atoms in order of decreasing degree (ties by
// index), giving each the smallest colour that none of its coloured neighbours
// holds.  rfo_set_colored_probes builds the probe block on the device: column
// k * n_orb + o carries the sign s[a][o] on orbital o of every atom a of colour k
// and zeros elsewhere, with weight one (one sample of the ensemble).
#include <unordered_map>

#include "api_internal.h"

using namespace rfo_api;

namespace {

// rden[(a * n_orb + o) * sp + colour[a] * n_orb + o] = sign[a][o]; the rest of the
// block is cleared beforehand
__global__ __launch_bounds__(256) void k_colored_fill(const int32_t *__restrict__ colour,
                                                      const double *__restrict__ sign, int64_t n_atoms,
                                                      int n_orb, int sp, double *__restrict__ rden) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_atoms * n_orb) return;
  const int64_t a = e / n_orb;
  const int o = (int)(e - a * n_orb);
  rden[e * sp + (int64_t)colour[a] * n_orb + o] = sign[e];
}

}  // namespace

extern "C" {

int rfo_color_atoms(int64_t n_atoms, const double *positions, double r_max, int32_t *colours_out,
                    int32_t *n_colours_out) {
  if (n_atoms < 1 || n_atoms > ((int64_t)1 << 30) || !positions || !colours_out || !n_colours_out ||
      !(r_max > 0.0) || !std::isfinite(r_max))
    return RFO_E_INVALID;
  const int64_t n = n_atoms;
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) lo[d] = hi[d] = positions[d];
  for (int64_t a = 0; a < n; ++a)
    for (int d = 0; d < 3; ++d) {
      const double v = positions[a * 3 + d];
      if (!std::isfinite(v)) return RFO_E_INVALID;
      lo[d] = std::min(lo[d], v);
      hi[d] = std::max(hi[d], v);
    }
  // cell list: cells of side r_max, keyed by their integer coordinates
  int64_t dims[3];
  for (int d = 0; d < 3; ++d) dims[d] = (int64_t)std::floor((hi[d] - lo[d]) / r_max) + 1;
  if ((double)dims[0] * dims[1] * dims[2] > 4e9) return RFO_E_UNSUPPORTED;
  auto cell_of = [&](int64_t a, int64_t *c) {
    for (int d = 0; d < 3; ++d)
      c[d] = std::min(dims[d] - 1, (int64_t)std::floor((positions[a * 3 + d] - lo[d]) / r_max));
  };
  std::unordered_map<int64_t, std::vector<int64_t>> cells;
  cells.reserve((size_t)n);
  for (int64_t a = 0; a < n; ++a) {
    int64_t c[3];
    cell_of(a, c);
    cells[(c[0] * dims[1] + c[1]) * dims[2] + c[2]].push_back(a);
  }
  // neighbour lists (distance < r_max, strictly), each in increasing atom order
  std::vector<int64_t> ptr((size_t)n + 1, 0), idx;
  const double r2 = r_max * r_max;
  for (int64_t a = 0; a < n; ++a) {
    int64_t c[3];
    cell_of(a, c);
    const size_t first = idx.size();
    for (int64_t dx = -1; dx <= 1; ++dx)
      for (int64_t dy = -1; dy <= 1; ++dy)
        for (int64_t dz = -1; dz <= 1; ++dz) {
          const int64_t x = c[0] + dx, y = c[1] + dy, z = c[2] + dz;
          if (x < 0 || y < 0 || z < 0 || x >= dims[0] || y >= dims[1] || z >= dims[2]) continue;
          auto it = cells.find((x * dims[1] + y) * dims[2] + z);
          if (it == cells.end()) continue;
          for (int64_t b : it->second) {
            if (b == a) continue;
            double s = 0.0;
            for (int d = 0; d < 3; ++d) {
              const double t = positions[a * 3 + d] - positions[b * 3 + d];
              s += t * t;
            }
            if (s < r2) idx.push_back(b);
          }
        }
    std::sort(idx.begin() + (std::ptrdiff_t)first, idx.end());
    ptr[(size_t)a + 1] = (int64_t)idx.size();
  }
  // Welsh-Powell: decreasing degree, ties by index; smallest colour free of the
  // coloured neighbours
  std::vector<int64_t> order((size_t)n);
  for (int64_t a = 0; a < n; ++a) order[(size_t)a] = a;
  std::stable_sort(order.begin(), order.end(), [&](int64_t x, int64_t y) {
    return ptr[(size_t)x + 1] - ptr[(size_t)x] > ptr[(size_t)y + 1] - ptr[(size_t)y];
  });
  std::vector<int32_t> colour((size_t)n, -1);
  std::vector<char> taken;
  int32_t q = 0;
  for (int64_t a : order) {
    const int64_t deg = ptr[(size_t)a + 1] - ptr[(size_t)a];
    taken.assign((size_t)deg + 1, 0);
    for (int64_t z = ptr[(size_t)a]; z < ptr[(size_t)a + 1]; ++z) {
      const int32_t cb = colour[(size_t)idx[(size_t)z]];
      if (cb >= 0 && cb <= deg) taken[(size_t)cb] = 1;
    }
    int32_t k = 0;
    while (taken[(size_t)k]) ++k;
    colour[(size_t)a] = k;
    q = std::max(q, k + 1);
  }
  std::copy(colour.begin(), colour.end(), colours_out);
  *n_colours_out = q;
  return RFO_OK;
}

int rfo_set_colored_probes(rfo_ctx *ctx, const int32_t *colours, int n_orb, const double *signs) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  ctx->mom_p = 0;
  ctx->has_dens = false;
  ctx->has_q = false;
  if (!ctx->has_h) return fail(ctx, RFO_E_STATE, "set the Hamiltonian before the probes");
  if (!colours || !signs) return fail(ctx, RFO_E_INVALID, "NULL argument");
  if (n_orb < 1 || ctx->n % n_orb != 0)
    return fail(ctx, RFO_E_INVALID, "n_orb must divide the %lld orbitals", (long long)ctx->n);
  const int64_t n_atoms = ctx->n / n_orb;
  int32_t q = 0;
  for (int64_t a = 0; a < n_atoms; ++a) {
    if (colours[a] < 0) return fail(ctx, RFO_E_INVALID, "negative colour of atom %lld", (long long)a);
    q = std::max(q, colours[a] + 1);
  }
  for (int64_t e = 0; e < n_atoms * n_orb; ++e)
    if (signs[e] != 1.0 && signs[e] != -1.0) return fail(ctx, RFO_E_INVALID, "signs must be +-1");
  const int64_t s = (int64_t)q * n_orb;
  if (s > (1 << 20)) return fail(ctx, RFO_E_INVALID, "too many probe columns");
  HIPCHK(hipSetDevice(ctx->device));
  ctx->has_r = false;
  ctx->has_grad = false;
  const int sp = s <= 64 ? 64 : (int)((s + 127) / 128 * 128);
  const size_t n = (size_t)ctx->n;
  TRY(ensure(ctx, ctx->rden, n * sp * sizeof(double)));
  TRY(ensure(ctx, ctx->w, sp * sizeof(double)));
  struct Staging {
    DevBuf col, sign;
    ~Staging() {
      release(col);
      release(sign);
    }
  } st;
  DevBuf &dcol = st.col, &dsign = st.sign;
  TRY(ensure(ctx, dcol, (size_t)n_atoms * sizeof(int32_t)));
  TRY(ensure(ctx, dsign, n * sizeof(double)));
  HIPCHK(hipMemsetAsync(ctx->rden.p, 0, n * sp * sizeof(double), ctx->stream));
  HIPCHK(hipMemcpyAsync(dcol.p, colours, (size_t)n_atoms * sizeof(int32_t), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipMemcpyAsync(dsign.p, signs, n * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  k_colored_fill<<<(unsigned)((n + 255) / 256), 256, 0, ctx->stream>>>(P<int32_t>(dcol), P<double>(dsign),
                                                                     n_atoms, n_orb, sp, P<double>(ctx->rden));
  HIPCHK(hipGetLastError());
  std::vector<double> w((size_t)sp, 0.0);
  for (int64_t c = 0; c < s; ++c) w[(size_t)c] = 1.0;
  HIPCHK(hipMemcpyAsync(ctx->w.p, w.data(), sp * sizeof(double), hipMemcpyHostToDevice, ctx->stream));
  HIPCHK(hipStreamSynchronize(ctx->stream));
  release(ctx->sgn);
  ctx->signs = false;
  ctx->w_uniform = 1.0;
  ctx->s = s;
  ctx->sp = sp;
  ctx->has_r = true;
  return RFO_OK;
}

}  // extern "C"
