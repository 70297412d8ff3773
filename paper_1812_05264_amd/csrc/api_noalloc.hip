// C ABI: the moment call without device allocation (rfo_fermi_moments_noalloc).
//
// Its work memory (the two vector slots, the moment partials and moments, the
// Chebyshev coefficients and their quadrature tables, the trace results and the
// transposed moments) lives in one file-scope device array, `scratch`, of
// kScratchBytes.  Each device holds its own copy until the process ends; the
// library looks up its address on a device once (hipGetSymbolAddress), the first
// time the call runs there, and from then on passes that address to the
// kernels.  The array's name in host code is a host-side stand-in and is never
// used as a device address.  Every call on a device shares that device's array,
// so calls that overlap on one device (several contexts or host threads) race.
#include <mutex>

#include "api_internal.h"

using namespace rfo_api;

constexpr size_t kScratchBytes = (size_t)128 << 20;  // 128 MiB per device

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};  // device address of `scratch` per device, once resolved

// The device address of the scratch array on ctx's device (which is current).
int scratch_address(rfo_ctx *ctx, char **out) {
  if (ctx->device < 0 || ctx->device >= kMaxDevices)
    return fail(ctx, RFO_E_UNSUPPORTED, "device %d: the scratch table holds %d devices", ctx->device,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[ctx->device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ctx, RFO_E_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch[ctx->device] = p;
  }
  *out = static_cast<char *>(g_scratch[ctx->device]);
  return RFO_OK;
}

// Clears the status flag with a kernel (a fill node, unlike a memset node, replays
// correctly when a caller captures the call in a graph).
__global__ void k_clear_flag(int *flag) {
  if (threadIdx.x == 0) *flag = 0;
}

// moments [p][sp] (internal) -> out [s][p] (the ABI's layout)
__global__ __launch_bounds__(256) void k_moments_to_probe_major(const double *__restrict__ mom,
                                                                int64_t p, int sp, int64_t s,
                                                                double *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= s * p) return;
  const int64_t c = i / p, k = i - c * p;
  out[i] = mom[k * sp + c];
}

size_t round256(size_t b) { return (b + 255) / 256 * 256; }

// The context's work buffers pointed at regions of the scratch array for the
// duration of one call (views: nothing is allocated or freed), and timing off
// (its events would be created on first use).  The destructor restores them.
struct ScratchViews {
  rfo_ctx *c;
  DevBuf vec, ring, moments, coef, samples, costab, small;
  bool timing;
  explicit ScratchViews(rfo_ctx *ctx)
      : c(ctx), vec(ctx->vec), ring(ctx->ring), moments(ctx->moments), coef(ctx->coef),
        samples(ctx->samples), costab(ctx->costab), small(ctx->small), timing(ctx->timing) {
    ctx->timing = false;
  }
  ~ScratchViews() {
    c->vec = vec;
    c->ring = ring;
    c->moments = moments;
    c->coef = coef;
    c->samples = samples;
    c->costab = costab;
    c->small = small;
    c->timing = timing;
  }
};

}  // namespace

extern "C" {

int rfo_fermi_moments_noalloc(rfo_ctx *ctx, double T, double mu, int64_t n_terms,
                              double *moments_out, double *NEF_out) {
  if (!ctx) return RFO_E_INVALID;
  ctx->err.clear();
  TRY(validate_call(ctx, T, mu, n_terms));
  if (ctx->has_s)
    return fail(ctx, RFO_E_UNSUPPORTED, "the allocation-free call does not take an overlap");
  const Plan pl = make_plan(ctx);
  const int64_t p = n_terms, nq = 4 * p;
  const size_t sp = (size_t)ctx->sp;
  // regions of the scratch array, each 256-byte aligned
  const size_t sz_vec = round256(2 * pl.slot_bytes);
  const size_t sz_ring = round256((size_t)pl.ring * pl.grid * sp * sizeof(double));
  const size_t sz_mom = round256((size_t)p * sp * sizeof(double));
  const size_t sz_coef = round256((size_t)3 * p * sizeof(double));
  const size_t sz_samp = round256((size_t)3 * nq * sizeof(double));
  const size_t sz_cos = round256((size_t)4 * nq * sizeof(double));
  const size_t sz_small = round256(64 * sizeof(double));
  const size_t sz_out = round256((size_t)ctx->s * p * sizeof(double));
  const size_t need = sz_vec + sz_ring + sz_mom + sz_coef + sz_samp + sz_cos + sz_small + sz_out;
  if (need > kScratchBytes)
    return fail(ctx, RFO_E_INVALID,
                "this call needs %zu bytes of work memory; the allocation-free call has %zu "
                "(use rfo_fermi_moments)", need, kScratchBytes);
  char *base = nullptr;
  TRY(scratch_address(ctx, &base));

  ScratchViews views(ctx);
  size_t off = 0;
  auto take = [&](DevBuf &b, size_t bytes) {
    b.p = base + off;
    b.bytes = bytes;
    off += bytes;
  };
  take(ctx->vec, sz_vec);
  take(ctx->ring, sz_ring);
  take(ctx->moments, sz_mom);
  take(ctx->coef, sz_coef);
  take(ctx->samples, sz_samp);
  take(ctx->costab, sz_cos);
  take(ctx->small, sz_small);
  double *mom_out_dev = reinterpret_cast<double *>(base + off);

  k_clear_flag<<<1, 64, 0, ctx->stream>>>(P<int>(ctx->flags));
  HIPCHK(hipGetLastError());
  HIPCHK(rfo::launch_coefficients(ctx->e_min, ctx->e_max, T, mu, p, nq, P<double>(ctx->samples),
                                  P<double>(ctx->costab), P<double>(ctx->coef), ctx->stream));
  size_t n_events = 0;
  TRY(run_forward(ctx, pl, p, ctx->vec, false, nullptr, &n_events, ctx->doubling));
  double *obs = P<double>(ctx->small);
  HIPCHK(rfo::launch_traces(P<double>(ctx->moments), P<double>(ctx->w), P<double>(ctx->coef), p,
                            ctx->sp, obs, ctx->stream));
  TRY(copy_out(ctx, NEF_out, obs, 3 * sizeof(double)));
  if (moments_out) {
    const int64_t total = ctx->s * p;
    k_moments_to_probe_major<<<(unsigned)((total + 255) / 256), 256, 0, ctx->stream>>>(
        P<double>(ctx->moments), p, ctx->sp, ctx->s, mom_out_dev);
    HIPCHK(hipGetLastError());
    TRY(copy_out(ctx, moments_out, mom_out_dev, (size_t)total * sizeof(double)));
  }
  TRY(check_flags_and_finish(ctx, 0));
  // the moments stay in the shared scratch array, which the next call may overwrite
  ctx->mom_p = 0;
  return RFO_OK;
}

}  // extern "C"
