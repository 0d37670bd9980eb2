// The plain device-pointer evaluation for callers that cannot allocate
// device memory: the strengths are staged in a static device array of the
// library instead of the geometry's staging buffer, and nothing is allocated
// by the call.  One array per GPU (each device that loads the library holds
// its own copy until the process ends); every call on a GPU shares it.
#include <mutex>

#include "tsqbx_internal.h"

namespace {

constexpr size_t kScratchBytes = TSQBX_NOALLOC_SCRATCH_BYTES;
static_assert(kScratchBytes % 256 == 0, "scratch size");

// The staging of tsqbx_eval_async_noalloc: positions and strengths at offset
// 0, strength-weighted normals after them (SourceStage layout).
static __device__ __align__(256) char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_addr[kMaxDevices] = {};  // device address of each GPU's copy

size_t align256(size_t b) { return (b + 255) / 256 * 256; }

struct Guard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit Guard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~Guard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

}  // namespace

namespace tsqbx {

// The device address of this GPU's scratch array, looked up once per device
// (with that device current) and kept; called by tsqbx_ctx_create.  The
// array's name is only a host-side stand-in: kernels and copies must use the
// address this returns.
hipError_t noalloc_scratch_init(int device, void **out) {
  *out = nullptr;
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_addr[device]) {
    Guard g(device);
    if (g.err != hipSuccess) return g.err;
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    scratch_addr[device] = p;
  }
  *out = scratch_addr[device];
  return hipSuccess;
}

}  // namespace tsqbx

using namespace tsqbx;

extern "C" int tsqbx_eval_async_noalloc(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p,
                                        unsigned layers, const double *d_sigma,
                                        double *d_out_slp, double *d_out_dlp,
                                        double *d_out_sprime, unsigned flags,
                                        void *hip_stream) {
  TraceRange trace_("tsqbx_eval_async_noalloc");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = tsqbx_check_request(g, p, layers);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !d_sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  if (g->n_targets > 0 && (((layers & TSQBX_SLP) && !d_out_slp) ||
                           ((layers & TSQBX_DLP) && !d_out_dlp) ||
                           ((layers & TSQBX_SPRIME) && !d_out_sprime)))
    return fail(TSQBX_E_INVALID, "output for a requested layer is NULL");
  const int64_t N = g->n_sources;
  const size_t pos = align256(stage_pos_bytes(N));
  const size_t need = pos + ((layers & TSQBX_DLP) ? stage_nrm_bytes(N) : 0);
  if (need > kScratchBytes)
    return fail(TSQBX_E_RANGE,
                "eval_async_noalloc: %lld sources need %zu bytes of staging, more than the "
                "%zu-byte scratch array",
                (long long)N, need, kScratchBytes);
  if (!ctx->scratch) return fail(TSQBX_E_STATE, "eval_async_noalloc: no scratch array on this device");
  Guard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  char *base = (char *)ctx->scratch;
  const SourceStage st = stage_views(base, (layers & TSQBX_DLP) ? base + pos : nullptr, N);
  const int64_t mean = g->n_targets > 0 ? (g->pairs + g->n_targets - 1) / g->n_targets : 0;
  const Tuning tn = lookup_tuning(ctx, p, layers, mean);
  Outputs o;
  o.s = d_out_slp;
  o.d = d_out_dlp;
  o.t = d_out_sprime;
  hipStream_t s = (hipStream_t)hip_stream;
  TSQBX_HIP(launch_stage(g, d_sigma, layers, st, false, s));
  TSQBX_HIP(launch_eval_plain(g, p, layers, st, o, (flags & TSQBX_ACCUMULATE) != 0, tn,
                              (flags & TSQBX_PER_TARGET) != 0, s));
  return TSQBX_OK;
}
