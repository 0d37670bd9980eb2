// Serving: evaluation requests against device-resident geometries, admitted
// under a device-memory budget and batched continuously.
//
// submit() copies the density into a pinned host arena (pageable memory if
// that arena is full).  The scheduler (tsqbx_sched.h) admits queued requests
// in FIFO order while their buffers fit in the budget (one device arena of
// exactly that size) and a request slot is free; this file is its device
// executor, which launches everything admitted together as one step: density
// uploads, one staging kernel and one persistent kernel over the step's work
// units, then output downloads into pinned memory.  Up to kStreams steps are
// in flight on separate streams, so requests that arrive while a step runs
// are launched in the next step and overlap with it on the device.  When a
// step's event has fired, the executor copies the outputs to the callers'
// buffers and the scheduler releases the memory.  Every request is summed by the same device
// routine with the same group width whatever it is batched with, so its
// result does not depend on the mix.  Helmholtz requests (complex density and
// outputs) share the steps: their densities are uploaded by DMA and they get
// their own staging, table and persistent launches in the step.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <tuple>
#include <vector>

#include "tsqbx_internal.h"
#include "tsqbx_sched.h"

using namespace tsqbx;

namespace {

constexpr int kStreams = 4;
constexpr int kUnitSteps = 8;  // default wave-steps (group_lanes-wide passes) per unit
// Requests per step: small enough that the next step's density reads (PCIe)
// overlap this step's evaluation on another stream, large enough to amortise
// the step's launches.
constexpr int kMaxStepRequests = 32;  // the default
constexpr int64_t kNoDma = int64_t(1) << 40;  // no density is uploaded by DMA
// By default no density goes up by DMA: the staging kernel reads pinned
// densities over PCIe.  DMA for the larger geometries raises the saturation
// rate of the serving mix (about 58k-61k against 52k requests/s with a
// threshold of 32768 sources) but makes it vary from run to run (45k-60k at
// 131072) and raises the p99 latency under Poisson load (3-5 ms against
// about 1 ms at 0.7x saturation): the copies of one step queue on the copy
// engines ahead of the next step's.  It stays a tuning the caller chooses.
constexpr int64_t kDmaMinSources = kNoDma;
constexpr size_t kAlign = 256;
// Completed requests whose status stays queryable (poll, wait); older ones
// are forgotten, so that a long-running server holds bounded host memory.
constexpr size_t kKeepDone = 4096;
// Latency percentiles cover the most recent completions, at most this many.
constexpr size_t kLatWindow = 65536;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request : Job {
  const tsqbx_geometry *geom = nullptr;
  int p = 0;
  unsigned layers = 0;
  double k = 0.0;                   // > 0: a Helmholtz request (complex values)
  size_t cw() const { return k > 0.0 ? 2 : 1; }  // doubles per value
  // host staging: [sigma (N) | one T-vector per requested layer, in the order
  // single layer, double layer, S'], pinned when it fits
  double *h_stage = nullptr;
  bool pinned = false;
  bool borrowed = false;            // caller's pinned buffers, no staging
  const double *sigma_src = nullptr;  // what the upload reads
  size_t pin_off = 0, pin_bytes = 0;
  std::vector<double> pageable;  // fallback staging
  double *out[3] = {nullptr, nullptr, nullptr};  // caller's outputs per layer
};

struct StreamSlot {
  hipStream_t s = nullptr;
  hipEvent_t ev = nullptr;
  bool busy = false;
  // the step's work items, staging items, copy items, units and wave ranges:
  // one pinned host block and its device copy (grown on demand)
  char *h_meta = nullptr, *d_meta = nullptr;
  size_t cap_meta = 0;
};

}  // namespace

// The server is the scheduler's device executor.
struct tsqbx_server final : public Executor {
  tsqbx_ctx *ctx = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_slots = 1;
  // launch shape and step shape, fixed once a caller's request has been
  // submitted (a request's bits depend on the group width only)
  Tuning tn;
  int unit_steps = kUnitSteps;
  int step_requests = kMaxStepRequests;
  int64_t dma_min_sources = kDmaMinSources;
  std::atomic<bool> used{false};
  char *arena_base = nullptr;
  char *pinned_base = nullptr;  // pinned host arena for densities and outputs
  size_t pinned_cap = 0;
  Arena pinned;
  std::mutex pinned_mu;
  StreamSlot strm[kStreams];
  std::unique_ptr<Scheduler> sched;

  int streams() const override { return kStreams; }
  void thread_start() override { (void)hipSetDevice(device); }
  int launch(int stream, const std::vector<Job *> &jobs, std::string &err) override;
  int query(int stream) override {
    const hipError_t q = hipEventQuery(strm[stream].ev);
    if (q == hipSuccess) return 1;
    return q == hipErrorNotReady ? 0 : TSQBX_E_DEVICE;
  }
  void sync(int stream) override { (void)hipStreamSynchronize(strm[stream].s); }
  // Outputs staged in the request's host buffer go to the caller's buffers.
  int finish(Job *job, int step_status) override {
    if (step_status != TSQBX_OK) return TSQBX_E_DEVICE;
    Request *r = static_cast<Request *>(job);
    const size_t N = (size_t)r->geom->n_sources, T = (size_t)r->geom->n_targets;
    const size_t cw = r->cw();
    if (!r->borrowed && T) {
      const double *h = r->h_stage + cw * N;
      for (int l = 0; l < 3; ++l)
        if (r->layers & (1u << l)) {
          std::memcpy(r->out[l], h, cw * T * sizeof(double));
          h += cw * T;
        }
    }
    return TSQBX_OK;
  }
  SchedLimits limits() const {
    SchedLimits lim;
    lim.budget = budget;
    lim.max_slots = max_slots;
    lim.max_step_jobs = step_requests;
    lim.keep_done = kKeepDone;
    lim.lat_window = kLatWindow;
    return lim;
  }
  // A fresh scheduler with the current limits (the old one idle).
  void restart_scheduler() {
    if (sched) sched->stop();
    sched = std::make_unique<Scheduler>(this, limits());
    sched->start();
  }
  void release(Job *job) override {
    Request *r = static_cast<Request *>(job);
    if (r->pinned) {
      std::lock_guard<std::mutex> g(pinned_mu);
      pinned.release(r->pin_off, r->pin_bytes);
    }
    r->pinned = false;
    r->h_stage = nullptr;
    std::vector<double>().swap(r->pageable);
  }
};

static int n_layers(unsigned layers) {
  return ((layers & TSQBX_SLP) ? 1 : 0) + ((layers & TSQBX_DLP) ? 1 : 0) +
         ((layers & TSQBX_SPRIME) ? 1 : 0);
}

// Device bytes of a request: [sigma (N) | positions and strengths
// (stage_pos_bytes) | strength-weighted normals (stage_nrm_bytes), double
// layer only | one T-vector per requested layer].
static size_t request_bytes(const tsqbx_geometry *g, unsigned layers) {
  const size_t N = (size_t)g->n_sources, T = (size_t)g->n_targets;
  size_t b = align_up(N * sizeof(double)) + align_up(stage_pos_bytes(g->n_sources));
  if (layers & TSQBX_DLP) b += align_up(stage_nrm_bytes(g->n_sources));
  b += n_layers(layers) * align_up(T * sizeof(double));
  return std::max<size_t>(b, kAlign);
}

// Device bytes of a Helmholtz request: [sigma (N complex) | records (2 (N+1))
// | table T (p+1) | S' table 2 T (p+1), S' only | one complex T-vector per
// requested layer].
static size_t request_bytes_helm(const tsqbx_geometry *g, int p, unsigned layers) {
  const size_t N = (size_t)g->n_sources, T = std::max<size_t>((size_t)g->n_targets, 1);
  size_t b = align_up(2 * N * sizeof(double)) + align_up(2 * (N + 1) * sizeof(double4));
  b += align_up(T * (size_t)(p + 1) * sizeof(double));
  if (layers & TSQBX_SPRIME) b += align_up(2 * T * (size_t)(p + 1) * sizeof(double));
  b += n_layers(layers) * align_up(2 * (size_t)g->n_targets * sizeof(double));
  return std::max<size_t>(b, kAlign);
}

// Launch one step (called by the scheduler with its lock released).
// Densities in pinned host memory are read by the staging kernel directly
// and outputs are written back by one copy kernel; only requests whose host
// staging had to fall back to pageable memory use DMA copies.
int tsqbx_server::launch(int stream, const std::vector<Job *> &jobs, std::string &err) {
  TraceRange trace_("tsqbx server step launch");
  StreamSlot &ss = strm[stream];
  hipStream_t s = ss.s;
  hipError_t e = hipSuccess;
  auto fail_e = [&](hipError_t x, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(x);
    return TSQBX_E_DEVICE;
  };
  const size_t K = jobs.size();
  std::vector<WorkItem> items;         // Laplace requests
  std::vector<StageItem> stage;
  std::vector<HelmWorkItem> hitems;    // Helmholtz requests
  std::vector<HelmPrepItem> hprep;
  std::vector<CopyItem> copies;
  std::vector<WorkUnit> units, hunits;
  std::vector<int32_t> wave_begin, hwave_begin;
  // DMA copies: densities of pageable-staged and of Helmholtz requests up,
  // outputs of pageable-staged requests down: (destination, source, doubles)
  std::vector<std::tuple<double *, const double *, size_t>> dma_up, pageable_down;
  int64_t max_t = 0, hmax_n = 0, hmax_t = 0;
  LayerClass lc;
  int p_all = -1;
  unsigned h_first = 0;
  bool h_same = true;
  const int64_t per_unit = (int64_t)unit_steps * (64 / tn.group_lanes);
  for (size_t i = 0; i < K; ++i) {
    Request *r = static_cast<Request *>(jobs[i]);
    const tsqbx_geometry *g = r->geom;
    const size_t N = (size_t)g->n_sources, T = (size_t)g->n_targets;
    const size_t cw = r->cw();
    char *base = arena_base + r->arena_off;
    double *d_sigma = (double *)base;
    size_t off = align_up(cw * N * sizeof(double));
    const bool host_pinned = r->borrowed || r->pinned;
    double *d_out[3] = {nullptr, nullptr, nullptr};
    if (r->k > 0.0) {
      HelmStage hs;
      const size_t T1 = std::max<size_t>(T, 1);
      hs.rec = (double4 *)(base + off);
      off += align_up(2 * (N + 1) * sizeof(double4));
      hs.tab = (double *)(base + off);
      off += align_up(T1 * (size_t)(r->p + 1) * sizeof(double));
      if (r->layers & TSQBX_SPRIME) {
        hs.tabs = (double *)(base + off);
        off += align_up(2 * T1 * (size_t)(r->p + 1) * sizeof(double));
      }
      for (int l = 0; l < 3; ++l)
        if (r->layers & (1u << l)) {
          d_out[l] = (double *)(base + off);
          off += align_up(2 * T * sizeof(double));
        }
      if (N) dma_up.emplace_back(d_sigma, r->sigma_src, 2 * N);
      HelmPrepItem q{};
      q.pos_w = g->src_pos;
      q.nrm = g->src_nrm;
      q.perm = g->src_perm;
      q.sigma = d_sigma;
      q.rec = hs.rec;
      q.n = g->n_sources;
      q.tgt = g->tgt;
      q.n_targets = g->n_targets;
      q.k = r->k;
      q.p = r->p;
      q.tab = hs.tab;
      q.tabs = hs.tabs;
      HelmWorkItem w{};
      w.tgt = g->tgt;
      w.tnrm = g->tgt_nrm;
      w.idx = g->idx;
      w.rec = hs.rec;
      w.tab = hs.tab;
      w.tabs = hs.tabs;
      w.out_s = d_out[0];
      w.out_d = d_out[1];
      w.out_t = d_out[2];
      w.k = r->k;
      w.p = r->p;
      w.layers = (int32_t)r->layers;
      w.n_src = (uint32_t)g->n_sources;
      if (hitems.empty()) h_first = r->layers;
      else if (r->layers != h_first) h_same = false;
      const int32_t hi = (int32_t)hitems.size();
      hprep.push_back(q);
      hitems.push_back(w);
      hmax_n = std::max<int64_t>(hmax_n, g->n_sources);
      hmax_t = std::max<int64_t>(hmax_t, g->n_targets);
      for (int64_t k = 0; k < g->n_targets; k += per_unit) {
        hwave_begin.push_back((int32_t)hunits.size());
        hunits.push_back(WorkUnit{hi, (int32_t)k, (int32_t)std::min<int64_t>(per_unit, g->n_targets - k), 0});
      }
    } else {
      char *spos = base + off, *snrm = nullptr;
      off += align_up(stage_pos_bytes(g->n_sources));
      if (r->layers & TSQBX_DLP) {
        snrm = base + off;
        off += align_up(stage_nrm_bytes(g->n_sources));
      }
      const SourceStage stg = stage_views(spos, snrm, g->n_sources);
      for (int l = 0; l < 3; ++l)
        if (r->layers & (1u << l)) {
          d_out[l] = (double *)(base + off);
          off += align_up(T * sizeof(double));
        }
      // a density in pinned memory is read by the staging kernel over PCIe,
      // unless the geometry is large enough for a DMA upload (dma_min_sources)
      const bool zero_copy = host_pinned && g->n_sources < dma_min_sources;
      const double *sig = r->sigma_src;
      if (!zero_copy) {
        if (N) dma_up.emplace_back(d_sigma, r->sigma_src, N);
        sig = d_sigma;
      }
      stage.push_back(make_stage_item(g, sig, r->layers, stg, zero_copy, false));
      WorkItem w{};
      w.tgt = g->tgt;
      w.idx = g->idx;
      w.xy = stg.xy;
      w.zq = stg.zq;
      w.nxy = stg.nxy;
      w.nz = stg.nz;
      w.out_s = d_out[0];
      w.out_d = d_out[1];
      w.out_t = d_out[2];
      w.tnrm = g->tgt_nrm;
      w.p = r->p;
      w.layers = (int32_t)r->layers;
      if (items.empty()) p_all = r->p;
      lc.add(r->layers);
      if (r->p != p_all) p_all = -1;
      const int32_t li = (int32_t)items.size();
      items.push_back(w);
      // fixed-size units, one per wave: constant host work per unit, and the
      // dispatcher balances the waves
      for (int64_t k = 0; k < g->n_targets; k += per_unit) {
        wave_begin.push_back((int32_t)units.size());
        units.push_back(WorkUnit{li, (int32_t)k, (int32_t)std::min<int64_t>(per_unit, g->n_targets - k), 0});
      }
    }
    max_t = std::max<int64_t>(max_t, (int64_t)(cw * T));
    // outputs: into the caller's pinned buffers or the request's host staging
    if (T) {
      double *h = r->h_stage + cw * N;  // host staging: requested layers in order
      for (int l = 0; l < 3; ++l) {
        if (!(r->layers & (1u << l))) continue;
        double *dst = r->borrowed ? r->out[l] : h;
        if (!r->borrowed) h += cw * T;
        if (host_pinned)
          copies.push_back(CopyItem{d_out[l], dst, (int64_t)(cw * T), 0});
        else
          pageable_down.emplace_back(dst, d_out[l], cw * T);
      }
    }
  }
  wave_begin.push_back((int32_t)units.size());
  hwave_begin.push_back((int32_t)hunits.size());
  if (copies.size() > 65535) return fail_e(hipErrorInvalidValue, "too many copies in one step");
  // one metadata block
  const size_t KL = items.size(), KH = hitems.size();
  const size_t o_items = 0;
  const size_t o_stage = align_up(o_items + KL * sizeof(WorkItem));
  const size_t o_copy = align_up(o_stage + KL * sizeof(StageItem));
  const size_t o_units = align_up(o_copy + copies.size() * sizeof(CopyItem));
  const size_t o_wave = align_up(o_units + units.size() * sizeof(WorkUnit));
  const size_t o_hitems = align_up(o_wave + wave_begin.size() * sizeof(int32_t));
  const size_t o_hprep = align_up(o_hitems + KH * sizeof(HelmWorkItem));
  const size_t o_hunits = align_up(o_hprep + KH * sizeof(HelmPrepItem));
  const size_t o_hwave = align_up(o_hunits + hunits.size() * sizeof(WorkUnit));
  const size_t total = align_up(o_hwave + hwave_begin.size() * sizeof(int32_t));
  if (ss.cap_meta < total) {
    if (ss.d_meta) (void)hipFree(ss.d_meta);
    if (ss.h_meta) (void)hipHostFree(ss.h_meta);
    ss.d_meta = ss.h_meta = nullptr;
    ss.cap_meta = 0;
    const size_t cap = std::max<size_t>(total * 2, size_t(1) << 20);
    e = hipMalloc((void **)&ss.d_meta, cap);
    if (e == hipSuccess) e = hipHostMalloc((void **)&ss.h_meta, cap, 0);
    if (e != hipSuccess) return fail_e(e, "step metadata buffers");
    ss.cap_meta = cap;
  }
  auto put = [&](size_t o, const void *src, size_t n) {
    if (n) std::memcpy(ss.h_meta + o, src, n);
  };
  put(o_items, items.data(), KL * sizeof(WorkItem));
  const int64_t stage_total = assign_stage_blocks(stage.data(), (int)KL);
  put(o_stage, stage.data(), KL * sizeof(StageItem));
  put(o_copy, copies.data(), copies.size() * sizeof(CopyItem));
  put(o_units, units.data(), units.size() * sizeof(WorkUnit));
  put(o_wave, wave_begin.data(), wave_begin.size() * sizeof(int32_t));
  put(o_hitems, hitems.data(), KH * sizeof(HelmWorkItem));
  put(o_hprep, hprep.data(), KH * sizeof(HelmPrepItem));
  put(o_hunits, hunits.data(), hunits.size() * sizeof(WorkUnit));
  put(o_hwave, hwave_begin.data(), hwave_begin.size() * sizeof(int32_t));
  e = hipMemcpyAsync(ss.d_meta, ss.h_meta, total, hipMemcpyHostToDevice, s);
  for (size_t i = 0; i < dma_up.size() && e == hipSuccess; ++i)
    e = hipMemcpyAsync(std::get<0>(dma_up[i]), std::get<1>(dma_up[i]),
                       std::get<2>(dma_up[i]) * sizeof(double), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return fail_e(e, "step upload");
  e = launch_stage_multi((const StageItem *)(ss.d_meta + o_stage), (int)KL, stage_total, s);
  if (e == hipSuccess && KH)
    e = launch_helm_prepare_multi((const HelmPrepItem *)(ss.d_meta + o_hprep), (int)KH, hmax_n,
                                  hmax_t, s);
  if (e == hipSuccess && !units.empty()) {
    PersistentArgs a{(const WorkItem *)(ss.d_meta + o_items), (const WorkUnit *)(ss.d_meta + o_units),
                     (const int32_t *)(ss.d_meta + o_wave), (int32_t)wave_begin.size() - 1};
    e = launch_persistent(a, lc.get(), p_all, tn, s);
  }
  if (e == hipSuccess && !hunits.empty()) {
    HelmPersistentArgs a{(const HelmWorkItem *)(ss.d_meta + o_hitems),
                         (const WorkUnit *)(ss.d_meta + o_hunits),
                         (const int32_t *)(ss.d_meta + o_hwave), (int32_t)hwave_begin.size() - 1};
    e = launch_helm_persistent(a, h_same && h_first >= 1 && h_first <= 7 ? h_first : kLayersAny,
                               tn, s);
  }
  if (e == hipSuccess)
    e = launch_copy_multi((const CopyItem *)(ss.d_meta + o_copy), (int)copies.size(), max_t, s);
  for (size_t i = 0; i < pageable_down.size() && e == hipSuccess; ++i)
    e = hipMemcpyAsync(std::get<0>(pageable_down[i]), std::get<1>(pageable_down[i]),
                       std::get<2>(pageable_down[i]) * sizeof(double), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipEventRecord(ss.ev, s);
  if (e != hipSuccess) return fail_e(e, "step launch");
  return TSQBX_OK;
}

extern "C" {

int tsqbx_server_request_bytes(const tsqbx_geometry *geom, unsigned layers, size_t *out) {
  if (!geom || !out) return fail(TSQBX_E_INVALID, "geometry or out is NULL");
  if (layers == 0 || (layers & ~7u)) return fail(TSQBX_E_INVALID, "bad layer mask %u", layers);
  *out = request_bytes(geom, layers);
  return TSQBX_OK;
}

int tsqbx_server_request_bytes_helmholtz(const tsqbx_geometry *geom, int p, unsigned layers,
                                         size_t *out) {
  if (!geom || !out) return fail(TSQBX_E_INVALID, "geometry or out is NULL");
  if (layers == 0 || (layers & ~7u)) return fail(TSQBX_E_INVALID, "bad layer mask %u", layers);
  if (p < 0 || p > TSQBX_P_MAX)
    return fail(TSQBX_E_RANGE, "expansion order p = %d is outside [0, %d]", p, TSQBX_P_MAX);
  *out = request_bytes_helm(geom, p, layers);
  return TSQBX_OK;
}

int tsqbx_server_create(tsqbx_ctx *ctx, size_t hbm_budget, int max_slots, tsqbx_server **out) {
  if (!ctx || !out) return fail(TSQBX_E_INVALID, "ctx or out is NULL");
  *out = nullptr;
  if (hbm_budget < kAlign || max_slots <= 0)
    return fail(TSQBX_E_INVALID, "budget must be at least %zu bytes and max_slots positive", kAlign);
  int prev = -1;
  (void)hipGetDevice(&prev);
  TSQBX_HIP(hipSetDevice(ctx->device));
  auto *sv = new tsqbx_server;
  sv->ctx = ctx;
  sv->device = ctx->device;
  sv->budget = hbm_budget / kAlign * kAlign;
  sv->max_slots = max_slots;
  // one launch shape for the server's lifetime (by default that of near-field
  // lists of a few hundred sources); a request's result then does not
  // depend on its step
  sv->tn = clamp_to_common(default_tuning(16, 3u, 256));
  hipError_t e = hipMalloc((void **)&sv->arena_base, sv->budget);
  // pinned host arena: densities and outputs of queued and running requests
  sv->pinned_cap = std::min<size_t>(sv->budget, size_t(1) << 30);
  if (e == hipSuccess && hipHostMalloc((void **)&sv->pinned_base, sv->pinned_cap, 0) != hipSuccess) {
    sv->pinned_base = nullptr;  // requests then stage through pageable memory
    sv->pinned_cap = 0;
  }
  if (sv->pinned_cap) sv->pinned.init(sv->pinned_cap);
  for (int k = 0; k < kStreams && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&sv->strm[k].s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->strm[k].ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (auto &ss : sv->strm) {
      if (ss.ev) (void)hipEventDestroy(ss.ev);
      if (ss.s) (void)hipStreamDestroy(ss.s);
    }
    if (sv->arena_base) (void)hipFree(sv->arena_base);
    if (sv->pinned_base) (void)hipHostFree(sv->pinned_base);
    delete sv;
    if (prev >= 0) (void)hipSetDevice(prev);
    return fail_hip(e, "server setup");
  }
  sv->restart_scheduler();
  if (prev >= 0) (void)hipSetDevice(prev);
  *out = sv;
  return TSQBX_OK;
}

static bool is_pinned_host(const void *p) {
  if (!p) return true;
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // clear the error a pageable pointer leaves behind
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

// k > 0: a Helmholtz request (complex density and outputs, interleaved).
// internal: a request of the autotuner (does not fix the tuning).
static int submit_impl(tsqbx_server *sv, const tsqbx_geometry *geom, int p, unsigned layers,
                       double k, const double *sigma_host, double *const out_host[3],
                       uint64_t *ticket, bool borrow, bool internal = false) {
  if (!sv || !geom || !ticket) return fail(TSQBX_E_INVALID, "server, geometry or ticket is NULL");
  if (!internal) sv->used = true;
  if (geom->ctx != sv->ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  const bool helm = k != 0.0;
  int rc = helm ? check_helmholtz_request(geom, p, layers, k) : tsqbx_check_request(geom, p, layers);
  if (rc != TSQBX_OK) return rc;
  if (geom->n_sources > 0 && !sigma_host) return fail(TSQBX_E_INVALID, "sigma is NULL");
  for (int l = 0; l < 3; ++l)
    if (geom->n_targets > 0 && (layers & (1u << l)) && !out_host[l])
      return fail(TSQBX_E_INVALID, "output for a requested layer is NULL");
  if (borrow) {
    const double *bufs[4] = {geom->n_sources ? sigma_host : nullptr, nullptr, nullptr, nullptr};
    for (int l = 0; l < 3; ++l)
      if (geom->n_targets && (layers & (1u << l))) bufs[1 + l] = out_host[l];
    for (const double *b : bufs)
      if (!is_pinned_host(b))
        return fail(TSQBX_E_INVALID, "submit_pinned: a buffer is not pinned host memory");
  }
  const size_t bytes = helm ? request_bytes_helm(geom, p, layers) : request_bytes(geom, layers);
  auto *r = new Request;
  r->geom = geom;
  r->p = p;
  r->layers = layers;
  r->k = helm ? k : 0.0;
  const size_t cw = r->cw();
  const size_t N = (size_t)geom->n_sources, T = (size_t)geom->n_targets;
  if (borrow) {
    r->borrowed = true;
    r->sigma_src = sigma_host;
  } else {
    const size_t words = cw * (N + T * n_layers(layers));
    r->pin_bytes = align_up(std::max<size_t>(words, 1) * sizeof(double));
    {
      std::lock_guard<std::mutex> g(sv->pinned_mu);
      r->pinned = sv->pinned_cap > 0 && sv->pinned.alloc(r->pin_bytes, &r->pin_off);
    }
    if (r->pinned) {
      r->h_stage = (double *)(sv->pinned_base + r->pin_off);
    } else {
      r->pageable.resize(std::max<size_t>(words, 1));
      r->h_stage = r->pageable.data();
    }
    if (N) std::memcpy(r->h_stage, sigma_host, cw * N * sizeof(double));
    r->sigma_src = r->h_stage;
  }
  for (int l = 0; l < 3; ++l) r->out[l] = (layers & (1u << l)) ? out_host[l] : nullptr;
  r->bytes = bytes;
  r->pair_terms = geom->pairs * (int64_t)(p + 1) * n_layers(layers);
  rc = sv->sched->submit(r, ticket);  // r belongs to the scheduler from here on
  if (rc == TSQBX_E_STATE) return fail(rc, "server is shutting down");
  if (rc == TSQBX_E_BUDGET)
    return fail(rc, "request needs %zu bytes but the budget is %zu", bytes, sv->budget);
  return rc;
}

int tsqbx_server_submit(tsqbx_server *sv, const tsqbx_geometry *geom, int p, unsigned layers,
                        const double *sigma_host, double *out_slp_host, double *out_dlp_host,
                        double *out_sprime_host, uint64_t *ticket) {
  TraceRange trace_("tsqbx_server_submit");
  double *const outs[3] = {out_slp_host, out_dlp_host, out_sprime_host};
  return submit_impl(sv, geom, p, layers, 0.0, sigma_host, outs, ticket, false);
}

int tsqbx_server_submit_pinned(tsqbx_server *sv, const tsqbx_geometry *geom, int p,
                               unsigned layers, const double *sigma_host, double *out_slp_host,
                               double *out_dlp_host, double *out_sprime_host, uint64_t *ticket) {
  TraceRange trace_("tsqbx_server_submit_pinned");
  double *const outs[3] = {out_slp_host, out_dlp_host, out_sprime_host};
  return submit_impl(sv, geom, p, layers, 0.0, sigma_host, outs, ticket, true);
}

int tsqbx_server_submit_helmholtz(tsqbx_server *sv, const tsqbx_geometry *geom, int p,
                                  unsigned layers, double k, const double *sigma_host,
                                  double *out_slp_host, double *out_dlp_host,
                                  double *out_sprime_host, uint64_t *ticket) {
  TraceRange trace_("tsqbx_server_submit_helmholtz");
  if (!(k > 0.0)) return fail(TSQBX_E_RANGE, "the wavenumber k = %g must be positive and finite", k);
  double *const outs[3] = {out_slp_host, out_dlp_host, out_sprime_host};
  return submit_impl(sv, geom, p, layers, k, sigma_host, outs, ticket, false);
}

int tsqbx_server_submit_helmholtz_pinned(tsqbx_server *sv, const tsqbx_geometry *geom, int p,
                                         unsigned layers, double k, const double *sigma_host,
                                         double *out_slp_host, double *out_dlp_host,
                                         double *out_sprime_host, uint64_t *ticket) {
  TraceRange trace_("tsqbx_server_submit_helmholtz_pinned");
  if (!(k > 0.0)) return fail(TSQBX_E_RANGE, "the wavenumber k = %g must be positive and finite", k);
  double *const outs[3] = {out_slp_host, out_dlp_host, out_sprime_host};
  return submit_impl(sv, geom, p, layers, k, sigma_host, outs, ticket, true);
}

int tsqbx_server_get_tuning(tsqbx_server *sv, tsqbx_server_tuning *out) {
  if (!sv || !out) return fail(TSQBX_E_INVALID, "server or out is NULL");
  out->group_lanes = sv->tn.group_lanes;
  out->unroll = sv->tn.unroll;
  out->waves_per_block = sv->tn.waves_per_block;
  out->unit_steps = sv->unit_steps;
  out->step_requests = sv->step_requests;
  out->dma_min_sources = sv->dma_min_sources >= kNoDma ? 0 : sv->dma_min_sources;
  return TSQBX_OK;
}

static int check_server_tuning(const tsqbx_server_tuning *t) {
  Tuning tn;
  tn.group_lanes = t->group_lanes;
  tn.unroll = t->unroll;
  tn.waves_per_block = t->waves_per_block;
  tn.xcd_remap = 1;
  if (!tuning_supported(tn))
    return fail(TSQBX_E_RANGE, "unsupported launch shape (group_lanes %d, unroll %d, waves %d)",
                t->group_lanes, t->unroll, t->waves_per_block);
  if (t->unit_steps < 1 || t->unit_steps > 64 || t->step_requests < 1 || t->step_requests > 256)
    return fail(TSQBX_E_RANGE, "unit_steps must lie in [1, 64] and step_requests in [1, 256]");
  if (t->dma_min_sources < 0) return fail(TSQBX_E_RANGE, "dma_min_sources must not be negative");
  return TSQBX_OK;
}

// Install a tuning on an idle server (caller holds no request in it).
static void apply_server_tuning(tsqbx_server *sv, const tsqbx_server_tuning &t) {
  sv->tn.group_lanes = t.group_lanes;
  sv->tn.unroll = t.unroll;
  sv->tn.waves_per_block = t.waves_per_block;
  sv->tn.xcd_remap = 1;
  sv->unit_steps = t.unit_steps;
  sv->step_requests = t.step_requests;
  sv->dma_min_sources = t.dma_min_sources > 0 ? t.dma_min_sources : kNoDma;
  sv->restart_scheduler();
}

int tsqbx_server_set_tuning(tsqbx_server *sv, const tsqbx_server_tuning *t) {
  if (!sv || !t) return fail(TSQBX_E_INVALID, "server or tuning is NULL");
  if (sv->used) return fail(TSQBX_E_STATE, "the server has taken requests; its tuning is fixed");
  int rc = check_server_tuning(t);
  if (rc != TSQBX_OK) return rc;
  apply_server_tuning(sv, *t);
  return TSQBX_OK;
}

int tsqbx_server_autotune(tsqbx_server *sv, int64_t n, const tsqbx_geometry *const *geoms,
                          const int *p, const unsigned *layers, const double *const *sigmas,
                          int n_requests, tsqbx_server_tuning *out, double *best_ms) {
  TraceRange trace_("tsqbx_server_autotune");
  if (!sv || n <= 0 || !geoms || !p || !layers || n_requests <= 0)
    return fail(TSQBX_E_INVALID, "server, geometries, orders or layers missing, or no requests");
  if (sv->used) return fail(TSQBX_E_STATE, "the server has taken requests; its tuning is fixed");
  int64_t max_n = 1, max_t = 1;
  for (int64_t i = 0; i < n; ++i) {
    if (!geoms[i] || geoms[i]->ctx != sv->ctx)
      return fail(TSQBX_E_INVALID, "geometry %lld is NULL or of another context", (long long)i);
    int rc = tsqbx_check_request(geoms[i], p[i], layers[i]);
    if (rc != TSQBX_OK) return rc;
    size_t b = 0;
    tsqbx_server_request_bytes(geoms[i], layers[i], &b);
    if (b > sv->budget) return fail(TSQBX_E_BUDGET, "request %lld can never fit the budget", (long long)i);
    max_n = std::max<int64_t>(max_n, geoms[i]->n_sources);
    max_t = std::max<int64_t>(max_t, geoms[i]->n_targets);
    if (sigmas && geoms[i]->n_sources > 0 && !is_pinned_host(sigmas[i]))
      return fail(TSQBX_E_INVALID, "density %lld is not pinned host memory", (long long)i);
  }
  // densities of ones and throw-away outputs in pinned host memory (the
  // requests' results are not kept, so they may share them)
  double *h_sigma = nullptr, *h_out = nullptr;
  int prev = -1;
  (void)hipGetDevice(&prev);
  TSQBX_HIP(hipSetDevice(sv->device));
  struct Free {
    double **a, **b;
    int prev;
    ~Free() {
      if (*a) (void)hipHostFree(*a);
      if (*b) (void)hipHostFree(*b);
      if (prev >= 0) (void)hipSetDevice(prev);
    }
  } fr{&h_sigma, &h_out, prev};
  TSQBX_HIP(hipHostMalloc((void **)&h_sigma, (size_t)max_n * sizeof(double), 0));
  TSQBX_HIP(hipHostMalloc((void **)&h_out, 3 * (size_t)max_t * sizeof(double), 0));
  for (int64_t i = 0; i < max_n; ++i) h_sigma[i] = 1.0;
  auto burst = [&](int count, double *ms) -> int {
    const double t0 = sched_now_s();
    for (int r = 0; r < count; ++r) {
      const int64_t i = r % n;
      double *const outs[3] = {h_out, h_out + max_t, h_out + 2 * max_t};
      uint64_t tk = 0;
      const double *sg = sigmas ? sigmas[i] : h_sigma;
      int rc = submit_impl(sv, geoms[i], p[i], layers[i], 0.0, sg, outs, &tk, true, true);
      if (rc != TSQBX_OK) {
        (void)sv->sched->drain(600.0);  // the buffers stay in use until then
        return rc;
      }
    }
    if (sv->sched->drain(600.0) != TSQBX_OK)
      return fail(TSQBX_E_TIMEOUT, "autotune burst did not finish");
    *ms = (sched_now_s() - t0) * 1e3;
    return TSQBX_OK;
  };
  tsqbx_server_tuning cur{};
  tsqbx_server_get_tuning(sv, &cur);
  // best of two bursts per candidate, after a warm-up burst
  auto time_of = [&](const tsqbx_server_tuning &t, double *ms) -> int {
    apply_server_tuning(sv, t);
    double a = 0, b = 0, w = 0;
    int rc = burst(std::min(n_requests, 64), &w);
    if (rc == TSQBX_OK) rc = burst(n_requests, &a);
    if (rc == TSQBX_OK) rc = burst(n_requests, &b);
    *ms = std::min(a, b);
    return rc;
  };
  // a candidate replaces the best only when clearly faster: burst times vary
  // by a few per cent from run to run
  constexpr double kTuneMargin = 0.97;
  double best = 0;
  int rc = time_of(cur, &best);
  tsqbx_server_tuning best_t = cur;
  // one field at a time, each from the best so far
  const int gu[3][2] = {{16, 2}, {32, 2}, {64, 2}};
  for (int k = 0; k < 3 && rc == TSQBX_OK; ++k) {
    tsqbx_server_tuning t = best_t;
    t.group_lanes = gu[k][0];
    t.unroll = gu[k][1];
    if (t.group_lanes == best_t.group_lanes && t.unroll == best_t.unroll) continue;
    double ms = 0;
    rc = time_of(t, &ms);
    if (rc == TSQBX_OK && ms < kTuneMargin * best) best = ms, best_t = t;
  }
  for (int w : {1, 2, 4}) {
    if (rc != TSQBX_OK || w == best_t.waves_per_block) continue;
    tsqbx_server_tuning t = best_t;
    t.waves_per_block = w;
    double ms = 0;
    rc = time_of(t, &ms);
    if (rc == TSQBX_OK && ms < kTuneMargin * best) best = ms, best_t = t;
  }
  for (int u : {4, 8, 16}) {
    if (rc != TSQBX_OK || u == best_t.unit_steps) continue;
    tsqbx_server_tuning t = best_t;
    t.unit_steps = u;
    double ms = 0;
    rc = time_of(t, &ms);
    if (rc == TSQBX_OK && ms < kTuneMargin * best) best = ms, best_t = t;
  }
  for (int q : {16, 32, 64}) {
    if (rc != TSQBX_OK || q == best_t.step_requests) continue;
    tsqbx_server_tuning t = best_t;
    t.step_requests = q;
    double ms = 0;
    rc = time_of(t, &ms);
    if (rc == TSQBX_OK && ms < kTuneMargin * best) best = ms, best_t = t;
  }
  apply_server_tuning(sv, rc == TSQBX_OK ? best_t : cur);  // fresh statistics too
  if (rc != TSQBX_OK) return rc;
  if (out) *out = best_t;
  if (best_ms) *best_ms = best;
  return TSQBX_OK;
}

int tsqbx_server_poll(tsqbx_server *sv, uint64_t ticket, int *done) {
  if (!sv || !done) return fail(TSQBX_E_INVALID, "server or done is NULL");
  int status = TSQBX_OK;
  if (sv->sched->poll(ticket, done, &status) != TSQBX_OK)
    return fail(TSQBX_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  if (status != TSQBX_OK) return fail(status, "request %llu failed", (unsigned long long)ticket);
  return TSQBX_OK;
}

int tsqbx_server_wait(tsqbx_server *sv, uint64_t ticket, double timeout_s) {
  TraceRange trace_("tsqbx_server_wait");
  if (!sv) return fail(TSQBX_E_INVALID, "server is NULL");
  int status = TSQBX_OK;
  const int rc = sv->sched->wait(ticket, timeout_s, &status);
  if (rc == TSQBX_E_INVALID)
    return fail(rc, "unknown ticket %llu", (unsigned long long)ticket);
  if (rc == TSQBX_E_TIMEOUT)
    return fail(rc, "request %llu not done after %.3f s", (unsigned long long)ticket, timeout_s);
  if (status != TSQBX_OK) return fail(status, "request %llu failed", (unsigned long long)ticket);
  return TSQBX_OK;
}

int tsqbx_server_cancel(tsqbx_server *sv, uint64_t ticket) {
  if (!sv) return fail(TSQBX_E_INVALID, "server is NULL");
  const int rc = sv->sched->cancel(ticket);
  if (rc == TSQBX_E_INVALID)
    return fail(rc, "unknown ticket %llu", (unsigned long long)ticket);
  if (rc == TSQBX_E_STATE)
    return fail(rc, "request %llu is no longer queued", (unsigned long long)ticket);
  return rc;
}

int tsqbx_server_drain(tsqbx_server *sv, double timeout_s) {
  TraceRange trace_("tsqbx_server_drain");
  if (!sv) return fail(TSQBX_E_INVALID, "server is NULL");
  if (sv->sched->drain(timeout_s) != TSQBX_OK)
    return fail(TSQBX_E_TIMEOUT, "requests still pending after %.3f s", timeout_s);
  return TSQBX_OK;
}

int tsqbx_server_get_stats(tsqbx_server *sv, tsqbx_server_stats *out) {
  if (!sv || !out) return fail(TSQBX_E_INVALID, "server or out is NULL");
  sv->sched->stats(out);
  return TSQBX_OK;
}

int tsqbx_server_destroy(tsqbx_server *sv) {
  if (!sv) return TSQBX_OK;
  sv->sched->stop();  // refuses new requests, finishes the queued and running ones
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(sv->device);
  for (auto &ss : sv->strm) {
    if (ss.s) (void)hipStreamSynchronize(ss.s);
    if (ss.d_meta) (void)hipFree(ss.d_meta);
    if (ss.h_meta) (void)hipHostFree(ss.h_meta);
    if (ss.ev) (void)hipEventDestroy(ss.ev);
    if (ss.s) (void)hipStreamDestroy(ss.s);
  }
  if (sv->arena_base) (void)hipFree(sv->arena_base);
  sv->sched.reset();  // forgets the remaining requests
  if (sv->pinned_base) (void)hipHostFree(sv->pinned_base);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete sv;
  return TSQBX_OK;
}

}  // extern "C"
