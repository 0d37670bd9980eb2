// Serving: evaluation requests against device-resident geometries, admitted
// under a device-memory budget and batched continuously.
//
// submit() copies the density into a pinned host arena (pageable memory if
// that arena is full).  A scheduler thread admits queued requests in FIFO
// order while their buffers fit in the budget (one device arena of exactly
// that size) and a request slot is free, and launches everything it admitted
// as one step: density uploads, one staging kernel and one persistent kernel
// over the step's work units, then output downloads into pinned memory.  Up to kStreams steps are in flight on
// separate streams, so requests that arrive while a step runs are launched in
// the next step and overlap with it on the device.  A completion thread polls
// the steps' events, copies outputs to the callers' buffers, releases the
// memory and wakes the scheduler.  Every request is summed by the same device
// routine with the same group width whatever it is batched with, so its
// result does not depend on the mix.  Helmholtz requests (complex density and
// outputs) share the steps: their densities are uploaded by DMA and they get
// their own staging, table and persistent launches in the step.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <list>
#include <thread>
#include <tuple>
#include <vector>

#include "tsqbx_arena.h"
#include "tsqbx_internal.h"

using namespace tsqbx;

namespace {

constexpr int kStreams = 4;
constexpr int kUnitSteps = 8;  // wave-steps (group_lanes-wide passes) per unit
// Requests per step: small enough that the next step's density reads (PCIe)
// overlap this step's evaluation on another stream, large enough to amortise
// the step's launches.
constexpr int kMaxStepRequests = 32;
constexpr size_t kAlign = 256;
// Completed requests whose status stays queryable (poll, wait); older ones
// are forgotten, so that a long-running server holds bounded host memory.
constexpr size_t kKeepDone = 4096;
// Latency percentiles cover the most recent completions, at most this many.
constexpr size_t kLatWindow = 65536;

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

struct Request {
  uint64_t ticket = 0;
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
  size_t bytes = 0, arena_off = 0;
  double t_submit = 0, t_launch = 0, t_done = 0;
  int status = TSQBX_OK;
  bool done = false;
  int waiters = 0;                  // threads blocked in tsqbx_server_wait on it
};

struct Step {
  int stream = -1;
  std::vector<Request *> reqs;
  hipEvent_t done_ev = nullptr;
  double t_launch = 0;
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

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - i;
  return i + 1 < v.size() ? v[i] * (1 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct tsqbx_server {
  tsqbx_ctx *ctx = nullptr;
  int device = 0;
  size_t budget = 0;
  int max_slots = 0;
  Tuning tn;
  char *arena_base = nullptr;
  Arena arena;
  char *pinned_base = nullptr;  // pinned host arena for densities and outputs
  size_t pinned_cap = 0;
  Arena pinned;
  std::mutex pinned_mu;
  StreamSlot streams[kStreams];

  std::mutex mu;
  std::condition_variable cv_sched, cv_done, cv_comp;
  std::deque<Request *> queue;
  std::map<uint64_t, Request *> all;
  std::vector<Step> inflight;
  uint64_t next_ticket = 1;
  bool stopping = false;
  size_t bytes_in_flight = 0, peak_bytes = 0;
  int reqs_in_flight = 0;
  tsqbx_server_stats st{};
  std::vector<double> lat_ms, queue_ms;  // rings of the last kLatWindow completions
  size_t lat_next = 0;
  std::deque<uint64_t> retired;          // completed tickets, oldest first
  double busy_since = -1, busy_acc = 0;
  double host_launch_s = 0;  // scheduler time spent issuing steps
  std::thread sched, comp;

  int launch_step(Step &step, std::string &err);
  // Record a completion (caller holds mu): latency rings, and forget the
  // oldest completed requests beyond kKeepDone (not one a waiter still holds).
  void retire(Request *r) {
    const double lat = (r->t_done - r->t_submit) * 1e3, qu = (r->t_launch - r->t_submit) * 1e3;
    if (lat_ms.size() < kLatWindow) {
      lat_ms.push_back(lat);
      queue_ms.push_back(qu);
    } else {
      lat_ms[lat_next] = lat;
      queue_ms[lat_next] = qu;
    }
    lat_next = (lat_next + 1) % kLatWindow;
    retired.push_back(r->ticket);
    while (retired.size() > kKeepDone) {
      auto it = all.find(retired.front());
      if (it != all.end()) {
        if (it->second->waiters > 0) break;
        delete it->second;
        all.erase(it);
      }
      retired.pop_front();
    }
  }
  void release_host_stage(Request *r) {
    if (r->pinned) {
      std::lock_guard<std::mutex> g(pinned_mu);
      pinned.release(r->pin_off, r->pin_bytes);
    }
    r->pinned = false;
    r->h_stage = nullptr;
    std::vector<double>().swap(r->pageable);
  }
  void scheduler();
  void completer();
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

// Launch one step (called by the scheduler with the lock released).
// Densities in pinned host memory are read by the staging kernel directly
// and outputs are written back by one copy kernel; only requests whose host
// staging had to fall back to pageable memory use DMA copies.
int tsqbx_server::launch_step(Step &step, std::string &err) {
  StreamSlot &ss = streams[step.stream];
  hipStream_t s = ss.s;
  hipError_t e = hipSuccess;
  auto fail_e = [&](hipError_t x, const char *what) {
    err = std::string(what) + ": " + hipGetErrorString(x);
    return TSQBX_E_DEVICE;
  };
  const size_t K = step.reqs.size();
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
  const int64_t per_unit = (int64_t)kUnitSteps * (64 / tn.group_lanes);
  for (size_t i = 0; i < K; ++i) {
    Request *r = step.reqs[i];
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
      const double *sig = r->sigma_src;
      if (!host_pinned) {
        if (N) dma_up.emplace_back(d_sigma, r->sigma_src, N);
        sig = d_sigma;
      }
      stage.push_back(make_stage_item(g, sig, r->layers, stg, host_pinned));
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
  step.done_ev = ss.ev;
  return TSQBX_OK;
}

void tsqbx_server::scheduler() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_sched.wait(lk, [&] {
      if (stopping && queue.empty()) return true;
      if (queue.empty()) return false;
      bool free_stream = false;
      for (auto &ss : streams) free_stream |= !ss.busy;
      return free_stream && reqs_in_flight < max_slots &&
             bytes_in_flight + queue.front()->bytes <= budget;
    });
    if (stopping && queue.empty()) break;
    // admit in FIFO order while memory and slots allow
    Step step;
    for (int k = 0; k < kStreams; ++k)
      if (!streams[k].busy) {
        step.stream = k;
        break;
      }
    while (!queue.empty() && reqs_in_flight < max_slots &&
           step.reqs.size() < (size_t)kMaxStepRequests) {
      Request *r = queue.front();
      size_t off = 0;
      if (bytes_in_flight + r->bytes > budget || !arena.alloc(r->bytes, &off)) break;
      queue.pop_front();
      r->arena_off = off;
      bytes_in_flight += r->bytes;
      peak_bytes = std::max(peak_bytes, bytes_in_flight);
      ++reqs_in_flight;
      ++st.admitted;
      step.reqs.push_back(r);
    }
    if (step.reqs.empty()) {
      // the head fits the budget but not the fragmented arena: wait for a release
      cv_sched.wait_for(lk, std::chrono::milliseconds(1));
      continue;
    }
    streams[step.stream].busy = true;
    const double t0 = now_s();
    for (Request *r : step.reqs) r->t_launch = t0;
    step.t_launch = t0;
    if (busy_since < 0) busy_since = t0;
    lk.unlock();
    std::string err;
    const double th0 = now_s();
    int rc;
    {
      TraceRange trace_("tsqbx server step launch");
      rc = launch_step(step, err);
    }
    const double th1 = now_s();
    lk.lock();
    host_launch_s += th1 - th0;
    if (rc != TSQBX_OK) {
      // the stream may hold partial work: wait for it, then fail the step's requests
      lk.unlock();
      (void)hipStreamSynchronize(streams[step.stream].s);
      lk.lock();
      for (Request *r : step.reqs) {
        r->status = rc;
        r->done = true;
        r->t_done = now_s();
        arena.release(r->arena_off, r->bytes);
        bytes_in_flight -= r->bytes;
        --reqs_in_flight;
        ++st.failed;
        release_host_stage(r);
        retire(r);
      }
      streams[step.stream].busy = false;
      fprintf(stderr, "tsqbx server: step failed: %s\n", err.c_str());
      if (inflight.empty() && busy_since >= 0) {
        busy_acc += now_s() - busy_since;
        busy_since = -1;
      }
      cv_done.notify_all();
      continue;
    }
    ++st.steps;
    inflight.push_back(std::move(step));
    cv_comp.notify_all();
  }
}

void tsqbx_server::completer() {
  (void)hipSetDevice(device);
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_comp.wait(lk, [&] { return !inflight.empty() || (stopping && queue.empty() && reqs_in_flight == 0); });
    if (inflight.empty()) break;
    // find a finished step (poll without the lock)
    std::vector<hipEvent_t> evs;
    for (auto &s : inflight) evs.push_back(s.done_ev);
    lk.unlock();
    int found = -1;
    hipError_t qerr = hipSuccess;
    for (int spin = 0; found < 0; ++spin) {
      for (size_t i = 0; i < evs.size(); ++i) {
        hipError_t q = hipEventQuery(evs[i]);
        if (q == hipSuccess) {
          found = (int)i;
          break;
        }
        if (q != hipErrorNotReady) {
          found = (int)i;
          qerr = q;
          break;
        }
      }
      if (found < 0) {
        if (spin < 200)
          std::this_thread::yield();
        else
          std::this_thread::sleep_for(std::chrono::microseconds(20));
      }
      if (spin > 0 && spin % 64 == 0) {
        // new steps may have been launched meanwhile
        std::lock_guard<std::mutex> g(mu);
        if (inflight.size() != evs.size()) break;
      }
    }
    lk.lock();
    if (found < 0) continue;
    Step step = std::move(inflight[found]);
    inflight.erase(inflight.begin() + found);
    StreamSlot &ss = streams[step.stream];
    const double t1 = now_s();
    for (Request *r : step.reqs) {
      const size_t N = (size_t)r->geom->n_sources, T = (size_t)r->geom->n_targets;
      const size_t cw = r->cw();
      if (qerr == hipSuccess) {
        if (!r->borrowed && T) {
          const double *h = r->h_stage + cw * N;
          for (int l = 0; l < 3; ++l)
            if (r->layers & (1u << l)) {
              std::memcpy(r->out[l], h, cw * T * sizeof(double));
              h += cw * T;
            }
        }
        ++st.completed;
        st.pair_terms_completed += r->geom->pairs * (int64_t)(r->p + 1) * n_layers(r->layers);
      } else {
        r->status = TSQBX_E_DEVICE;
        ++st.failed;
      }
      r->t_done = t1;
      r->done = true;
      arena.release(r->arena_off, r->bytes);
      bytes_in_flight -= r->bytes;
      --reqs_in_flight;
      release_host_stage(r);
      retire(r);
    }
    ss.busy = false;
    if (inflight.empty() && busy_since >= 0) {
      busy_acc += t1 - busy_since;
      busy_since = -1;
    }
    cv_done.notify_all();
    cv_sched.notify_all();
  }
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
  // one launch shape for the server's lifetime (near-field lists of a few
  // hundred sources); a request's result then does not depend on its step
  sv->tn = default_tuning(16, 3u, 256);
  sv->st.budget_bytes = sv->budget;
  hipError_t e = hipMalloc((void **)&sv->arena_base, sv->budget);
  // pinned host arena: densities and outputs of queued and running requests
  sv->pinned_cap = std::min<size_t>(sv->budget, size_t(1) << 30);
  if (e == hipSuccess && hipHostMalloc((void **)&sv->pinned_base, sv->pinned_cap, 0) != hipSuccess) {
    sv->pinned_base = nullptr;  // requests then stage through pageable memory
    sv->pinned_cap = 0;
  }
  if (sv->pinned_cap) sv->pinned.init(sv->pinned_cap);
  for (int k = 0; k < kStreams && e == hipSuccess; ++k) {
    e = hipStreamCreateWithFlags(&sv->streams[k].s, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->streams[k].ev, hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    for (auto &ss : sv->streams) {
      if (ss.ev) (void)hipEventDestroy(ss.ev);
      if (ss.s) (void)hipStreamDestroy(ss.s);
    }
    if (sv->arena_base) (void)hipFree(sv->arena_base);
    if (sv->pinned_base) (void)hipHostFree(sv->pinned_base);
    delete sv;
    if (prev >= 0) (void)hipSetDevice(prev);
    return fail_hip(e, "server setup");
  }
  sv->arena.init(sv->budget);
  sv->sched = std::thread([sv] { sv->scheduler(); });
  sv->comp = std::thread([sv] { sv->completer(); });
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
static int submit_impl(tsqbx_server *sv, const tsqbx_geometry *geom, int p, unsigned layers,
                       double k, const double *sigma_host, double *const out_host[3],
                       uint64_t *ticket, bool borrow) {
  if (!sv || !geom || !ticket) return fail(TSQBX_E_INVALID, "server, geometry or ticket is NULL");
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
  std::lock_guard<std::mutex> lk(sv->mu);
  ++sv->st.submitted;
  if (sv->stopping) {
    sv->release_host_stage(r);
    delete r;
    return fail(TSQBX_E_STATE, "server is shutting down");
  }
  if (bytes > sv->budget) {
    ++sv->st.rejected;
    sv->release_host_stage(r);
    delete r;
    return fail(TSQBX_E_BUDGET, "request needs %zu bytes but the budget is %zu", bytes, sv->budget);
  }
  r->ticket = sv->next_ticket++;
  r->t_submit = now_s();
  sv->all[r->ticket] = r;
  sv->queue.push_back(r);
  *ticket = r->ticket;
  sv->cv_sched.notify_all();
  return TSQBX_OK;
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

int tsqbx_server_poll(tsqbx_server *sv, uint64_t ticket, int *done) {
  if (!sv || !done) return fail(TSQBX_E_INVALID, "server or done is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return fail(TSQBX_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  *done = it->second->done ? 1 : 0;
  if (it->second->done && it->second->status != TSQBX_OK)
    return fail(it->second->status, "request %llu failed", (unsigned long long)ticket);
  return TSQBX_OK;
}

int tsqbx_server_wait(tsqbx_server *sv, uint64_t ticket, double timeout_s) {
  TraceRange trace_("tsqbx_server_wait");
  if (!sv) return fail(TSQBX_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->all.find(ticket);
  if (it == sv->all.end()) return fail(TSQBX_E_INVALID, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = it->second;
  ++r->waiters;  // keeps r from being forgotten while this thread waits
  const bool ok =
      sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), [&] { return r->done; });
  --r->waiters;
  if (!ok)
    return fail(TSQBX_E_TIMEOUT, "request %llu not done after %.3f s", (unsigned long long)ticket, timeout_s);
  if (r->status != TSQBX_OK) return fail(r->status, "request %llu failed", (unsigned long long)ticket);
  return TSQBX_OK;
}

int tsqbx_server_drain(tsqbx_server *sv, double timeout_s) {
  TraceRange trace_("tsqbx_server_drain");
  if (!sv) return fail(TSQBX_E_INVALID, "server is NULL");
  std::unique_lock<std::mutex> lk(sv->mu);
  if (!sv->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                            [&] { return sv->queue.empty() && sv->reqs_in_flight == 0; }))
    return fail(TSQBX_E_TIMEOUT, "requests still pending after %.3f s", timeout_s);
  return TSQBX_OK;
}

int tsqbx_server_get_stats(tsqbx_server *sv, tsqbx_server_stats *out) {
  if (!sv || !out) return fail(TSQBX_E_INVALID, "server or out is NULL");
  std::lock_guard<std::mutex> lk(sv->mu);
  *out = sv->st;
  out->bytes_in_flight = sv->bytes_in_flight;
  out->peak_bytes_in_flight = sv->peak_bytes;
  out->latency_p50_ms = percentile(sv->lat_ms, 0.50);
  out->latency_p90_ms = percentile(sv->lat_ms, 0.90);
  out->latency_p99_ms = percentile(sv->lat_ms, 0.99);
  out->latency_max_ms = sv->lat_ms.empty() ? 0.0 : *std::max_element(sv->lat_ms.begin(), sv->lat_ms.end());
  out->queue_p50_ms = percentile(sv->queue_ms, 0.50);
  out->queue_p99_ms = percentile(sv->queue_ms, 0.99);
  out->busy_s = sv->busy_acc + (sv->busy_since >= 0 ? now_s() - sv->busy_since : 0.0);
  out->host_launch_s = sv->host_launch_s;
  return TSQBX_OK;
}

int tsqbx_server_destroy(tsqbx_server *sv) {
  if (!sv) return TSQBX_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stopping = true;
  }
  sv->cv_sched.notify_all();
  sv->cv_comp.notify_all();
  if (sv->sched.joinable()) sv->sched.join();
  {
    // wake the completer once the last step is done
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->cv_done.wait(lk, [&] { return sv->reqs_in_flight == 0; });
  }
  sv->cv_comp.notify_all();
  if (sv->comp.joinable()) sv->comp.join();
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(sv->device);
  for (auto &ss : sv->streams) {
    if (ss.s) (void)hipStreamSynchronize(ss.s);
    if (ss.d_meta) (void)hipFree(ss.d_meta);
    if (ss.h_meta) (void)hipHostFree(ss.h_meta);
    if (ss.ev) (void)hipEventDestroy(ss.ev);
    if (ss.s) (void)hipStreamDestroy(ss.s);
  }
  if (sv->arena_base) (void)hipFree(sv->arena_base);
  for (auto &kv : sv->all) delete kv.second;
  if (sv->pinned_base) (void)hipHostFree(sv->pinned_base);
  if (prev >= 0) (void)hipSetDevice(prev);
  delete sv;
  return TSQBX_OK;
}

}  // extern "C"
