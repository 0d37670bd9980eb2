// Batched evaluation: many (geometry, p, layers) items in one persistent
// kernel launch, captured once into a HIP graph and replayed; the Helmholtz
// plan does the same for (geometry, p, layers, k) items.
//
// The targets of all items, largest item first and in device (Morton) order
// within an item, are cut into one contiguous range per wave of about equal
// estimated cost (a static schedule: no atomics, no waiting).  Consecutive
// waves hold neighbouring targets and run on the same XCD, so they share
// source records in that XCD's L2.
// Each target is summed by the same device routine as the plain path, so a
// plan's results equal plain evaluations with the same group width bit for bit.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "tsqbx_internal.h"

using namespace tsqbx;

struct tsqbx_plan {
  tsqbx_ctx *ctx = nullptr;
  int device = 0;
  std::vector<tsqbx_item> items;
  std::vector<SourceStage> stages;
  WorkItem *d_items = nullptr;
  WorkUnit *d_units = nullptr;
  int32_t *d_wave_begin = nullptr;
  int32_t n_waves = 0;
  StageItem *d_stage = nullptr;  // staging of every item, one launch
  int64_t max_sources = 0;
  int64_t stage_total = 0;   // staging launch's index space (assign_stage_blocks)
  int64_t n_units = 0;
  int64_t pairs = 0, pair_terms = 0;
  int grid = 0;
  unsigned layer_class = kLayersMixed;  // see LayerClass
  int p_all = -1;            // the order shared by every item, or -1
  Tuning tn;
  int oversub = 8;           // schedule ranges per resident wave slot
  int step_cost = 60;        // fixed cost of a wave-step in the schedule
  uint64_t tune_key = 0;     // the plan's bucket in the context's plan-tuning table
  std::vector<ScheduleItem> sched;  // items as the schedule sees them
  std::vector<int32_t> order;       // items largest first
  size_t sched_bytes = 0;           // device bytes of units and wave_begin
  size_t device_bytes = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  // Helmholtz plans
  bool helm = false;
  std::vector<tsqbx_helm_item> hitems;
  std::vector<HelmStage> hstages;
  HelmWorkItem *d_hitems = nullptr;
  HelmPrepItem *d_hprep = nullptr;
  int64_t max_targets = 0;
};

namespace {

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

void free_plan(tsqbx_plan *pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  for (auto &s : pl->stages) {
    if (s.xy) (void)hipFree(s.xy);    // the blocks' bases
    if (s.nxy) (void)hipFree(s.nxy);
  }
  for (auto &h : pl->hstages) {
    if (h.rec) (void)hipFree(h.rec);
    if (h.tab) (void)hipFree(h.tab);
    if (h.tabs) (void)hipFree(h.tabs);
  }
  if (pl->d_hitems) (void)hipFree(pl->d_hitems);
  if (pl->d_hprep) (void)hipFree(pl->d_hprep);
  if (pl->d_items) (void)hipFree(pl->d_items);
  if (pl->d_stage) (void)hipFree(pl->d_stage);
  if (pl->d_units) (void)hipFree(pl->d_units);
  if (pl->d_wave_begin) (void)hipFree(pl->d_wave_begin);
  delete pl;
}

int layer_count(unsigned l) { return ((l & 1u) ? 1 : 0) + ((l & 2u) ? 1 : 0) + ((l & 4u) ? 1 : 0); }

// Relative cost (vector instructions) of one pair: four per recurrence
// order plus the per-pair setup and the closing sums of each layer.
double pair_cost(int p, unsigned layers) {
  double setup = layers == TSQBX_SLP ? 35.0 : 42.0;
  if (layers & TSQBX_DLP) setup += 8.0;
  if (layers & TSQBX_SPRIME) setup += 9.0;
  return 4.0 * std::max(p - 1, 0) + setup;
}

// The same for the Helmholtz kernel: about 85 instructions of setup and
// sincos, and per order the Legendre and Hankel recurrences with each
// layer's complex sums.
double helm_pair_cost(int p, unsigned layers) {
  double per = 6.0;
  if (layers & TSQBX_SLP) per += 4.0;
  if (layers & TSQBX_DLP) per += 12.0;
  if (layers & TSQBX_SPRIME) per += 8.0;
  return 85.0 + per * std::max(p - 1, 0);
}

}  // namespace

namespace tsqbx {

// Items by estimated cost (pairs times the cost of one pair), largest first;
// ties keep their order.
std::vector<int32_t> order_largest_first(const std::vector<ScheduleItem> &items) {
  std::vector<int32_t> ord(items.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::vector<double> icost(items.size());
  for (size_t i = 0; i < items.size(); ++i)
    icost[i] = (double)items[i].geom->pairs * pair_cost(items[i].p, items[i].layers);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) { return icost[a] > icost[b]; });
  return ord;
}

void build_schedule(const std::vector<ScheduleItem> &items, const std::vector<int32_t> &order,
                    int group_lanes, int max_waves, double step_cost, std::vector<WorkUnit> *units,
                    std::vector<int32_t> *wave_begin) {
  const int G = group_lanes, TPW = 64 / G;
  // the wave-steps: TPW consecutive targets of one item, costed by the
  // longest of their lists (the group lanes run in lockstep)
  struct WStep {
    int32_t item, first, count;
    double cost;
  };
  std::vector<WStep> steps;
  double total = 0.0;
  for (int32_t oi : order) {
    const tsqbx_geometry *g = items[oi].geom;
    const double pc = items[oi].helmholtz ? helm_pair_cost(items[oi].p, items[oi].layers)
                                          : pair_cost(items[oi].p, items[oi].layers);
    for (int64_t k = 0; k < g->n_targets; k += TPW) {
      const int32_t cnt = (int32_t)std::min<int64_t>(TPW, g->n_targets - k);
      int64_t chunks = 0;
      for (int32_t x = 0; x < cnt; ++x)
        chunks = std::max<int64_t>(chunks, (g->host_row_len[k + x] + G - 1) / G);
      const double c = (double)chunks * pc + step_cost;
      steps.push_back(WStep{oi, (int32_t)k, cnt, c});
      total += c;
    }
  }
  units->clear();
  wave_begin->assign(1, 0);
  if (steps.empty()) return;
  const int64_t W = std::max<int64_t>(1, std::min<int64_t>(max_waves, (int64_t)steps.size()));
  // cut the step sequence where the running cost crosses w * total / W
  size_t sidx = 0;
  double acc = 0.0;
  for (int64_t w = 0; w < W; ++w) {
    const double bound = (w + 1 == W) ? 1e300 : total * (double)(w + 1) / (double)W;
    while (sidx < steps.size() && (acc + 0.5 * steps[sidx].cost <= bound)) {
      const WStep &st = steps[sidx];
      WorkUnit *last = units->empty() ? nullptr : &units->back();
      const bool same_wave = (int64_t)units->size() > wave_begin->back();
      if (last && same_wave && last->item == st.item && last->first + last->count == st.first)
        last->count += st.count;  // extend the wave's current run
      else
        units->push_back(WorkUnit{st.item, st.first, st.count, 0});
      acc += st.cost;
      ++sidx;
    }
    wave_begin->push_back((int32_t)units->size());
  }
}

}  // namespace tsqbx

namespace {

int log2_bucket(int64_t v) {
  int b = 0;
  while (b < 40 && (int64_t(1) << (b + 1)) <= v) ++b;
  return b;
}

// A plan's bucket in the context's plan-tuning table: kernel family, the
// orders present (one bit each), the union of the layer masks, and the mean
// list length and target count rounded down to powers of two.
uint64_t plan_tuning_key(bool helm, uint64_t pmask, unsigned layers, int64_t mean_list,
                         int64_t targets) {
  return (uint64_t)(helm ? 1 : 0) | (uint64_t)(layers & 7u) << 1 |
         (uint64_t)log2_bucket(mean_list) << 4 | (uint64_t)log2_bucket(targets) << 10 |
         (pmask & ((uint64_t(1) << (TSQBX_P_MAX + 1)) - 1)) << 16;
}

bool plan_tuning_valid(const PlanTuning &t) {
  const int G = t.tn.group_lanes, U = t.tn.unroll, W = t.tn.waves_per_block;
  if (!((G == 64 && (U == 1 || U == 2)) || ((G == 32 || G == 16) && U == 2))) return false;
  if (!(W == 1 || W == 2 || W == 4)) return false;
  return t.oversub >= 1 && t.oversub <= 32 && t.step_cost >= 0 && t.step_cost <= 100000;
}

PlanTuning plan_tuning_of(const tsqbx_plan *pl) {
  PlanTuning t;
  t.tn = pl->tn;
  t.oversub = pl->oversub;
  t.step_cost = pl->step_cost;
  return t;
}

// (Re)build the static schedule for the plan's current tuning and upload it.
// A captured graph is dropped: the next execute captures the new launch.
hipError_t plan_schedule(tsqbx_plan *pl) {
  std::vector<WorkUnit> units;
  std::vector<int32_t> wave_begin;
  const int cus = pl->ctx->num_cus > 0 ? pl->ctx->num_cus : 256;
  build_schedule(pl->sched, pl->order, pl->tn.group_lanes, persistent_max_waves(cus, pl->oversub),
                 (double)pl->step_cost, &units, &wave_begin);
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->d_units) (void)hipFree(pl->d_units);
  if (pl->d_wave_begin) (void)hipFree(pl->d_wave_begin);
  pl->exec = nullptr;
  pl->graph = nullptr;
  pl->d_units = nullptr;
  pl->d_wave_begin = nullptr;
  pl->device_bytes -= pl->sched_bytes;
  pl->n_units = (int64_t)units.size();
  pl->n_waves = (int32_t)wave_begin.size() - 1;
  pl->grid = (pl->n_waves + pl->tn.waves_per_block - 1) / pl->tn.waves_per_block;
  pl->sched_bytes = units.size() * sizeof(WorkUnit) + wave_begin.size() * sizeof(int32_t);
  pl->device_bytes += pl->sched_bytes;
  hipError_t e = hipSuccess;
  if (pl->n_units) e = hipMalloc((void **)&pl->d_units, units.size() * sizeof(WorkUnit));
  if (e == hipSuccess && pl->n_units)
    e = hipMemcpy(pl->d_units, units.data(), units.size() * sizeof(WorkUnit), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMalloc((void **)&pl->d_wave_begin, wave_begin.size() * sizeof(int32_t));
  if (e == hipSuccess)
    e = hipMemcpy(pl->d_wave_begin, wave_begin.data(), wave_begin.size() * sizeof(int32_t),
                  hipMemcpyHostToDevice);
  return e;
}

// The plan's launches on s: staging (Helmholtz: and the j_n tables), then
// the persistent kernel.  ev (nullable): three events recorded before the
// staging, between the two and after the evaluation.
hipError_t plan_launch(tsqbx_plan *pl, hipStream_t s, hipEvent_t *ev) {
  hipError_t e = ev ? hipEventRecord(ev[0], s) : hipSuccess;
  if (e != hipSuccess) return e;
  if (pl->helm)
    e = launch_helm_prepare_multi(pl->d_hprep, (int)pl->hitems.size(), pl->max_sources,
                                  pl->max_targets, s);
  else
    e = launch_stage_multi(pl->d_stage, (int)pl->items.size(), pl->stage_total, s);
  if (e == hipSuccess && ev) e = hipEventRecord(ev[1], s);
  if (e == hipSuccess && pl->n_units > 0) {
    if (pl->helm) {
      HelmPersistentArgs a{pl->d_hitems, pl->d_units, pl->d_wave_begin, pl->n_waves};
      e = launch_helm_persistent(a, pl->layer_class, pl->tn, s);
    } else {
      PersistentArgs a{pl->d_items, pl->d_units, pl->d_wave_begin, pl->n_waves};
      e = launch_persistent(a, pl->layer_class, pl->p_all, pl->tn, s);
    }
  }
  if (e == hipSuccess && ev) e = hipEventRecord(ev[2], s);
  return e;
}

// Take the context's tuning for the plan's bucket, if one was installed.
void apply_cached_tuning(tsqbx_plan *pl) {
  std::lock_guard<std::mutex> lk(pl->ctx->tuning_mu);
  auto it = pl->ctx->plan_tuning.find(pl->tune_key);
  if (it == pl->ctx->plan_tuning.end() || !plan_tuning_valid(it->second)) return;
  pl->tn = it->second.tn;
  pl->oversub = it->second.oversub;
  pl->step_cost = it->second.step_cost;
}

}  // namespace

extern "C" {

int tsqbx_schedule_preview(int64_t n_items, const int64_t *n_targets, const int64_t *row_len,
                           const int32_t *p, const uint32_t *layers, int group_lanes,
                           int max_waves, int32_t *units, int64_t units_cap, int64_t *n_units,
                           int32_t *wave_begin, int32_t *n_waves) {
  if (n_items < 0 || n_items > 65535)
    return fail(TSQBX_E_RANGE, "schedule_preview: n_items = %lld is outside [0, 65535]",
                (long long)n_items);
  if (!n_units || !n_waves || !wave_begin || (n_items > 0 && (!n_targets || !p || !layers)))
    return fail(TSQBX_E_INVALID, "schedule_preview: a required pointer is NULL");
  if (!(group_lanes == 16 || group_lanes == 32 || group_lanes == 64))
    return fail(TSQBX_E_INVALID, "schedule_preview: group_lanes = %d is not 16, 32 or 64",
                group_lanes);
  if (max_waves < 1) return fail(TSQBX_E_RANGE, "schedule_preview: max_waves < 1");
  // host-only stand-ins for the geometries: target counts and list lengths
  std::vector<tsqbx_geometry> geo(n_items);
  std::vector<ScheduleItem> sched(n_items);
  int64_t off = 0;
  for (int64_t i = 0; i < n_items; ++i) {
    if (n_targets[i] < 0) return fail(TSQBX_E_RANGE, "schedule_preview: n_targets < 0");
    int rc = tsqbx_check_request(nullptr, p[i], layers[i]);
    if (rc != TSQBX_OK) return rc;
    if (n_targets[i] > 0 && !row_len) return fail(TSQBX_E_INVALID, "row_len is NULL");
    geo[i].n_targets = n_targets[i];
    geo[i].host_row_len.assign(row_len + off, row_len + off + n_targets[i]);
    for (int64_t v : geo[i].host_row_len) {
      if (v < 0) return fail(TSQBX_E_RANGE, "schedule_preview: a list length is negative");
      geo[i].pairs += v;
    }
    off += n_targets[i];
    sched[i] = ScheduleItem{&geo[i], p[i], layers[i]};
  }
  std::vector<WorkUnit> u;
  std::vector<int32_t> wb;
  build_schedule(sched, order_largest_first(sched), group_lanes, max_waves, 60.0, &u, &wb);
  *n_units = (int64_t)u.size();
  *n_waves = (int32_t)wb.size() - 1;
  if ((int64_t)u.size() > units_cap || (u.size() && !units))
    return fail(TSQBX_E_RANGE, "schedule_preview: %lld units do not fit the buffer of %lld",
                (long long)u.size(), (long long)units_cap);
  for (size_t k = 0; k < u.size(); ++k) {
    units[3 * k] = u[k].item;
    units[3 * k + 1] = u[k].first;
    units[3 * k + 2] = u[k].count;
  }
  std::copy(wb.begin(), wb.end(), wave_begin);
  return TSQBX_OK;
}

int tsqbx_plan_create(tsqbx_ctx *ctx, int64_t n_items, const tsqbx_item *items, unsigned flags,
                      tsqbx_plan **out) {
  TraceRange trace_("tsqbx_plan_create");
  if (!ctx || !out || n_items < 0 || (n_items > 0 && !items))
    return fail(TSQBX_E_INVALID, "plan_create: ctx, out or items is NULL, or n_items < 0");
  *out = nullptr;
  if (n_items > 65535) return fail(TSQBX_E_RANGE, "a plan holds at most 65535 items");
  for (int64_t i = 0; i < n_items; ++i) {
    const tsqbx_item &it = items[i];
    if (!it.geom) return fail(TSQBX_E_INVALID, "item %lld: geometry is NULL", (long long)i);
    if (it.geom->ctx != ctx)
      return fail(TSQBX_E_INVALID, "item %lld: geometry belongs to another context", (long long)i);
    int rc = tsqbx_check_request(it.geom, it.p, it.layers);
    if (rc != TSQBX_OK) return rc;
    if (it.geom->n_sources > 0 && !it.d_sigma)
      return fail(TSQBX_E_INVALID, "item %lld: sigma is NULL", (long long)i);
    if (it.geom->n_targets > 0 &&
        (((it.layers & TSQBX_SLP) && !it.d_out_slp) || ((it.layers & TSQBX_DLP) && !it.d_out_dlp) ||
         ((it.layers & TSQBX_SPRIME) && !it.d_out_sprime)))
      return fail(TSQBX_E_INVALID, "item %lld: output for a requested layer is NULL", (long long)i);
  }
  Guard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");

  auto *pl = new tsqbx_plan;
  pl->ctx = ctx;
  pl->device = ctx->device;
  pl->items.assign(items, items + n_items);

  // one launch shape for the whole plan, from the pair-weighted mean list length
  int64_t tot_pairs = 0, tot_targets = 0;
  int pmax = 0;
  unsigned lay_all = 0;
  LayerClass lc;
  if (!pl->items.empty()) pl->p_all = pl->items[0].p;
  for (auto &it : pl->items) {
    lc.add(it.layers);
    if (it.p != pl->p_all) pl->p_all = -1;
    tot_pairs += it.geom->pairs;
    tot_targets += it.geom->n_targets;
    pmax = std::max(pmax, it.p);
    lay_all |= it.layers;
    pl->pairs += it.geom->pairs;
    pl->pair_terms += it.geom->pairs * (int64_t)(it.p + 1) * layer_count(it.layers);
  }
  pl->layer_class = lc.get();
  const int64_t mean_list = tot_targets ? (tot_pairs + tot_targets - 1) / tot_targets : 0;
  pl->tn = clamp_to_common(lookup_tuning(ctx, pmax, lay_all ? lay_all : 1u, mean_list));
  if (pl->tn.unroll > 2) pl->tn.unroll = 2;  // the persistent kernels keep two pairs in flight
  if (pl->tn.group_lanes < 64) pl->tn.unroll = 2;
  if (!tuning_supported(pl->tn)) pl->tn = clamp_to_common(default_tuning(pmax, 3u, mean_list));
  uint64_t pmask = 0;
  for (auto &it : pl->items) pmask |= uint64_t(1) << it.p;
  pl->tune_key = plan_tuning_key(false, pmask, lay_all, mean_list, tot_targets);
  apply_cached_tuning(pl);

  // static schedule over the resident waves, items largest first
  pl->sched.resize(n_items);
  for (int64_t i = 0; i < n_items; ++i)
    pl->sched[i] = ScheduleItem{pl->items[i].geom, pl->items[i].p, pl->items[i].layers};
  pl->order = order_largest_first(pl->sched);

  // per-item staging and the device copies of items and units
  std::vector<WorkItem> witems(n_items);
  std::vector<StageItem> sitems(n_items);
  hipError_t e = hipSuccess;
  pl->stages.resize(n_items);
  for (int64_t i = 0; i < n_items && e == hipSuccess; ++i) {
    const tsqbx_item &it = pl->items[i];
    const int64_t N = it.geom->n_sources;
    void *spos = nullptr, *snrm = nullptr;
    e = hipMalloc(&spos, stage_pos_bytes(N));
    pl->device_bytes += stage_pos_bytes(N);
    if (e == hipSuccess && (it.layers & TSQBX_DLP)) {
      e = hipMalloc(&snrm, stage_nrm_bytes(N));
      pl->device_bytes += stage_nrm_bytes(N);
    }
    pl->stages[i] = stage_views(spos, snrm, N);
    // positions once; every execution stages the strengths only
    if (e == hipSuccess) e = launch_stage_positions(it.geom, pl->stages[i], nullptr);
    sitems[i] = make_stage_item(it.geom, it.d_sigma, it.layers, pl->stages[i], false, true);
    pl->max_sources = std::max<int64_t>(pl->max_sources, it.geom->n_sources);
    WorkItem &w = witems[i];
    w = WorkItem{};
    w.tgt = it.geom->tgt;
    w.idx = it.geom->idx;
    w.xy = pl->stages[i].xy;
    w.zq = pl->stages[i].zq;
    w.nxy = pl->stages[i].nxy;
    w.nz = pl->stages[i].nz;
    w.out_s = it.d_out_slp;
    w.out_d = it.d_out_dlp;
    w.out_t = it.d_out_sprime;
    w.tnrm = it.geom->tgt_nrm;
    w.p = it.p;
    w.layers = (int32_t)it.layers;
    w.accumulate = (flags & TSQBX_ACCUMULATE) ? 1 : 0;
  }
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);  // positions in place before any execution
  if (e == hipSuccess && n_items) e = hipMalloc((void **)&pl->d_items, n_items * sizeof(WorkItem));
  if (e == hipSuccess && n_items)
    e = hipMemcpy(pl->d_items, witems.data(), n_items * sizeof(WorkItem), hipMemcpyHostToDevice);
  pl->stage_total = assign_stage_blocks(sitems.data(), (int)n_items);
  if (e == hipSuccess && n_items) e = hipMalloc((void **)&pl->d_stage, n_items * sizeof(StageItem));
  if (e == hipSuccess && n_items)
    e = hipMemcpy(pl->d_stage, sitems.data(), n_items * sizeof(StageItem), hipMemcpyHostToDevice);
  pl->device_bytes += n_items * (sizeof(WorkItem) + sizeof(StageItem));
  if (e == hipSuccess) e = plan_schedule(pl);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_plan(pl);
    return fail_hip(e, "plan setup");
  }
  *out = pl;
  return TSQBX_OK;
}

int tsqbx_plan_create_helmholtz(tsqbx_ctx *ctx, int64_t n_items, const tsqbx_helm_item *items,
                                unsigned flags, tsqbx_plan **out) {
  TraceRange trace_("tsqbx_plan_create_helmholtz");
  if (!ctx || !out || n_items < 0 || (n_items > 0 && !items))
    return fail(TSQBX_E_INVALID, "plan_create: ctx, out or items is NULL, or n_items < 0");
  *out = nullptr;
  if (n_items > 65535) return fail(TSQBX_E_RANGE, "a plan holds at most 65535 items");
  for (int64_t i = 0; i < n_items; ++i) {
    const tsqbx_helm_item &it = items[i];
    if (!it.geom) return fail(TSQBX_E_INVALID, "item %lld: geometry is NULL", (long long)i);
    if (it.geom->ctx != ctx)
      return fail(TSQBX_E_INVALID, "item %lld: geometry belongs to another context", (long long)i);
    int rc = check_helmholtz_request(it.geom, it.p, it.layers, it.k);
    if (rc != TSQBX_OK) return rc;
    if (it.geom->n_sources > 0 && !it.d_sigma)
      return fail(TSQBX_E_INVALID, "item %lld: sigma is NULL", (long long)i);
    if (it.geom->n_targets > 0 &&
        (((it.layers & TSQBX_SLP) && !it.d_out_slp) || ((it.layers & TSQBX_DLP) && !it.d_out_dlp) ||
         ((it.layers & TSQBX_SPRIME) && !it.d_out_sprime)))
      return fail(TSQBX_E_INVALID, "item %lld: output for a requested layer is NULL", (long long)i);
  }
  Guard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");

  auto *pl = new tsqbx_plan;
  pl->ctx = ctx;
  pl->device = ctx->device;
  pl->helm = true;
  pl->hitems.assign(items, items + n_items);

  int64_t tot_pairs = 0, tot_targets = 0;
  int pmax = 0;
  unsigned lay_all = 0, first = n_items ? items[0].layers : 0;
  bool same = true;
  for (auto &it : pl->hitems) {
    same = same && it.layers == first;
    tot_pairs += it.geom->pairs;
    tot_targets += it.geom->n_targets;
    pmax = std::max(pmax, it.p);
    lay_all |= it.layers;
    pl->pairs += it.geom->pairs;
    pl->pair_terms += it.geom->pairs * (int64_t)(it.p + 1) * layer_count(it.layers);
  }
  pl->layer_class = same && first >= 1 && first <= 7 ? first : kLayersAny;
  const int64_t mean_list = tot_targets ? (tot_pairs + tot_targets - 1) / tot_targets : 0;
  pl->tn = clamp_to_common(
      lookup_tuning(ctx, pmax, (lay_all ? lay_all : 1u) | TSQBX_HELMHOLTZ, mean_list));
  pl->tn.unroll = std::min(std::max(pl->tn.unroll, 1), 2);
  if (pl->tn.group_lanes < 64) pl->tn.unroll = 2;
  if (!tuning_supported(pl->tn)) pl->tn = clamp_to_common(default_tuning(pmax, lay_all, mean_list));
  uint64_t pmask = 0;
  for (auto &it : pl->hitems) pmask |= uint64_t(1) << it.p;
  pl->tune_key = plan_tuning_key(true, pmask, lay_all, mean_list, tot_targets);
  apply_cached_tuning(pl);

  // item order: largest first; static schedule over the resident waves
  std::vector<int64_t> ord(n_items);
  std::iota(ord.begin(), ord.end(), 0);
  std::vector<double> icost(n_items);
  for (int64_t i = 0; i < n_items; ++i)
    icost[i] = (double)pl->hitems[i].geom->pairs * helm_pair_cost(pl->hitems[i].p, pl->hitems[i].layers);
  std::stable_sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return icost[a] > icost[b]; });
  pl->sched.resize(n_items);
  for (int64_t i = 0; i < n_items; ++i)
    pl->sched[i] = ScheduleItem{pl->hitems[i].geom, pl->hitems[i].p, pl->hitems[i].layers, true};
  pl->order.assign(ord.begin(), ord.end());

  // per-item staging, tables and the device copies of items and units
  std::vector<HelmWorkItem> witems(n_items);
  std::vector<HelmPrepItem> pitems(n_items);
  hipError_t e = hipSuccess;
  pl->hstages.resize(n_items);
  for (int64_t i = 0; i < n_items && e == hipSuccess; ++i) {
    const tsqbx_helm_item &it = pl->hitems[i];
    const tsqbx_geometry *g = it.geom;
    HelmStage &st = pl->hstages[i];
    const size_t N1 = (size_t)g->n_sources + 1, T = std::max<size_t>(1, (size_t)g->n_targets);
    e = hipMalloc((void **)&st.rec, 2 * N1 * sizeof(double4));
    if (e == hipSuccess) e = hipMalloc((void **)&st.tab, T * (size_t)(it.p + 1) * sizeof(double));
    if (e == hipSuccess && (it.layers & TSQBX_SPRIME))
      e = hipMalloc((void **)&st.tabs, 2 * T * (size_t)(it.p + 1) * sizeof(double));
    pl->device_bytes += 2 * N1 * sizeof(double4) + T * (size_t)(it.p + 1) * sizeof(double) *
                                                       ((it.layers & TSQBX_SPRIME) ? 3 : 1);
    HelmWorkItem &w = witems[i];
    w = HelmWorkItem{};
    w.tgt = g->tgt;
    w.tnrm = g->tgt_nrm;
    w.idx = g->idx;
    w.rec = st.rec;
    w.tab = st.tab;
    w.tabs = st.tabs;
    w.out_s = it.d_out_slp;
    w.out_d = it.d_out_dlp;
    w.out_t = it.d_out_sprime;
    w.k = it.k;
    w.p = it.p;
    w.layers = (int32_t)it.layers;
    w.accumulate = (flags & TSQBX_ACCUMULATE) ? 1 : 0;
    w.n_src = (uint32_t)g->n_sources;
    HelmPrepItem &q = pitems[i];
    q = HelmPrepItem{};
    q.pos_w = g->src_pos;
    q.nrm = g->src_nrm;
    q.perm = g->src_perm;
    q.sigma = it.d_sigma;
    q.rec = st.rec;
    q.n = g->n_sources;
    q.tgt = g->tgt;
    q.n_targets = g->n_targets;
    q.k = it.k;
    q.p = it.p;
    q.tab = st.tab;
    q.tabs = (it.layers & TSQBX_SPRIME) ? st.tabs : nullptr;
    pl->max_sources = std::max<int64_t>(pl->max_sources, g->n_sources);
    pl->max_targets = std::max<int64_t>(pl->max_targets, g->n_targets);
  }
  if (e == hipSuccess && n_items) e = hipMalloc((void **)&pl->d_hprep, n_items * sizeof(HelmPrepItem));
  if (e == hipSuccess && n_items)
    e = hipMemcpy(pl->d_hprep, pitems.data(), n_items * sizeof(HelmPrepItem), hipMemcpyHostToDevice);
  if (e == hipSuccess && n_items) e = hipMalloc((void **)&pl->d_hitems, n_items * sizeof(HelmWorkItem));
  if (e == hipSuccess && n_items)
    e = hipMemcpy(pl->d_hitems, witems.data(), n_items * sizeof(HelmWorkItem), hipMemcpyHostToDevice);
  pl->device_bytes += n_items * (sizeof(HelmWorkItem) + sizeof(HelmPrepItem));
  if (e == hipSuccess) e = plan_schedule(pl);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    free_plan(pl);
    return fail_hip(e, "plan setup");
  }
  *out = pl;
  return TSQBX_OK;
}

int tsqbx_plan_execute(tsqbx_plan *pl, void *hip_stream) {
  TraceRange trace_("tsqbx_plan_execute");
  if (!pl) return fail(TSQBX_E_INVALID, "plan is NULL");
  Guard dg(pl->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  if (!pl->exec) {
    // capture: staging of every item (one kernel; Helmholtz: and the tables),
    // then the persistent kernel
    hipStream_t cs = pl->cap_stream;
    TSQBX_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = plan_launch(pl, cs, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail_hip(e != hipSuccess ? e : e2, "plan capture");
    }
    pl->graph = g;
    e = hipGraphInstantiate(&pl->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      pl->exec = nullptr;
      return fail_hip(e, "hipGraphInstantiate");
    }
  }
  TSQBX_HIP(hipGraphLaunch(pl->exec, (hipStream_t)hip_stream));
  return TSQBX_OK;
}

int tsqbx_plan_get_tuning(const tsqbx_plan *pl, tsqbx_plan_tuning *out) {
  if (!pl || !out) return fail(TSQBX_E_INVALID, "plan or out is NULL");
  out->group_lanes = pl->tn.group_lanes;
  out->unroll = pl->tn.unroll;
  out->waves_per_block = pl->tn.waves_per_block;
  out->oversubscription = pl->oversub;
  out->step_cost = pl->step_cost;
  return TSQBX_OK;
}

int tsqbx_plan_set_tuning(tsqbx_plan *pl, const tsqbx_plan_tuning *t) {
  TraceRange trace_("tsqbx_plan_set_tuning");
  if (!pl || !t) return fail(TSQBX_E_INVALID, "plan or tuning is NULL");
  PlanTuning pt = plan_tuning_of(pl);
  pt.tn.group_lanes = t->group_lanes;
  pt.tn.unroll = t->unroll;
  pt.tn.waves_per_block = t->waves_per_block;
  pt.oversub = t->oversubscription;
  pt.step_cost = t->step_cost;
  if (!plan_tuning_valid(pt))
    return fail(TSQBX_E_INVALID,
                "plan tuning (group_lanes %d, unroll %d, waves_per_block %d, oversubscription "
                "%d, step_cost %d) is not supported",
                t->group_lanes, t->unroll, t->waves_per_block, t->oversubscription, t->step_cost);
  Guard dg(pl->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  TSQBX_HIP(hipDeviceSynchronize());  // earlier launches may still read the schedule
  pl->tn = pt.tn;
  pl->oversub = pt.oversub;
  pl->step_cost = pt.step_cost;
  TSQBX_HIP(plan_schedule(pl));
  return TSQBX_OK;
}

int tsqbx_plan_profile(tsqbx_plan *pl, int reps, void *hip_stream, tsqbx_plan_timing *out) {
  TraceRange trace_("tsqbx_plan_profile");
  if (!pl || !out) return fail(TSQBX_E_INVALID, "plan or out is NULL");
  if (reps < 1 || reps > 1000) return fail(TSQBX_E_RANGE, "reps = %d is outside [1, 1000]", reps);
  Guard dg(pl->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
  hipError_t e = hipSuccess;
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreate(&ev[k]);
  double st = 0.0, ev_ms = 0.0;
  for (int r = 0; r <= reps && e == hipSuccess; ++r) {
    e = plan_launch(pl, s, ev);
    if (e == hipSuccess) e = hipEventSynchronize(ev[2]);
    float a = 0.f, b = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&a, ev[0], ev[1]);
    if (e == hipSuccess) e = hipEventElapsedTime(&b, ev[1], ev[2]);
    if (r > 0) {  // the first run warms up
      st += a;
      ev_ms += b;
    }
  }
  for (auto &x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) return fail_hip(e, "plan profile");
  out->stage_ms = st / reps;
  out->eval_ms = ev_ms / reps;
  out->reps = reps;
  return TSQBX_OK;
}

int tsqbx_plan_autotune(tsqbx_plan *pl, void *hip_stream, tsqbx_plan_tuning *out,
                        double *best_ms) {
  TraceRange trace_("tsqbx_plan_autotune");
  if (!pl) return fail(TSQBX_E_INVALID, "plan is NULL");
  Guard dg(pl->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  TSQBX_HIP(hipDeviceSynchronize());
  PlanTuning best = plan_tuning_of(pl);
  double best_t = 1e300;
  // time one candidate; keep it if it beats the best so far
  auto trial = [&](const PlanTuning &c) -> int {
    if (!plan_tuning_valid(c)) return TSQBX_OK;
    pl->tn = c.tn;
    pl->oversub = c.oversub;
    pl->step_cost = c.step_cost;
    hipError_t e = plan_schedule(pl);
    if (e != hipSuccess) return fail_hip(e, "plan autotune schedule");
    tsqbx_plan_timing tm;
    int rc = tsqbx_plan_profile(pl, 3, hip_stream, &tm);
    if (rc != TSQBX_OK) return rc;
    if (tm.eval_ms < best_t) {
      best_t = tm.eval_ms;
      best = c;
    }
    return TSQBX_OK;
  };
  int rc = trial(best);  // the current tuning first
  static const int GU[][2] = {{64, 1}, {64, 2}, {32, 2}, {16, 2}};
  for (auto &gu : GU) {
    if (rc != TSQBX_OK) break;
    PlanTuning c = best;
    c.tn.group_lanes = gu[0];
    c.tn.unroll = gu[1];
    rc = trial(c);
  }
  for (int w : {1, 2, 4}) {
    if (rc != TSQBX_OK) break;
    PlanTuning c = best;
    c.tn.waves_per_block = w;
    rc = trial(c);
  }
  for (int o : {1, 2, 4, 8, 16}) {
    if (rc != TSQBX_OK) break;
    PlanTuning c = best;
    c.oversub = o;
    rc = trial(c);
  }
  for (int sc : {0, 15, 60, 240, 1000}) {
    if (rc != TSQBX_OK) break;
    PlanTuning c = best;
    c.step_cost = sc;
    rc = trial(c);
  }
  // leave the plan on the best tuning (also after a failure)
  pl->tn = best.tn;
  pl->oversub = best.oversub;
  pl->step_cost = best.step_cost;
  hipError_t e = plan_schedule(pl);
  if (rc != TSQBX_OK) return rc;
  if (e != hipSuccess) return fail_hip(e, "plan autotune schedule");
  {
    std::lock_guard<std::mutex> lk(pl->ctx->tuning_mu);
    pl->ctx->plan_tuning[pl->tune_key] = best;
  }
  if (out) tsqbx_plan_get_tuning(pl, out);
  if (best_ms) *best_ms = best_t;
  return TSQBX_OK;
}

int tsqbx_plan_get_info(const tsqbx_plan *pl, tsqbx_plan_info *out) {
  if (!pl || !out) return fail(TSQBX_E_INVALID, "plan or out is NULL");
  out->n_items = (int64_t)(pl->helm ? pl->hitems.size() : pl->items.size());
  out->n_units = pl->n_units;
  out->pairs = pl->pairs;
  out->pair_terms = pl->pair_terms;
  out->grid_blocks = pl->grid;
  out->waves_per_block = pl->tn.waves_per_block;
  out->device_bytes = pl->device_bytes;
  return TSQBX_OK;
}

int tsqbx_plan_destroy(tsqbx_plan *pl) {
  if (!pl) return TSQBX_OK;
  Guard dg(pl->device);
  (void)hipDeviceSynchronize();
  free_plan(pl);
  return TSQBX_OK;
}

}  // extern "C"
