// Internal declarations shared by the host runtime and the kernels of
// libtsqbx.so.  Not part of the public ABI (include/tsqbx.h).
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <cstdint>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "tsqbx.h"

namespace tsqbx {

// One target in device order: its center, the offset t - c, and the CSR row
// of its center (64 bytes, read once per target with one scalar load).
struct alignas(64) TargetRec {
  double c[3];
  double d[3];
  int64_t row_begin;
  int32_t row_len;
  int32_t out_index;  // caller's target index
};
static_assert(sizeof(TargetRec) == 64, "TargetRec layout");

// One device row (a center that at least one target uses) for the
// conventional path: the center, its list (unpadded length), the caller's
// center index and the row's targets in row_tgts[tgt_begin ..].
struct alignas(64) CenterRec {
  double c[3];
  int64_t row_begin;
  int32_t len;
  int32_t center;
  int32_t tgt_begin;
  int32_t tgt_count;
  int64_t pad;
};
static_assert(sizeof(CenterRec) == 64, "CenterRec layout");

// Device rows are padded to a multiple of this many entries with index N,
// which names a zero-strength staging record.
constexpr int kRowPad = 16;

// Per-source staging built for each evaluation: the position, the strength
// q = w sigma and, for the double layer, q times the normal, in four arrays
// of 16 or 8 bytes per source.  A wave's gather of one array then reads, for
// a run of consecutive sources, consecutive bytes across its lanes: a
// 16-byte load over 64 lanes touches half the 64-byte sectors that the two
// halves of a 32-byte record would, and the vector memory pipeline's cost
// follows the sectors a load touches.  Entry N is the padding record: far
// from every center, with q = 0.  xy and zq share one block of
// stage_pos_bytes(N), nxy and nz one of stage_nrm_bytes(N) (xy and nxy are
// the blocks' bases).
struct SourceStage {
  double2 *xy = nullptr;    // [N + 1] (x, y)
  double2 *zq = nullptr;    // [N + 1] (z, q)
  double2 *nxy = nullptr;   // [N + 1] (q nx, q ny)
  double *nz = nullptr;     // [N + 1] q nz
};
inline size_t stage_pos_bytes(int64_t n) { return (size_t)(n + 1) * 32; }
inline size_t stage_nrm_bytes(int64_t n) { return (size_t)(n + 1) * 24; }
// The four arrays inside blocks of those sizes (nrm may be null).
inline SourceStage stage_views(void *pos, void *nrm, int64_t n) {
  SourceStage s;
  s.xy = (double2 *)pos;
  s.zq = pos ? s.xy + (n + 1) : nullptr;
  s.nxy = (double2 *)nrm;
  s.nz = nrm ? (double *)(s.nxy + (n + 1)) : nullptr;
  return s;
}

// Output vectors of one evaluation (device pointers, caller's target order);
// null for a layer not evaluated.
struct Outputs {
  double *s = nullptr;  // single layer
  double *d = nullptr;  // double layer
  double *t = nullptr;  // S', normal derivative of the single layer at the target
};

// Helmholtz staging of one geometry (allocated by its first Helmholtz call):
// rec[2i] = (x, y, z, Re q), rec[2i+1] = (Im q, nu), i = 0..N (N: padding);
// tab: (2n+1) j_n(k |t - c|) per device-order target, rows of p + 1;
// tabs (allocated by the first S' call): (2n+1) k j_n'(k |t - c|) and
// (2n+1) j_n(k |t - c|) / |t - c|, rows of 2 (p + 1).
struct HelmStage {
  double4 *rec = nullptr;  // [2 (N + 1)]
  double *tab = nullptr;   // [T (TSQBX_P_MAX + 1)]
  double *tabs = nullptr;  // [T 2 (TSQBX_P_MAX + 1)] or null
};

struct Tuning {
  int waves_per_block = 4;
  int group_lanes = 64;
  int unroll = 2;
  int xcd_remap = 1;
};

// Tuning of a plan's persistent kernel: its launch shape and the two knobs of
// its static schedule (ranges per resident wave slot, fixed cost of a
// wave-step).
struct PlanTuning {
  Tuning tn;
  int oversub = 8;
  int step_cost = 60;
};

}  // namespace tsqbx

struct tsqbx_ctx {
  int device = 0;
  int num_cus = 0;
  hipStream_t stream = nullptr;  // stream of the synchronous tsqbx_eval
  std::mutex mu;
  // host-pointer eval staging (grown on demand)
  double *d_sigma = nullptr;
  size_t d_sigma_cap = 0;
  double *d_out = nullptr;
  size_t d_out_cap = 0;
  // tuning table: key = (p, layers, list bucket)
  std::map<uint64_t, tsqbx::Tuning> tuning;
  // plan tunings: key = plan bucket (see plan_tuning_key)
  std::map<uint64_t, tsqbx::PlanTuning> plan_tuning;
  std::mutex tuning_mu;
  // device address of the GPU's scratch array of tsqbx_eval_async_noalloc
  void *scratch = nullptr;
};

struct tsqbx_geometry {
  tsqbx_ctx *ctx = nullptr;
  int device = 0;
  int64_t n_sources = 0, n_centers = 0, n_targets = 0, nnz = 0, pairs = 0, max_list = 0;
  bool has_normals = false;
  bool has_target_normals = false;
  double4 *src_pos = nullptr;    // [N] (x, y, z, w) in device order
  double *src_w = nullptr;       // [N] w in device order
  double4 *src_nrm = nullptr;    // [N] (nx, ny, nz, 0) or null
  int64_t *src_perm = nullptr;   // [N] device order -> caller index, null if identity
  int32_t *src_rank = nullptr;   // [N] caller index -> device order, null if identity
  tsqbx::TargetRec *tgt = nullptr;  // [T] in device order
  double4 *tgt_nrm = nullptr;    // [T] (nx, ny, nz, 0) at the targets, device order, or null
  int32_t *idx = nullptr;        // [nnz'] lists in device numbering, one row per target group
  int64_t n_rows = 0;            // rows = distinct centers with targets
  int64_t max_row_targets = 0;   // most targets any row has
  tsqbx::CenterRec *ctr = nullptr;  // [n_rows]
  int32_t *row_tgts = nullptr;   // [T] device-order targets grouped by row
  tsqbx::SourceStage stage;      // staging used by the plain path (positions written at creation)
  // layers the last tsqbx_stage_async call staged for (0: none yet)
  mutable std::atomic<unsigned> staged_layers{0};
  tsqbx::HelmStage helm;         // Helmholtz staging, allocated on first use
  size_t device_bytes = 0;
  std::vector<int64_t> host_row_len;  // per device-order target, for planning
};

namespace tsqbx {

// A roctx range around one entry point, visible in rocprofv3 --marker-trace.
struct TraceRange {
  explicit TraceRange(const char *name) { roctxRangePushA(name); }
  ~TraceRange() { roctxRangePop(); }
  TraceRange(const TraceRange &) = delete;
  TraceRange &operator=(const TraceRange &) = delete;
};

// error reporting (thread-local message)
int fail(int code, const char *fmt, ...);
int fail_hip(hipError_t e, const char *what);
#define TSQBX_HIP(call)                                   \
  do {                                                    \
    hipError_t e__ = (call);                              \
    if (e__ != hipSuccess) return ::tsqbx::fail_hip(e__, #call); \
  } while (0)

// kernel launchers (tsqbx_eval.hip, tsqbx_stage.hip)
// positions_ready: st already holds the positions and the padding entry
// (launch_stage_positions), so only the strengths are written.
hipError_t launch_stage(const tsqbx_geometry *g, const double *d_sigma, unsigned layers,
                        const SourceStage &st, bool positions_ready, hipStream_t s);
hipError_t launch_stage_positions(const tsqbx_geometry *g, const SourceStage &st, hipStream_t s);
hipError_t launch_eval(const tsqbx_geometry *g, int p, unsigned layers, const SourceStage &st,
                       const Outputs &out, bool accumulate, const Tuning &tn, hipStream_t s);
// The plain Laplace path (tsqbx_eval_rows.hip): where targets share rows
// (on average 1.5 or more per row, at most 16 in any) and one wave takes a
// target, one wave per row walks each list once for up to four targets
// (k_eval_rows), with the bits of launch_eval; per_target
// (TSQBX_PER_TARGET) keeps launch_eval.
bool rows_kernel_pays(const tsqbx_geometry *g, const Tuning &tn);
hipError_t launch_eval_plain(const tsqbx_geometry *g, int p, unsigned layers,
                             const SourceStage &st, const Outputs &out, bool accumulate,
                             const Tuning &tn, bool per_target, hipStream_t s);
// Tunings every kernel takes (blocks of up to 4 waves) ...
bool tuning_supported(const Tuning &tn);
// ... and those of the plain Laplace kernel, which also takes blocks of 8
// waves (8 Morton-adjacent targets per block share more of their sources in
// the compute unit's L1).
bool eval_tuning_supported(const Tuning &tn);
// A tuning for the persistent (batched, served) and Helmholtz kernels: blocks
// of at most 4 waves.
inline Tuning clamp_to_common(Tuning t) {
  if (t.waves_per_block > 4) t.waves_per_block = 4;
  return t;
}
// Conventional QBX (tsqbx_conventional.hip): mode 1 forms the local
// coefficients of every row's center from the staged sources into
// coeffs_out, mode 2 evaluates coeffs_in at the targets into out, mode 3
// forms and evaluates in one launch.  Coefficients: [n_centers][(p+1)^2],
// compact real layout; out in the caller's target order.
hipError_t launch_qbxl(const tsqbx_geometry *g, int p, int mode, const SourceStage &st,
                       const double *coeffs_in, double *coeffs_out, double *out, bool accumulate,
                       hipStream_t s);
// Helmholtz (tsqbx_helmholtz.hip): staging of q = w sigma (sigma complex,
// interleaved), the per-target table and the pair kernel; outputs complex,
// interleaved, in the caller's target order.
hipError_t launch_helmholtz(const tsqbx_geometry *g, int p, unsigned layers, double k,
                            const double *d_sigma, const HelmStage &st, const Outputs &out,
                            bool accumulate, const Tuning &tn, hipStream_t s);

// Staging of many items in one launch (batched and served paths).
struct StageItem {
  const double4 *pos_w;
  const double *w;           // weights in device order
  const double4 *nrm;
  const void *order;         // host_sigma: rank (int32, caller -> device); else perm (int64)
  const double *sigma;       // caller order; device or pinned host memory
  double2 *xy;               // the item's SourceStage arrays
  double2 *zq;
  double2 *nxy;
  double *nz;
  int64_t n;
  int32_t want_dlp;
  int32_t host_sigma;        // 1: walk sources in caller order (contiguous reads of sigma)
  int64_t begin;             // first element of the item in the launch's index space
  int32_t strengths_only;    // 1: positions and padding entry already in place
  int32_t unused;
};
static_assert(sizeof(StageItem) == 104, "StageItem layout");
StageItem make_stage_item(const tsqbx_geometry *g, const double *sigma, unsigned layers,
                          const SourceStage &st, bool sigma_on_host, bool positions_ready);
// Lay the items' n + 1 elements end to end, each item starting at a multiple
// of kStageBlock, in begin; returns the total (a multiple of kStageBlock).
constexpr int64_t kStageBlock = 256;
int64_t assign_stage_blocks(StageItem *items, int n_items);
// Staging of every item in one launch: one block of kStageBlock threads per
// kStageBlock elements of one item (total from assign_stage_blocks).
hipError_t launch_stage_multi(const StageItem *d_items, int n_items, int64_t total, hipStream_t s);

// Many contiguous copies in one launch (device or pinned host memory on
// either side).
struct CopyItem {          // 32 bytes
  const double *src;
  double *dst;
  int64_t n;
  int64_t pad;
};
hipError_t launch_copy_multi(const CopyItem *d_items, int n_items, int64_t max_n, hipStream_t s);

// Persistent batched kernel.
struct WorkItem {           // one (geometry, p, layers) item of a plan, 96 bytes
  const TargetRec *tgt;
  const int32_t *idx;
  const double2 *xy;        // the item's SourceStage arrays
  const double2 *zq;
  const double2 *nxy;
  const double *nz;
  double *out_s;
  double *out_d;
  int32_t p;
  int32_t layers;
  int32_t accumulate;
  int32_t pad0;
  const double4 *tnrm;      // target normals (S'), device order
  double *out_t;            // S' output
};
static_assert(sizeof(WorkItem) == 96, "WorkItem layout");
struct WorkUnit {           // a run of consecutive targets of one item, 16 bytes
  int32_t item;
  int32_t first;            // first device-order target
  int32_t count;
  int32_t pad;
};
// Each wave of the persistent kernel works through units
// [wave_begin[w], wave_begin[w + 1]); consecutive waves hold consecutive
// (spatially adjacent) targets, and logical wave numbers follow the XCD
// renumbering of blocks.
struct PersistentArgs {
  const WorkItem *items;
  const WorkUnit *units;
  const int32_t *wave_begin;  // [n_waves + 1]
  int32_t n_waves;
};
// Layer classes of the persistent kernel: 1, 2 or 3 when every item has that
// mask, kLayersSingle when items mix the single masks 1 and 2 (one layer
// each), kLayersMixed when items mix masks 1..3, kLayersAny when some item
// asks for S'.  A kernel compiled for fewer masks keeps fewer registers.
constexpr unsigned kLayersMixed = 0, kLayersAny = 8, kLayersSingle = 9;
struct LayerClass {
  unsigned first = 0, all = 0;
  bool same = true, both = false;  // both: some item has mask 3
  void add(unsigned mask) {
    if (!all) first = mask;
    else if (mask != first) same = false;
    all |= mask;
    both |= mask == (TSQBX_SLP | TSQBX_DLP);
  }
  unsigned get() const {
    if (same && first >= 1 && first <= 3) return first;
    if (all & TSQBX_SPRIME) return kLayersAny;
    return both ? kLayersMixed : kLayersSingle;
  }
};
// p_all: the order shared by every item, or -1.
hipError_t launch_persistent(const PersistentArgs &a, unsigned layer_class, int p_all,
                             const Tuning &tn, hipStream_t s);
// Waves of a static schedule: oversub ranges per resident wave slot (six
// waves per SIMD, four SIMDs per CU).
int persistent_max_waves(int num_cus, int oversub);

// One Helmholtz evaluation as the pair kernels read it: a geometry, its
// Helmholtz staging and table(s), k, p and the complex outputs (null for a
// layer not requested).  The plain path builds one per launch; a plan keeps
// one per item on the device.
struct HelmWorkItem {       // 96 bytes
  const TargetRec *tgt;
  const double4 *tnrm;      // target normals (S'), device order
  const int32_t *idx;
  const double4 *rec;       // staged records, 2 per source
  const double *tab;        // (2n+1) j_n(k |t - c|), rows of p + 1
  const double *tabs;       // S' rows of 2 (p + 1), or null
  double *out_s;
  double *out_d;
  double *out_t;
  double k;
  int32_t p;
  int32_t layers;
  int32_t accumulate;
  uint32_t n_src;           // index of the padding record
};
static_assert(sizeof(HelmWorkItem) == 96, "HelmWorkItem layout");
struct HelmPersistentArgs {
  const HelmWorkItem *items;
  const WorkUnit *units;
  const int32_t *wave_begin;  // [n_waves + 1]
  int32_t n_waves;
};
// Staging of the density and the per-target table(s) of one Helmholtz
// evaluation (before the pair kernel).
hipError_t launch_helm_prepare(const tsqbx_geometry *g, int p, unsigned layers, double k,
                               const double *d_sigma, const HelmStage &st, hipStream_t s);
// The same for many evaluations in two launches (plans).
struct HelmPrepItem {       // 96 bytes
  const double4 *pos_w;     // geometry sources (x, y, z, w), device order
  const double4 *nrm;       // source normals or null
  const int64_t *perm;      // device -> caller source order, or null
  const double *sigma;      // complex, caller order
  double4 *rec;             // [2 (n + 1)]
  int64_t n;                // sources
  const TargetRec *tgt;
  int64_t n_targets;
  double k;
  int32_t p;
  int32_t pad;
  double *tab;
  double *tabs;             // S' rows, or null when S' is not requested
};
static_assert(sizeof(HelmPrepItem) == 96, "HelmPrepItem layout");
hipError_t launch_helm_prepare_multi(const HelmPrepItem *d_items, int n_items, int64_t max_n,
                                     int64_t max_t, hipStream_t s);
// The Helmholtz persistent kernel over a plan's units; layer_class as for
// launch_persistent (1..7 exact masks, or kLayersAny).
hipError_t launch_helm_persistent(const HelmPersistentArgs &a, unsigned layer_class,
                                  const Tuning &tn, hipStream_t s);
// Checks of a Helmholtz request (order, layer mask, k, normals) as
// tsqbx_eval_helmholtz makes them; TSQBX_OK or the error (message set).
int check_helmholtz_request(const tsqbx_geometry *g, int p, unsigned layers, double k);

// Static schedule for the persistent kernel: the targets of the items (in the
// given order, device order within an item) cut into at most max_waves
// contiguous ranges of about equal estimated cost.
struct ScheduleItem {
  const tsqbx_geometry *geom;
  int p;
  unsigned layers;
  bool helmholtz = false;  // costed with the Helmholtz kernel's work per pair
};
// step_cost: the fixed cost of a wave-step beyond its pairs.
void build_schedule(const std::vector<ScheduleItem> &items, const std::vector<int32_t> &order,
                    int group_lanes, int max_waves, double step_cost, std::vector<WorkUnit> *units,
                    std::vector<int32_t> *wave_begin);

// Sort every row of a CSR in place (tsqbx_lists.hip): M rows, the longest of
// at most 8192 entries, every entry in [0, max_value].  hipErrorInvalidValue
// for longer rows or larger values.
hipError_t sort_rows(const int64_t *d_offsets, int32_t *d_indices, int64_t M, int64_t longest,
                     int64_t max_value, hipStream_t s);
constexpr int64_t kRowSortMax = 8192;

// The reordered geometry built on the device from a description whose arrays
// are device pointers (tsqbx_geometry_device.hip); the same layout, bit for
// bit, as the host build.  Synchronises s before returning.
int build_geometry_device(tsqbx_ctx *ctx, const tsqbx_geometry_desc *d, hipStream_t s,
                          tsqbx_geometry **out);

// Free a geometry's device arrays and the geometry (null: nothing).
void free_geometry(tsqbx_geometry *g);

// The device address of device's scratch array (tsqbx_noalloc.hip).
hipError_t noalloc_scratch_init(int device, void **out);

Tuning default_tuning(int p, unsigned layers, int64_t mean_list);
Tuning lookup_tuning(tsqbx_ctx *ctx, int p, unsigned layers, int64_t mean_list);
uint64_t tuning_key(int p, unsigned layers, int64_t mean_list);

}  // namespace tsqbx
