// Host runtime of libtsqbx.so: errors, contexts, device-resident geometry,
// plain evaluation and tuning.  See include/tsqbx.h for the contract.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "tsqbx_internal.h"

namespace tsqbx {

static thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
  char buf[1024];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int fail_hip(hipError_t e, const char *what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(TSQBX_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
  return fail(TSQBX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// Sets the context's device for the lifetime of the guard, restoring the
// caller's current device afterwards.
struct DeviceGuard {
  int prev = -1;
  hipError_t err = hipSuccess;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) err = hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

template <class F>
static void parallel_for(int64_t n, F &&f) {
  const int64_t hw = std::max<int64_t>(1, std::min<int64_t>(16, std::thread::hardware_concurrency()));
  const int64_t nt = std::min<int64_t>(hw, std::max<int64_t>(1, n / 256));
  if (nt <= 1) {
    for (int64_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::vector<std::thread> th;
  std::atomic<int64_t> next{0};
  for (int64_t k = 0; k < nt; ++k)
    th.emplace_back([&] {
      for (;;) {
        const int64_t b = next.fetch_add(64);
        if (b >= n) break;
        const int64_t e = std::min(n, b + 64);
        for (int64_t i = b; i < e; ++i) f(i);
      }
    });
  for (auto &t : th) t.join();
}

// 63-bit Morton keys of points in their bounding box (21 bits per axis).
static uint64_t spread21(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

static std::vector<uint64_t> morton_keys(const double *xyz, int64_t n) {
  std::vector<uint64_t> key(n);
  if (n == 0) return key;
  double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
  for (int64_t i = 0; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], xyz[3 * i + a]);
      hi[a] = std::max(hi[a], xyz[3 * i + a]);
    }
  double span = std::max({hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2], 1e-300});
  const double scale = double((1 << 21) - 1) / span;
  for (int64_t i = 0; i < n; ++i) {
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
      double v = (xyz[3 * i + a] - lo[a]) * scale;
      v = std::min(std::max(v, 0.0), double((1 << 21) - 1));
      q[a] = (uint64_t)v;
    }
    key[i] = spread21(q[0]) << 2 | spread21(q[1]) << 1 | spread21(q[2]);
  }
  return key;
}

static std::vector<int64_t> order_by_key(const std::vector<uint64_t> &key) {
  std::vector<int64_t> ord(key.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) {
    return key[a] != key[b] ? key[a] < key[b] : a < b;
  });
  return ord;
}

static int validate(const tsqbx_geometry_desc *d) {
  if (!d) return fail(TSQBX_E_INVALID, "geometry description is NULL");
  if (d->n_sources < 0 || d->n_centers < 0 || d->n_targets < 0)
    return fail(TSQBX_E_INVALID, "negative count (sources %lld, centers %lld, targets %lld)",
                (long long)d->n_sources, (long long)d->n_centers, (long long)d->n_targets);
  if (d->n_sources >= TSQBX_MAX_SOURCES)
    return fail(TSQBX_E_RANGE, "n_sources = %lld; a geometry holds fewer than %lld sources",
                (long long)d->n_sources, (long long)TSQBX_MAX_SOURCES);
  if (d->n_targets > INT32_MAX || d->n_centers > INT32_MAX)
    return fail(TSQBX_E_RANGE, "counts must stay below 2^31");
  if (d->n_sources > 0 && (!d->sources || !d->weights))
    return fail(TSQBX_E_INVALID, "sources or weights is NULL");
  if (d->n_centers > 0 && !d->centers) return fail(TSQBX_E_INVALID, "centers is NULL");
  if (!d->list_offsets) return fail(TSQBX_E_INVALID, "list_offsets is NULL");
  if (d->n_targets > 0 && !d->targets) return fail(TSQBX_E_INVALID, "targets is NULL");
  if (!d->target_center && d->n_targets > 0 && d->n_targets != d->n_centers)
    return fail(TSQBX_E_INVALID, "target_center is NULL but n_targets (%lld) != n_centers (%lld)",
                (long long)d->n_targets, (long long)d->n_centers);
  const int64_t *off = d->list_offsets;
  if (off[0] != 0) return fail(TSQBX_E_INVALID, "list_offsets[0] = %lld, expected 0", (long long)off[0]);
  for (int64_t i = 0; i < d->n_centers; ++i) {
    if (off[i + 1] < off[i])
      return fail(TSQBX_E_INVALID, "list_offsets decreases at center %lld", (long long)i);
    if (off[i + 1] - off[i] > (int64_t(1) << 30) - kRowPad)
      return fail(TSQBX_E_RANGE, "list of center %lld is longer than 2^30 - %d entries",
                  (long long)i, kRowPad);
  }
  const int64_t nnz = off[d->n_centers];
  if (nnz > 0 && !d->list_sources) return fail(TSQBX_E_INVALID, "list_sources is NULL");
  // the first entry out of range, over blocks of the list array in parallel
  constexpr int64_t kBlk = int64_t(1) << 16;
  const int64_t nblk = (nnz + kBlk - 1) / kBlk;
  std::atomic<int64_t> first_bad{INT64_MAX};
  parallel_for(nblk, [&](int64_t b) {
    const int64_t e = std::min(nnz, (b + 1) * kBlk);
    for (int64_t j = b * kBlk; j < e; ++j) {
      const int32_t s = d->list_sources[j];
      if (s < 0 || (int64_t)s >= d->n_sources) {
        int64_t cur = first_bad.load();
        while (j < cur && !first_bad.compare_exchange_weak(cur, j)) {
        }
        return;
      }
    }
  });
  if (first_bad.load() != INT64_MAX) {
    const int64_t j = first_bad.load();
    return fail(TSQBX_E_RANGE, "list_sources[%lld] = %d is outside [0, %lld)", (long long)j,
                d->list_sources[j], (long long)d->n_sources);
  }
  if (d->target_center)
    for (int64_t t = 0; t < d->n_targets; ++t) {
      const int32_t c = d->target_center[t];
      if (c < 0 || (int64_t)c >= d->n_centers)
        return fail(TSQBX_E_RANGE, "target_center[%lld] = %d is outside [0, %lld)", (long long)t, c,
                    (long long)d->n_centers);
    }
  return TSQBX_OK;
}

static int check_request(const tsqbx_geometry *g, int p, unsigned layers) {
  if (p < 0 || p > TSQBX_P_MAX)
    return fail(TSQBX_E_RANGE, "expansion order p = %d is outside [0, %d]", p, TSQBX_P_MAX);
  if (layers == 0 || (layers & ~7u))
    return fail(TSQBX_E_INVALID, "layers = %u is not a nonempty subset of SLP|DLP|SPRIME", layers);
  if (g && (layers & TSQBX_DLP) && !g->has_normals)
    return fail(TSQBX_E_INVALID, "double layer requested but the geometry has no normals");
  if (g && (layers & TSQBX_SPRIME) && !g->has_target_normals)
    return fail(TSQBX_E_INVALID, "S' requested but the geometry has no target normals");
  return TSQBX_OK;
}

// Tuning buckets: a Laplace layer mask, or SLP|DLP with TSQBX_HELMHOLTZ.
static int check_tuning_key(int p, unsigned layers) {
  if (layers & TSQBX_HELMHOLTZ) {
    const unsigned l = layers & ~(unsigned)TSQBX_HELMHOLTZ;
    if (p < 0 || p > TSQBX_P_MAX)
      return fail(TSQBX_E_RANGE, "expansion order p = %d is outside [0, %d]", p, TSQBX_P_MAX);
    if (l == 0 || (l & ~7u))
      return fail(TSQBX_E_INVALID, "Helmholtz layers = %u is not a nonempty subset of SLP|DLP|SPRIME", l);
    return TSQBX_OK;
  }
  return check_request(nullptr, p, layers);
}

uint64_t tuning_key(int p, unsigned layers, int64_t mean_list) {
  int bucket = 0;
  while (bucket < 40 && (int64_t(1) << (bucket + 1)) <= mean_list) ++bucket;
  return (uint64_t)p << 16 | (uint64_t)layers << 8 | (uint64_t)bucket;
}

Tuning default_tuning(int p, unsigned layers, int64_t mean_list) {
  (void)p;
  Tuning t;
  t.xcd_remap = 1;
  // short lists: several targets per wave; long lists: one target per wave
  t.group_lanes = mean_list < 384 ? 16 : 64;
  t.unroll = 2;
  // the plain Laplace kernel with one target per wave: blocks of 8 adjacent
  // targets (their lists overlap, and the block's waves share the L1)
  t.waves_per_block = (t.group_lanes == 64 && !(layers & TSQBX_HELMHOLTZ)) ? 8 : 4;
  return t;
}

Tuning lookup_tuning(tsqbx_ctx *ctx, int p, unsigned layers, int64_t mean_list) {
  std::lock_guard<std::mutex> lk(ctx->tuning_mu);
  auto it = ctx->tuning.find(tuning_key(p, layers, mean_list));
  if (it != ctx->tuning.end()) return it->second;
  return default_tuning(p, layers, mean_list);
}

static int64_t mean_list_of(const tsqbx_geometry *g) {
  return g->n_targets > 0 ? (g->pairs + g->n_targets - 1) / g->n_targets : 0;
}

}  // namespace tsqbx

void tsqbx::free_geometry(tsqbx_geometry *g) {
  if (!g) return;
  void *ptrs[] = {g->src_pos, g->src_w, g->src_nrm, g->src_perm, g->src_rank, g->tgt, g->tgt_nrm, g->idx,
                  g->ctr, g->row_tgts, g->stage.xy, g->stage.nxy, g->helm.rec, g->helm.tab,
                  g->helm.tabs};
  for (void *p : ptrs)
    if (p) (void)hipFree(p);
  delete g;
}

namespace tsqbx {

template <class T>
static hipError_t dev_upload(T **dst, const T *src, size_t n, size_t *bytes) {
  *dst = nullptr;
  if (n == 0) return hipSuccess;
  hipError_t e = hipMalloc((void **)dst, n * sizeof(T));
  if (e != hipSuccess) return e;
  *bytes += n * sizeof(T);
  if (src) return hipMemcpy(*dst, src, n * sizeof(T), hipMemcpyHostToDevice);
  return hipSuccess;
}

}  // namespace tsqbx

using namespace tsqbx;

extern "C" {

int tsqbx_version(void) { return 10300; }

const char *tsqbx_last_error(void) { return g_err.c_str(); }

int tsqbx_validate_geometry(const tsqbx_geometry_desc *desc) { return validate(desc); }

int tsqbx_check_request(const tsqbx_geometry *geom, int p, unsigned layers) {
  return check_request(geom, p, layers);
}

int tsqbx_ctx_create(int device, tsqbx_ctx **out) {
  if (!out) return fail(TSQBX_E_INVALID, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return fail_hip(e, "hipGetDeviceCount");
  if (device < 0 || device >= n)
    return fail(TSQBX_E_RANGE, "device %d is outside [0, %d)", device, n);
  DeviceGuard dg(device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  auto *c = new tsqbx_ctx;
  c->device = device;
  e = hipDeviceGetAttribute(&c->num_cus, hipDeviceAttributeMultiprocessorCount, device);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = noalloc_scratch_init(device, &c->scratch);
  if (e != hipSuccess) {
    if (c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return fail_hip(e, "context setup");
  }
  *out = c;
  return TSQBX_OK;
}

int tsqbx_ctx_destroy(tsqbx_ctx *ctx) {
  if (!ctx) return TSQBX_OK;
  DeviceGuard dg(ctx->device);
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  if (ctx->d_sigma) (void)hipFree(ctx->d_sigma);
  if (ctx->d_out) (void)hipFree(ctx->d_out);
  if (ctx->stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
  return TSQBX_OK;
}

// The device layout of a geometry, computed on the host (see
// tsqbx_geometry_layout): source and target orders, one row per distinct
// center in order of first use, rows padded to kRowPad with the padding
// record N, entries remapped to device source numbers and sorted.
struct HostLayout {
  std::vector<int64_t> src_ord;        // device -> caller source
  std::vector<int32_t> src_rank;       // caller -> device source
  std::vector<int32_t> tc;             // caller target -> center
  std::vector<int64_t> tgt_ord;        // device -> caller target
  std::vector<int64_t> row_of_center;  // center -> row, -1 if no target uses it
  std::vector<int64_t> row_center;     // row -> center
  std::vector<int64_t> row_off;        // [R + 1] padded offsets
  std::vector<int32_t> idx;            // [nnz_dev]
};

static void build_layout(const tsqbx_geometry_desc *d, bool reorder, HostLayout *L) {
  const int64_t N = d->n_sources, M = d->n_centers, T = d->n_targets;
  // device order of sources (Morton) and its inverse
  L->src_ord.resize(N);
  std::iota(L->src_ord.begin(), L->src_ord.end(), 0);
  if (reorder && N > 1) L->src_ord = order_by_key(morton_keys(d->sources, N));
  L->src_rank.resize(N);
  for (int64_t i = 0; i < N; ++i) L->src_rank[L->src_ord[i]] = (int32_t)i;

  // device order of targets: by Morton key of their center, then center, then index
  std::vector<int32_t> &tc = L->tc;
  tc.resize(T);
  for (int64_t t = 0; t < T; ++t) tc[t] = d->target_center ? d->target_center[t] : (int32_t)t;
  std::vector<int64_t> &tgt_ord = L->tgt_ord;
  tgt_ord.resize(T);
  std::iota(tgt_ord.begin(), tgt_ord.end(), 0);
  if (reorder && T > 1) {
    std::vector<uint64_t> ckey = morton_keys(d->centers, M);
    std::sort(tgt_ord.begin(), tgt_ord.end(), [&](int64_t a, int64_t b) {
      const uint64_t ka = ckey[tc[a]], kb = ckey[tc[b]];
      if (ka != kb) return ka < kb;
      if (tc[a] != tc[b]) return tc[a] < tc[b];
      return a < b;
    });
  }

  // one device row per distinct center, in order of first use
  L->row_of_center.assign(M, -1);
  L->row_center.clear();
  for (int64_t k = 0; k < T; ++k) {
    const int32_t c = tc[tgt_ord[k]];
    if (L->row_of_center[c] < 0) {
      L->row_of_center[c] = (int64_t)L->row_center.size();
      L->row_center.push_back(c);
    }
  }
  const int64_t R = (int64_t)L->row_center.size();
  L->row_off.assign(R + 1, 0);
  // rows padded to a multiple of kRowPad with the zero-strength record N
  for (int64_t r = 0; r < R; ++r) {
    const int64_t c = L->row_center[r];
    const int64_t len = d->list_offsets[c + 1] - d->list_offsets[c];
    L->row_off[r + 1] = L->row_off[r] + (len + kRowPad - 1) / kRowPad * kRowPad;
  }
  L->idx.resize(L->row_off[R]);
  parallel_for(R, [&](int64_t r) {
    const int64_t c = L->row_center[r];
    const int64_t b = d->list_offsets[c], e = d->list_offsets[c + 1];
    int32_t *dst = L->idx.data() + L->row_off[r];
    for (int64_t j = b; j < e; ++j) dst[j - b] = L->src_rank[d->list_sources[j]];
    std::sort(dst, dst + (e - b));
    for (int64_t j = e - b; j < L->row_off[r + 1] - L->row_off[r]; ++j) dst[j] = (int32_t)N;
  });
}

int tsqbx_geometry_layout(const tsqbx_geometry_desc *d, unsigned flags, int64_t *source_order,
                          int64_t *target_order, int64_t *target_row, int64_t *row_offsets,
                          int64_t row_offsets_cap, int32_t *rows, int64_t rows_cap,
                          tsqbx_layout_info *info) {
  TraceRange trace_("tsqbx_geometry_layout");
  if (!info) return fail(TSQBX_E_INVALID, "geometry_layout: info is NULL");
  int rc = validate(d);
  if (rc != TSQBX_OK) return rc;
  HostLayout L;
  build_layout(d, !(flags & TSQBX_NO_REORDER), &L);
  const int64_t R = (int64_t)L.row_center.size(), nnz = L.row_off[R];
  info->n_rows = R;
  info->nnz = nnz;
  info->pairs = 0;
  info->max_list = 0;
  for (int64_t t = 0; t < d->n_targets; ++t) {
    const int64_t len = d->list_offsets[L.tc[t] + 1] - d->list_offsets[L.tc[t]];
    info->pairs += len;
    info->max_list = std::max(info->max_list, len);
  }
  if ((row_offsets && row_offsets_cap < R + 1) || (rows && rows_cap < nnz))
    return fail(TSQBX_E_RANGE, "geometry_layout: %lld rows of %lld entries do not fit the buffers",
                (long long)R, (long long)nnz);
  if (source_order) std::copy(L.src_ord.begin(), L.src_ord.end(), source_order);
  if (target_order) std::copy(L.tgt_ord.begin(), L.tgt_ord.end(), target_order);
  if (target_row)
    for (int64_t k = 0; k < d->n_targets; ++k) target_row[k] = L.row_of_center[L.tc[L.tgt_ord[k]]];
  if (row_offsets) std::copy(L.row_off.begin(), L.row_off.end(), row_offsets);
  if (rows) std::copy(L.idx.begin(), L.idx.end(), rows);
  return TSQBX_OK;
}

// A reordered geometry with at least this many list entries is laid out on
// the device: the caller's arrays go up as they are and the device build
// (the same layout, bit for bit) reorders and remaps them there, about ten
// times faster than the host for a few million entries and more.
constexpr int64_t kDeviceBuildMinEntries = int64_t(1) << 20;

static int create_via_device(tsqbx_ctx *ctx, const tsqbx_geometry_desc *d, tsqbx_geometry **out) {
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  const int64_t N = d->n_sources, M = d->n_centers, T = d->n_targets;
  const int64_t nnz = d->list_offsets[M];
  std::vector<void *> tmp;
  struct Free {
    std::vector<void *> &v;
    ~Free() {
      for (void *p : v) (void)hipFree(p);
    }
  } fr{tmp};
  hipError_t e = hipSuccess;
  auto up = [&](const void *src, size_t bytes) -> void * {
    if (!src || bytes == 0 || e != hipSuccess) return nullptr;
    void *p = nullptr;
    e = hipMalloc(&p, bytes);
    if (e != hipSuccess) return nullptr;
    tmp.push_back(p);
    e = hipMemcpy(p, src, bytes, hipMemcpyHostToDevice);
    return p;
  };
  tsqbx_geometry_desc dd = *d;
  dd.sources = (const double *)up(d->sources, 3 * N * sizeof(double));
  dd.weights = (const double *)up(d->weights, N * sizeof(double));
  dd.normals = (const double *)up(d->normals, 3 * N * sizeof(double));
  dd.centers = (const double *)up(d->centers, 3 * M * sizeof(double));
  dd.list_offsets = (const int64_t *)up(d->list_offsets, (M + 1) * sizeof(int64_t));
  dd.list_sources = (const int32_t *)up(d->list_sources, nnz * sizeof(int32_t));
  dd.targets = (const double *)up(d->targets, 3 * T * sizeof(double));
  dd.target_center = (const int32_t *)up(d->target_center, T * sizeof(int32_t));
  dd.target_normals = (const double *)up(d->target_normals, 3 * T * sizeof(double));
  if (e != hipSuccess) return fail_hip(e, "geometry upload");
  return build_geometry_device(ctx, &dd, ctx->stream, out);  // synchronises before returning
}

int tsqbx_geometry_create(tsqbx_ctx *ctx, const tsqbx_geometry_desc *d, unsigned flags,
                          tsqbx_geometry **out) {
  TraceRange trace_("tsqbx_geometry_create");
  if (!ctx || !out) return fail(TSQBX_E_INVALID, "ctx or out is NULL");
  *out = nullptr;
  int rc = validate(d);
  if (rc != TSQBX_OK) return rc;
  const int64_t N = d->n_sources, M = d->n_centers, T = d->n_targets;
  const bool reorder = !(flags & TSQBX_NO_REORDER);
  if (reorder && d->list_offsets[M] >= kDeviceBuildMinEntries) return create_via_device(ctx, d, out);
  HostLayout L;
  build_layout(d, reorder, &L);
  const std::vector<int64_t> &src_ord = L.src_ord, &tgt_ord = L.tgt_ord;
  const std::vector<int32_t> &src_rank = L.src_rank, &tc = L.tc;
  const std::vector<int64_t> &row_of_center = L.row_of_center, &row_center = L.row_center;
  const std::vector<int64_t> &row_off = L.row_off;
  std::vector<int32_t> &idx = L.idx;
  const int64_t R = (int64_t)row_center.size();
  const int64_t nnz_dev = row_off[R];
  (void)M;

  std::vector<TargetRec> recs(T);
  std::vector<double4> tnrm(d->target_normals ? T : 0);
  int64_t pairs = 0, max_list = 0;
  std::vector<int64_t> host_row_len(T);
  for (int64_t k = 0; k < T; ++k) {
    const int64_t t = tgt_ord[k];
    const int32_t c = tc[t];
    const int64_t r = row_of_center[c];
    TargetRec &x = recs[k];
    for (int a = 0; a < 3; ++a) {
      x.c[a] = d->centers[3 * c + a];
      x.d[a] = d->targets[3 * t + a] - d->centers[3 * c + a];
    }
    const int64_t len = d->list_offsets[c + 1] - d->list_offsets[c];
    x.row_begin = row_off[r];
    x.row_len = (int32_t)(row_off[r + 1] - row_off[r]);
    x.out_index = (int32_t)t;
    if (d->target_normals)
      tnrm[k] = make_double4(d->target_normals[3 * t], d->target_normals[3 * t + 1],
                             d->target_normals[3 * t + 2], 0.0);
    pairs += len;
    max_list = std::max<int64_t>(max_list, len);
    host_row_len[k] = len;
  }

  int64_t g_max_row_targets = 0;
  // rows for the conventional path: center, unpadded list, targets by row
  std::vector<CenterRec> crec(R);
  std::vector<int32_t> row_tgts(T);
  {
    std::vector<int64_t> cnt(R + 1, 0);
    for (int64_t k = 0; k < T; ++k) ++cnt[row_of_center[tc[tgt_ord[k]]] + 1];
    for (int64_t r = 0; r < R; ++r) cnt[r + 1] += cnt[r];
    for (int64_t r = 0; r < R; ++r) {
      const int32_t c = (int32_t)row_center[r];
      CenterRec &x = crec[r];
      for (int a = 0; a < 3; ++a) x.c[a] = d->centers[3 * c + a];
      x.row_begin = row_off[r];
      x.len = (int32_t)(d->list_offsets[c + 1] - d->list_offsets[c]);
      x.center = c;
      x.tgt_begin = (int32_t)cnt[r];
      x.tgt_count = (int32_t)(cnt[r + 1] - cnt[r]);
      x.pad = 0;
      g_max_row_targets = std::max<int64_t>(g_max_row_targets, x.tgt_count);
    }
    std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
    for (int64_t k = 0; k < T; ++k) row_tgts[fill[row_of_center[tc[tgt_ord[k]]]]++] = (int32_t)k;
  }

  std::vector<double4> pos(N), nrm(d->normals ? N : 0);
  std::vector<double> wdev(N);
  std::vector<int64_t> perm(reorder ? N : 0);
  for (int64_t i = 0; i < N; ++i) {
    const int64_t s = src_ord[i];
    pos[i] = make_double4(d->sources[3 * s], d->sources[3 * s + 1], d->sources[3 * s + 2],
                          d->weights[s]);
    wdev[i] = d->weights[s];
    if (d->normals)
      nrm[i] = make_double4(d->normals[3 * s], d->normals[3 * s + 1], d->normals[3 * s + 2], 0.0);
    if (reorder) perm[i] = s;
  }

  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  auto *g = new tsqbx_geometry;
  g->ctx = ctx;
  g->device = ctx->device;
  g->n_sources = N;
  g->n_centers = M;
  g->n_targets = T;
  g->nnz = nnz_dev;
  g->pairs = pairs;
  g->max_list = max_list;
  g->has_normals = d->normals != nullptr;
  g->has_target_normals = d->target_normals != nullptr;
  g->host_row_len = std::move(host_row_len);
  size_t bytes = 0;
  hipError_t e = dev_upload(&g->src_pos, pos.data(), N, &bytes);
  if (e == hipSuccess) e = dev_upload(&g->src_w, wdev.data(), N, &bytes);
  if (e == hipSuccess && d->normals) e = dev_upload(&g->src_nrm, nrm.data(), N, &bytes);
  if (e == hipSuccess && reorder) e = dev_upload(&g->src_perm, perm.data(), N, &bytes);
  if (e == hipSuccess && reorder) e = dev_upload(&g->src_rank, src_rank.data(), N, &bytes);
  if (e == hipSuccess) e = dev_upload(&g->tgt, recs.data(), T, &bytes);
  if (e == hipSuccess && d->target_normals) e = dev_upload(&g->tgt_nrm, tnrm.data(), T, &bytes);
  if (e == hipSuccess) e = dev_upload(&g->idx, idx.data(), nnz_dev, &bytes);
  g->n_rows = R;
  g->max_row_targets = g_max_row_targets;
  if (e == hipSuccess) e = dev_upload(&g->ctr, crec.data(), R, &bytes);
  if (e == hipSuccess) e = dev_upload(&g->row_tgts, row_tgts.data(), T, &bytes);
  // staging blocks of the plain path (see SourceStage)
  char *spos = nullptr, *snrm = nullptr;
  if (e == hipSuccess) e = dev_upload<char>(&spos, nullptr, stage_pos_bytes(N), &bytes);
  if (e == hipSuccess && d->normals) e = dev_upload<char>(&snrm, nullptr, stage_nrm_bytes(N), &bytes);
  g->stage = stage_views(spos, snrm, N);
  // the positions and the padding entry, once: evaluations stage strengths only
  if (e == hipSuccess) e = launch_stage_positions(g, g->stage, nullptr);
  if (e == hipSuccess) e = hipStreamSynchronize(nullptr);
  if (e != hipSuccess) {
    free_geometry(g);
    return fail_hip(e, "geometry upload");
  }
  g->device_bytes = bytes;
  *out = g;
  return TSQBX_OK;
}

int tsqbx_geometry_destroy(tsqbx_geometry *g) {
  if (!g) return TSQBX_OK;
  DeviceGuard dg(g->device);
  (void)hipDeviceSynchronize();
  free_geometry(g);
  return TSQBX_OK;
}

int tsqbx_geometry_get_info(const tsqbx_geometry *g, tsqbx_geometry_info *out) {
  if (!g || !out) return fail(TSQBX_E_INVALID, "geometry or out is NULL");
  out->n_sources = g->n_sources;
  out->n_centers = g->n_centers;
  out->n_targets = g->n_targets;
  out->nnz = g->nnz;
  out->pairs = g->pairs;
  out->max_list = g->max_list;
  out->device_bytes = g->device_bytes;
  out->has_normals = g->has_normals ? 1 : 0;
  out->has_target_normals = g->has_target_normals ? 1 : 0;
  return TSQBX_OK;
}

// A NULL output for a requested layer, with targets to write, is an error.
static int check_outputs(const tsqbx_geometry *g, unsigned layers, const double *o_s,
                         const double *o_d, const double *o_t) {
  if (g->n_targets > 0 && (((layers & TSQBX_SLP) && !o_s) || ((layers & TSQBX_DLP) && !o_d) ||
                           ((layers & TSQBX_SPRIME) && !o_t)))
    return fail(TSQBX_E_INVALID, "output for a requested layer is NULL");
  return TSQBX_OK;
}

int tsqbx_eval_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, unsigned layers,
                     const double *d_sigma, double *d_out_slp, double *d_out_dlp,
                     double *d_out_sprime, unsigned flags, void *hip_stream) {
  TraceRange trace_("tsqbx_eval_async");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = check_request(g, p, layers);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !d_sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  rc = check_outputs(g, layers, d_out_slp, d_out_dlp, d_out_sprime);
  if (rc != TSQBX_OK) return rc;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  const Tuning tn = lookup_tuning(ctx, p, layers, mean_list_of(g));
  Outputs o;
  o.s = d_out_slp;
  o.d = d_out_dlp;
  o.t = d_out_sprime;
  TSQBX_HIP(launch_stage(g, d_sigma, layers, g->stage, true, s));
  g->staged_layers.store(layers);
  TSQBX_HIP(launch_eval_plain(g, p, layers, g->stage, o, (flags & TSQBX_ACCUMULATE) != 0, tn,
                              (flags & TSQBX_PER_TARGET) != 0, s));
  return TSQBX_OK;
}

int tsqbx_stage_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, unsigned layers,
                      const double *d_sigma, void *hip_stream) {
  TraceRange trace_("tsqbx_stage_async");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = check_request(g, 0, layers);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !d_sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  TSQBX_HIP(launch_stage(g, d_sigma, layers, g->stage, true, (hipStream_t)hip_stream));
  g->staged_layers.store(layers);
  return TSQBX_OK;
}

int tsqbx_eval_staged_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, unsigned layers,
                            double *d_out_slp, double *d_out_dlp, double *d_out_sprime,
                            unsigned flags, void *hip_stream) {
  TraceRange trace_("tsqbx_eval_staged_async");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = check_request(g, p, layers);
  if (rc != TSQBX_OK) return rc;
  const unsigned st = g->staged_layers.load();
  if (!st || ((layers & TSQBX_DLP) && !(st & TSQBX_DLP)))
    return fail(TSQBX_E_STATE, "the geometry's sources are not staged for layers %u", layers);
  rc = check_outputs(g, layers, d_out_slp, d_out_dlp, d_out_sprime);
  if (rc != TSQBX_OK) return rc;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  const Tuning tn = lookup_tuning(ctx, p, layers, mean_list_of(g));
  Outputs o;
  o.s = d_out_slp;
  o.d = d_out_dlp;
  o.t = d_out_sprime;
  TSQBX_HIP(launch_eval_plain(g, p, layers, g->stage, o, (flags & TSQBX_ACCUMULATE) != 0, tn,
                              (flags & TSQBX_PER_TARGET) != 0, (hipStream_t)hip_stream));
  return TSQBX_OK;
}

// Conventional QBX (Sec. 2.3): checks shared by the three entry points.
static int check_conventional(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p) {
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  return check_request(g, p, TSQBX_SLP);
}

int tsqbx_qbxl_form_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, const double *d_sigma,
                          double *d_coeffs, unsigned flags, void *hip_stream) {
  TraceRange trace_("tsqbx_qbxl_form_async");
  int rc = check_conventional(ctx, g, p);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !d_sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  if (g->n_rows > 0 && !d_coeffs) return fail(TSQBX_E_INVALID, "coefficient buffer is NULL");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  TSQBX_HIP(launch_stage(g, d_sigma, TSQBX_SLP, g->stage, true, s));
  g->staged_layers.store(TSQBX_SLP);
  TSQBX_HIP(launch_qbxl(g, p, 1, g->stage, nullptr, d_coeffs, nullptr,
                        (flags & TSQBX_ACCUMULATE) != 0, s));
  return TSQBX_OK;
}

int tsqbx_qbxl_eval_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, const double *d_coeffs,
                          double *d_out, unsigned flags, void *hip_stream) {
  TraceRange trace_("tsqbx_qbxl_eval_async");
  int rc = check_conventional(ctx, g, p);
  if (rc != TSQBX_OK) return rc;
  if (g->n_rows > 0 && !d_coeffs) return fail(TSQBX_E_INVALID, "coefficient buffer is NULL");
  if (g->n_targets > 0 && !d_out) return fail(TSQBX_E_INVALID, "output is NULL");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  TSQBX_HIP(launch_qbxl(g, p, 2, SourceStage{}, d_coeffs, nullptr, d_out,
                        (flags & TSQBX_ACCUMULATE) != 0, (hipStream_t)hip_stream));
  return TSQBX_OK;
}

int tsqbx_eval_conventional_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p,
                                  const double *d_sigma, double *d_out, unsigned flags,
                                  void *hip_stream) {
  TraceRange trace_("tsqbx_eval_conventional_async");
  int rc = check_conventional(ctx, g, p);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !d_sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  if (g->n_targets > 0 && !d_out) return fail(TSQBX_E_INVALID, "output is NULL");
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  hipStream_t s = (hipStream_t)hip_stream;
  TSQBX_HIP(launch_stage(g, d_sigma, TSQBX_SLP, g->stage, true, s));
  g->staged_layers.store(TSQBX_SLP);
  TSQBX_HIP(launch_qbxl(g, p, 3, g->stage, nullptr, nullptr, d_out,
                        (flags & TSQBX_ACCUMULATE) != 0, s));
  return TSQBX_OK;
}

int tsqbx_eval(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, unsigned layers,
               const double *sigma, double *out_slp, double *out_dlp, double *out_sprime,
               unsigned flags) {
  TraceRange trace_("tsqbx_eval");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = check_request(g, p, layers);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  rc = check_outputs(g, layers, out_slp, out_dlp, out_sprime);
  if (rc != TSQBX_OK) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  const size_t N = (size_t)g->n_sources, T = (size_t)g->n_targets;
  if (ctx->d_sigma_cap < N) {
    if (ctx->d_sigma) (void)hipFree(ctx->d_sigma);
    ctx->d_sigma = nullptr;
    ctx->d_sigma_cap = 0;
    TSQBX_HIP(hipMalloc((void **)&ctx->d_sigma, N * sizeof(double)));
    ctx->d_sigma_cap = N;
  }
  if (ctx->d_out_cap < 3 * T) {
    if (ctx->d_out) (void)hipFree(ctx->d_out);
    ctx->d_out = nullptr;
    ctx->d_out_cap = 0;
    TSQBX_HIP(hipMalloc((void **)&ctx->d_out, 3 * T * sizeof(double)));
    ctx->d_out_cap = 3 * T;
  }
  hipStream_t s = ctx->stream;
  if (N) TSQBX_HIP(hipMemcpyAsync(ctx->d_sigma, sigma, N * sizeof(double), hipMemcpyHostToDevice, s));
  Outputs o;
  o.s = ctx->d_out;
  o.d = ctx->d_out + T;
  o.t = ctx->d_out + 2 * T;
  const Tuning tn = lookup_tuning(ctx, p, layers, mean_list_of(g));
  TSQBX_HIP(launch_stage(g, ctx->d_sigma, layers, g->stage, true, s));
  g->staged_layers.store(layers);
  TSQBX_HIP(launch_eval_plain(g, p, layers, g->stage, o, false, tn,
                              (flags & TSQBX_PER_TARGET) != 0, s));
  // without ACCUMULATE the outputs go straight into the caller's arrays
  const bool acc = (flags & TSQBX_ACCUMULATE) != 0;
  double *const dev[3] = {o.s, o.d, o.t};
  double *const user[3] = {out_slp, out_dlp, out_sprime};
  const unsigned bit[3] = {TSQBX_SLP, TSQBX_DLP, TSQBX_SPRIME};
  std::vector<double> tmp[3];
  for (int l = 0; l < 3; ++l) {
    if (!T || !(layers & bit[l])) continue;
    double *dst = user[l];
    if (acc) {
      tmp[l].resize(T);
      dst = tmp[l].data();
    }
    TSQBX_HIP(hipMemcpyAsync(dst, dev[l], T * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  TSQBX_HIP(hipStreamSynchronize(s));
  for (int l = 0; l < 3; ++l)
    for (size_t i = 0; i < tmp[l].size(); ++i) user[l][i] += tmp[l][i];
  return TSQBX_OK;
}

int tsqbx_get_tuning(tsqbx_ctx *ctx, int p, unsigned layers, int64_t mean_list,
                     tsqbx_tuning *out) {
  if (!ctx || !out) return fail(TSQBX_E_INVALID, "ctx or out is NULL");
  int rc = check_tuning_key(p, layers);
  if (rc != TSQBX_OK) return rc;
  const Tuning t = lookup_tuning(ctx, p, layers, mean_list);
  out->waves_per_block = t.waves_per_block;
  out->group_lanes = t.group_lanes;
  out->unroll = t.unroll;
  out->xcd_remap = t.xcd_remap;
  return TSQBX_OK;
}

int tsqbx_set_tuning(tsqbx_ctx *ctx, int p, unsigned layers, int64_t mean_list,
                     const tsqbx_tuning *tuning) {
  if (!ctx || !tuning) return fail(TSQBX_E_INVALID, "ctx or tuning is NULL");
  int rc = check_tuning_key(p, layers);
  if (rc != TSQBX_OK) return rc;
  Tuning t;
  t.waves_per_block = tuning->waves_per_block;
  t.group_lanes = tuning->group_lanes;
  t.unroll = tuning->unroll;
  t.xcd_remap = tuning->xcd_remap;
  if (!((layers & TSQBX_HELMHOLTZ) ? tuning_supported(t) : eval_tuning_supported(t)))
    return fail(TSQBX_E_INVALID, "unsupported tuning (waves %d, group %d, unroll %d, remap %d)",
                t.waves_per_block, t.group_lanes, t.unroll, t.xcd_remap);
  std::lock_guard<std::mutex> lk(ctx->tuning_mu);
  ctx->tuning[tuning_key(p, layers, mean_list)] = t;
  return TSQBX_OK;
}

// The device's architecture name and the HIP runtime version: the tag of a
// saved tuning entry.
static int tuning_tag(const tsqbx_ctx *ctx, std::string *arch, int *runtime) {
  hipDeviceProp_t prop;
  hipError_t e = hipGetDeviceProperties(&prop, ctx->device);
  if (e != hipSuccess) return fail_hip(e, "hipGetDeviceProperties");
  arch->assign(prop.gcnArchName);
  for (char &c : *arch)
    if (c == '"' || c == '\\' || (unsigned char)c < 32) c = '_';
  e = hipRuntimeGetVersion(runtime);
  if (e != hipSuccess) return fail_hip(e, "hipRuntimeGetVersion");
  return TSQBX_OK;
}

int tsqbx_tuning_save(tsqbx_ctx *ctx, const char *path) {
  if (!ctx || !path) return fail(TSQBX_E_INVALID, "ctx or path is NULL");
  std::string arch;
  int rt = 0;
  int rc = tuning_tag(ctx, &arch, &rt);
  if (rc != TSQBX_OK) return rc;
  std::map<uint64_t, Tuning> plain;
  std::map<uint64_t, PlanTuning> plans;
  {
    std::lock_guard<std::mutex> lk(ctx->tuning_mu);
    plain = ctx->tuning;
    plans = ctx->plan_tuning;
  }
  FILE *f = std::fopen(path, "w");
  if (!f) return fail(TSQBX_E_INVALID, "tuning_save: cannot open %s for writing", path);
  for (auto &kv : plain)
    std::fprintf(f,
                 "{\"kind\": \"plain\", \"arch\": \"%s\", \"runtime\": %d, \"key\": %llu, "
                 "\"group_lanes\": %d, \"unroll\": %d, \"waves_per_block\": %d, "
                 "\"xcd_remap\": %d}\n",
                 arch.c_str(), rt, (unsigned long long)kv.first, kv.second.group_lanes,
                 kv.second.unroll, kv.second.waves_per_block, kv.second.xcd_remap);
  for (auto &kv : plans)
    std::fprintf(f,
                 "{\"kind\": \"plan\", \"arch\": \"%s\", \"runtime\": %d, \"key\": %llu, "
                 "\"group_lanes\": %d, \"unroll\": %d, \"waves_per_block\": %d, "
                 "\"oversubscription\": %d, \"step_cost\": %d}\n",
                 arch.c_str(), rt, (unsigned long long)kv.first, kv.second.tn.group_lanes,
                 kv.second.tn.unroll, kv.second.tn.waves_per_block, kv.second.oversub,
                 kv.second.step_cost);
  const bool ok = std::fflush(f) == 0;
  std::fclose(f);
  if (!ok) return fail(TSQBX_E_INVALID, "tuning_save: writing %s failed", path);
  return TSQBX_OK;
}

int tsqbx_tuning_load(tsqbx_ctx *ctx, const char *path, int *n_loaded) {
  if (!ctx || !path) return fail(TSQBX_E_INVALID, "ctx or path is NULL");
  if (n_loaded) *n_loaded = 0;
  std::string arch;
  int rt = 0;
  int rc = tuning_tag(ctx, &arch, &rt);
  if (rc != TSQBX_OK) return rc;
  FILE *f = std::fopen(path, "r");
  if (!f) return fail(TSQBX_E_INVALID, "tuning_load: cannot open %s", path);
  std::map<uint64_t, Tuning> plain;
  std::map<uint64_t, PlanTuning> plans;
  char line[512];
  int lineno = 0;
  while (std::fgets(line, sizeof line, f)) {
    ++lineno;
    if (line[0] == '\n' || line[0] == 0) continue;
    char kind[16] = {0}, a[128] = {0};
    int r = 0, n = 0;
    unsigned long long key = 0;
    if (std::sscanf(line, "{\"kind\": \"%15[a-z]\", \"arch\": \"%127[^\"]\", \"runtime\": %d, "
                          "\"key\": %llu, %n",
                    kind, a, &r, &key, &n) != 4 || n <= 0) {
      std::fclose(f);
      return fail(TSQBX_E_INVALID, "tuning_load: %s line %d is not a tuning entry", path, lineno);
    }
    const char *rest = line + n;
    bool ok = false;
    if (!std::strcmp(kind, "plain")) {
      Tuning t;
      ok = std::sscanf(rest,
                       "\"group_lanes\": %d, \"unroll\": %d, \"waves_per_block\": %d, "
                       "\"xcd_remap\": %d}",
                       &t.group_lanes, &t.unroll, &t.waves_per_block, &t.xcd_remap) == 4 &&
           ((key >> 8 & TSQBX_HELMHOLTZ) ? tuning_supported(t) : eval_tuning_supported(t));
      if (ok && arch == a && rt == r) plain[key] = t;
    } else if (!std::strcmp(kind, "plan")) {
      PlanTuning t;
      ok = std::sscanf(rest,
                       "\"group_lanes\": %d, \"unroll\": %d, \"waves_per_block\": %d, "
                       "\"oversubscription\": %d, \"step_cost\": %d}",
                       &t.tn.group_lanes, &t.tn.unroll, &t.tn.waves_per_block, &t.oversub,
                       &t.step_cost) == 5 &&
           tuning_supported(t.tn) && t.tn.unroll <= 2 && t.oversub >= 1 && t.oversub <= 32 &&
           t.step_cost >= 0 && t.step_cost <= 100000;
      if (ok && arch == a && rt == r) plans[key] = t;
    }
    if (!ok) {
      std::fclose(f);
      return fail(TSQBX_E_INVALID, "tuning_load: %s line %d is not a valid %s entry", path,
                  lineno, kind);
    }
  }
  std::fclose(f);
  {
    std::lock_guard<std::mutex> lk(ctx->tuning_mu);
    for (auto &kv : plain) ctx->tuning[kv.first] = kv.second;
    for (auto &kv : plans) ctx->plan_tuning[kv.first] = kv.second;
  }
  if (n_loaded) *n_loaded = (int)(plain.size() + plans.size());
  return TSQBX_OK;
}

int tsqbx_autotune(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, unsigned layers,
                   tsqbx_tuning *out, double *best_ms) {
  TraceRange trace_("tsqbx_autotune");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  int rc = check_request(g, p, layers);
  if (rc != TSQBX_OK) return rc;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  const size_t N = std::max<int64_t>(g->n_sources, 1), T = std::max<int64_t>(g->n_targets, 1);
  double *sig = nullptr, *o = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  std::vector<double> ones(N, 1.0);
  auto cleanup = [&] {
    if (sig) (void)hipFree(sig);
    if (o) (void)hipFree(o);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  };
  hipError_t e = hipMalloc((void **)&sig, N * sizeof(double));
  if (e == hipSuccess) e = hipMalloc((void **)&o, 3 * T * sizeof(double));
  if (e == hipSuccess) e = hipMemcpy(sig, ones.data(), N * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  hipStream_t s = ctx->stream;
  if (e == hipSuccess) e = launch_stage(g, sig, layers, g->stage, true, s);
  // the staging buffer now holds a density of ones: a later
  // tsqbx_eval_staged_async must stage again
  g->staged_layers.store(0);
  if (e != hipSuccess) {
    cleanup();
    return fail_hip(e, "autotune setup");
  }
  Outputs outs;
  outs.s = o;
  outs.d = o + T;
  outs.t = o + 2 * T;
  Tuning best;
  double best_t = 1e300;
  const int GU[][2] = {{64, 1}, {64, 2}, {64, 4}, {32, 2}, {16, 2}};
  const int W[] = {1, 2, 4, 8};
  for (auto &gu : GU)
    for (int w : W)
      for (int remap = 0; remap <= 1; ++remap) {
        Tuning t;
        t.group_lanes = gu[0];
        t.unroll = gu[1];
        t.waves_per_block = w;
        t.xcd_remap = remap;
        e = launch_eval_plain(g, p, layers, g->stage, outs, false, t, false, s);  // warm-up
        float best_rep = 1e30f;
        for (int rep = 0; rep < 3 && e == hipSuccess; ++rep) {
          e = hipEventRecord(e0, s);
          if (e == hipSuccess) e = launch_eval_plain(g, p, layers, g->stage, outs, false, t, false, s);
          if (e == hipSuccess) e = hipEventRecord(e1, s);
          if (e == hipSuccess) e = hipEventSynchronize(e1);
          float ms = 0;
          if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
          best_rep = std::min(best_rep, ms);
        }
        if (e != hipSuccess) {
          cleanup();
          return fail_hip(e, "autotune launch");
        }
        if (best_rep < best_t) {
          best_t = best_rep;
          best = t;
        }
      }
  cleanup();
  {
    std::lock_guard<std::mutex> lk(ctx->tuning_mu);
    ctx->tuning[tuning_key(p, layers, mean_list_of(g))] = best;
  }
  if (out) {
    out->waves_per_block = best.waves_per_block;
    out->group_lanes = best.group_lanes;
    out->unroll = best.unroll;
    out->xcd_remap = best.xcd_remap;
  }
  if (best_ms) *best_ms = best_t;
  return TSQBX_OK;
}

// ---- Helmholtz -------------------------------------------------------------

static int check_helmholtz(const tsqbx_geometry *g, int p, unsigned layers, double k) {
  if (p < 0 || p > TSQBX_P_MAX)
    return fail(TSQBX_E_RANGE, "expansion order p = %d is outside [0, %d]", p, TSQBX_P_MAX);
  if (layers == 0 || (layers & ~7u))
    return fail(TSQBX_E_INVALID, "Helmholtz layers = %u is not a nonempty subset of SLP|DLP|SPRIME",
                layers);
  if (!(k > 0.0) || !std::isfinite(k))
    return fail(TSQBX_E_RANGE, "the wavenumber k = %g must be positive and finite", k);
  if (g && (layers & TSQBX_DLP) && !g->has_normals)
    return fail(TSQBX_E_INVALID, "double layer requested but the geometry has no normals");
  if (g && (layers & TSQBX_SPRIME) && !g->has_target_normals)
    return fail(TSQBX_E_INVALID, "S' requested but the geometry has no target normals");
  return TSQBX_OK;
}

}  // extern "C"

namespace tsqbx {
int check_helmholtz_request(const tsqbx_geometry *g, int p, unsigned layers, double k) {
  return check_helmholtz(g, p, layers, k);
}
}  // namespace tsqbx

extern "C" {

// The geometry's Helmholtz staging, allocated on its first Helmholtz call,
// and its S' table on the first call that asks for S' (calls on one geometry
// do not overlap, so no lock is needed).
static hipError_t ensure_helm_stage(const tsqbx_geometry *cg, unsigned layers) {
  auto *g = const_cast<tsqbx_geometry *>(cg);
  if ((layers & TSQBX_SPRIME) && !g->helm.tabs) {
    size_t bytes = 0;
    hipError_t e = dev_upload<double>(&g->helm.tabs, nullptr,
                                      std::max<size_t>(1, (size_t)g->n_targets) *
                                          2 * (TSQBX_P_MAX + 1),
                                      &bytes);
    if (e != hipSuccess) {
      g->helm.tabs = nullptr;
      return e;
    }
    g->device_bytes += bytes;
  }
  if (g->helm.rec) return hipSuccess;
  size_t bytes = 0;
  hipError_t e = dev_upload<double4>(&g->helm.rec, nullptr, 2 * ((size_t)g->n_sources + 1), &bytes);
  if (e == hipSuccess)
    e = dev_upload<double>(&g->helm.tab, nullptr,
                           std::max<size_t>(1, (size_t)g->n_targets) * (TSQBX_P_MAX + 1), &bytes);
  if (e != hipSuccess) {
    if (g->helm.rec) (void)hipFree(g->helm.rec);
    if (g->helm.tab) (void)hipFree(g->helm.tab);
    g->helm.rec = nullptr;
    g->helm.tab = nullptr;
    return e;
  }
  g->device_bytes += bytes;
  return hipSuccess;
}

int tsqbx_eval_helmholtz_async(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, unsigned layers,
                               double k, const double *d_sigma, double *d_out_slp,
                               double *d_out_dlp, double *d_out_sprime, unsigned flags,
                               void *hip_stream) {
  TraceRange trace_("tsqbx_eval_helmholtz_async");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = check_helmholtz(g, p, layers, k);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !d_sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  rc = check_outputs(g, layers, d_out_slp, d_out_dlp, d_out_sprime);
  if (rc != TSQBX_OK) return rc;
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  TSQBX_HIP(ensure_helm_stage(g, layers));
  const Tuning tn = lookup_tuning(ctx, p, layers | TSQBX_HELMHOLTZ, mean_list_of(g));
  Outputs out;
  out.s = d_out_slp;
  out.d = d_out_dlp;
  out.t = d_out_sprime;
  TSQBX_HIP(launch_helmholtz(g, p, layers, k, d_sigma, g->helm, out,
                             (flags & TSQBX_ACCUMULATE) != 0, tn, (hipStream_t)hip_stream));
  return TSQBX_OK;
}

int tsqbx_eval_helmholtz(tsqbx_ctx *ctx, const tsqbx_geometry *g, int p, unsigned layers,
                         double k, const double *sigma, double *out_slp, double *out_dlp,
                         double *out_sprime, unsigned flags) {
  TraceRange trace_("tsqbx_eval_helmholtz");
  if (!ctx || !g) return fail(TSQBX_E_INVALID, "ctx or geometry is NULL");
  if (g->ctx != ctx) return fail(TSQBX_E_INVALID, "geometry belongs to another context");
  int rc = check_helmholtz(g, p, layers, k);
  if (rc != TSQBX_OK) return rc;
  if (g->n_sources > 0 && !sigma) return fail(TSQBX_E_INVALID, "sigma is NULL");
  rc = check_outputs(g, layers, out_slp, out_dlp, out_sprime);
  if (rc != TSQBX_OK) return rc;
  std::lock_guard<std::mutex> lk(ctx->mu);
  DeviceGuard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  TSQBX_HIP(ensure_helm_stage(g, layers));
  const size_t N = (size_t)g->n_sources, T = (size_t)g->n_targets;
  if (ctx->d_sigma_cap < 2 * N) {
    if (ctx->d_sigma) (void)hipFree(ctx->d_sigma);
    ctx->d_sigma = nullptr;
    ctx->d_sigma_cap = 0;
    TSQBX_HIP(hipMalloc((void **)&ctx->d_sigma, 2 * N * sizeof(double)));
    ctx->d_sigma_cap = 2 * N;
  }
  if (ctx->d_out_cap < 6 * T) {
    if (ctx->d_out) (void)hipFree(ctx->d_out);
    ctx->d_out = nullptr;
    ctx->d_out_cap = 0;
    TSQBX_HIP(hipMalloc((void **)&ctx->d_out, 6 * T * sizeof(double)));
    ctx->d_out_cap = 6 * T;
  }
  hipStream_t s = ctx->stream;
  if (N)
    TSQBX_HIP(hipMemcpyAsync(ctx->d_sigma, sigma, 2 * N * sizeof(double), hipMemcpyHostToDevice, s));
  double *const dev[3] = {ctx->d_out, ctx->d_out + 2 * T, ctx->d_out + 4 * T};
  const Tuning tn = lookup_tuning(ctx, p, layers | TSQBX_HELMHOLTZ, mean_list_of(g));
  Outputs out;
  out.s = dev[0];
  out.d = dev[1];
  out.t = dev[2];
  TSQBX_HIP(launch_helmholtz(g, p, layers, k, ctx->d_sigma, g->helm, out, false, tn, s));
  const bool acc = (flags & TSQBX_ACCUMULATE) != 0;
  double *const user[3] = {out_slp, out_dlp, out_sprime};
  std::vector<double> tmp[3];
  for (int l = 0; l < 3; ++l) {
    if (!T || !(layers & (1u << l))) continue;
    double *dst = user[l];
    if (acc) {
      tmp[l].resize(2 * T);
      dst = tmp[l].data();
    }
    TSQBX_HIP(hipMemcpyAsync(dst, dev[l], 2 * T * sizeof(double), hipMemcpyDeviceToHost, s));
  }
  TSQBX_HIP(hipStreamSynchronize(s));
  for (int l = 0; l < 3; ++l)
    for (size_t i = 0; i < tmp[l].size(); ++i) user[l][i] += tmp[l][i];
  return TSQBX_OK;
}

}  // extern "C"
