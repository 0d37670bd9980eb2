// Geometry creation from arrays in device memory: the device layout that
// tsqbx_geometry_create builds on the host (Morton orders of sources and of
// targets by their center, one padded, remapped and sorted row per distinct
// center), built on the device, so that near-field lists made on the device
// (the step before the evaluation, the near-field sets of the tree) reach a
// geometry without a round trip through host memory.  Every step is integer
// work or an exact copy, and the Morton keys are formed with the host's
// arithmetic, so the result equals the host-built geometry bit for bit.
#include <algorithm>
#include <cstring>
#include <type_traits>
#include <vector>

#include <rocprim/rocprim.hpp>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

constexpr int kBlock = 256;

// ---- validation --------------------------------------------------------------
// Error bits: offsets that do not start at 0 or decrease (1), a list longer
// than the layout allows (2), a source index out of range (4), a target's
// center out of range (8).
__global__ void __launch_bounds__(kBlock)
k_validate(const int64_t *__restrict__ off, int64_t M, const int32_t *__restrict__ list,
           int64_t nnz, int64_t N, const int32_t *__restrict__ tc, int64_t T,
           unsigned *__restrict__ err) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned e = 0;
  if (g == 0 && off[0] != 0) e |= 1u;
  for (int64_t i = g; i < M; i += stride) {
    const int64_t len = off[i + 1] - off[i];
    if (len < 0) e |= 1u;
    if (len > (int64_t(1) << 30) - kRowPad) e |= 2u;
  }
  for (int64_t j = g; j < nnz; j += stride) {
    const int32_t s = list[j];
    if (s < 0 || (int64_t)s >= N) e |= 4u;
  }
  if (tc)
    for (int64_t t = g; t < T; t += stride) {
      const int32_t c = tc[t];
      if (c < 0 || (int64_t)c >= M) e |= 8u;
    }
  if (e) atomicOr(err, e);
}

// ---- Morton keys ---------------------------------------------------------------
// Per-block minima and maxima of the points' coordinates, then one block
// folds them: out = (lo[3], scale) with scale = (2^21 - 1) / span as the host
// computes it (min and max are exact, so the order of the folding does not
// matter).
__global__ void __launch_bounds__(kBlock)
k_bbox_partial(const double *__restrict__ xyz, int64_t n, double *__restrict__ part) {
  __shared__ double sh[6][kBlock];
  const double big = __builtin_inf();
  double lo[3] = {big, big, big}, hi[3] = {-big, -big, -big};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    for (int a = 0; a < 3; ++a) {
      const double v = xyz[3 * i + a];
      lo[a] = v < lo[a] ? v : lo[a];
      hi[a] = v > hi[a] ? v : hi[a];
    }
  for (int a = 0; a < 3; ++a) {
    sh[a][threadIdx.x] = lo[a];
    sh[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        const double l = sh[a][threadIdx.x + w], h = sh[3 + a][threadIdx.x + w];
        sh[a][threadIdx.x] = l < sh[a][threadIdx.x] ? l : sh[a][threadIdx.x];
        sh[3 + a][threadIdx.x] = h > sh[3 + a][threadIdx.x] ? h : sh[3 + a][threadIdx.x];
      }
    __syncthreads();
  }
  if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void __launch_bounds__(kBlock) k_bbox_final(const double *__restrict__ part, int nb,
                                                       double *__restrict__ box) {
  __shared__ double sh[6][kBlock];
  const double big = __builtin_inf();
  double lo[3] = {big, big, big}, hi[3] = {-big, -big, -big};
  for (int b = threadIdx.x; b < nb; b += blockDim.x)
    for (int a = 0; a < 3; ++a) {
      lo[a] = part[6 * b + a] < lo[a] ? part[6 * b + a] : lo[a];
      hi[a] = part[6 * b + 3 + a] > hi[a] ? part[6 * b + 3 + a] : hi[a];
    }
  for (int a = 0; a < 3; ++a) {
    sh[a][threadIdx.x] = lo[a];
    sh[3 + a][threadIdx.x] = hi[a];
  }
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int a = 0; a < 3; ++a) {
        const double l = sh[a][threadIdx.x + w], h = sh[3 + a][threadIdx.x + w];
        sh[a][threadIdx.x] = l < sh[a][threadIdx.x] ? l : sh[a][threadIdx.x];
        sh[3 + a][threadIdx.x] = h > sh[3 + a][threadIdx.x] ? h : sh[3 + a][threadIdx.x];
      }
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  for (int a = 0; a < 3; ++a) {
    lo[a] = sh[a][0];
    hi[a] = sh[3 + a][0];
  }
  double span = 1e-300;
  for (int a = 0; a < 3; ++a) span = hi[a] - lo[a] > span ? hi[a] - lo[a] : span;
  for (int a = 0; a < 3; ++a) box[a] = lo[a];
  box[3] = double((1 << 21) - 1) / span;
}

__device__ __forceinline__ uint64_t spread21_dev(uint64_t v) {
  v &= 0x1fffffULL;
  v = (v | v << 32) & 0x1f00000000ffffULL;
  v = (v | v << 16) & 0x1f0000ff0000ffULL;
  v = (v | v << 8) & 0x100f00f00f00f00fULL;
  v = (v | v << 4) & 0x10c30c30c30c30c3ULL;
  v = (v | v << 2) & 0x1249249249249249ULL;
  return v;
}

// key[i]: the point's 63-bit Morton key (x in the highest bit of each
// triple); val[i] = i.
__global__ void __launch_bounds__(kBlock)
k_morton(const double *__restrict__ xyz, int64_t n, const double *__restrict__ box,
         uint64_t *__restrict__ key, int32_t *__restrict__ val) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double scale = box[3];
  const double top = double((1 << 21) - 1);
  uint64_t q[3];
  for (int a = 0; a < 3; ++a) {
    double v = (xyz[3 * i + a] - box[a]) * scale;  // two roundings, as on the host
    v = v > 0.0 ? v : 0.0;
    v = v < top ? v : top;
    q[a] = (uint64_t)v;
  }
  key[i] = spread21_dev(q[0]) << 2 | spread21_dev(q[1]) << 1 | spread21_dev(q[2]);
  if (val) val[i] = (int32_t)i;
}

// ---- sources in device order ------------------------------------------------
__global__ void __launch_bounds__(kBlock)
k_sources(const int32_t *__restrict__ ord, int64_t n, const double *__restrict__ xyz,
          const double *__restrict__ w, const double *__restrict__ nrm, double4 *__restrict__ pos,
          double *__restrict__ w_out, double4 *__restrict__ nrm_out, int64_t *__restrict__ perm,
          int32_t *__restrict__ rank) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const int64_t s = ord[k];
  pos[k] = make_double4(xyz[3 * s], xyz[3 * s + 1], xyz[3 * s + 2], w[s]);
  w_out[k] = w[s];
  if (nrm) nrm_out[k] = make_double4(nrm[3 * s], nrm[3 * s + 1], nrm[3 * s + 2], 0.0);
  perm[k] = s;
  rank[s] = (int32_t)k;
}

// ---- targets and rows ----------------------------------------------------------
// tc_of[t]: target t's center (the identity when no map is given).
__global__ void __launch_bounds__(kBlock)
k_target_centers(const int32_t *__restrict__ tc, int64_t T, uint32_t *__restrict__ key,
                 int32_t *__restrict__ val) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= T) return;
  key[t] = (uint32_t)(tc ? tc[t] : (int32_t)t);
  val[t] = (int32_t)t;
}

// The Morton key of each (sorted) target's center.
__global__ void __launch_bounds__(kBlock)
k_gather_center_keys(const int32_t *__restrict__ ord, int64_t T, const int32_t *__restrict__ tc,
                     const uint64_t *__restrict__ ckey, uint64_t *__restrict__ key) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  const int64_t t = ord[k];
  key[k] = ckey[tc ? tc[t] : t];
}

// flag[k] = 1 where a new center's run of targets starts.
__global__ void __launch_bounds__(kBlock)
k_row_flags(const int32_t *__restrict__ ord, int64_t T, const int32_t *__restrict__ tc,
            int32_t *__restrict__ flag) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  const int64_t c = tc ? tc[ord[k]] : ord[k];
  const int64_t cp = k == 0 ? -1 : (tc ? tc[ord[k - 1]] : ord[k - 1]);
  flag[k] = c != cp ? 1 : 0;
}

// At each run start: the row's center, first target and padded length.
__global__ void __launch_bounds__(kBlock)
k_row_setup(const int32_t *__restrict__ ord, int64_t T, const int32_t *__restrict__ tc,
            const int32_t *__restrict__ flag, const int32_t *__restrict__ row_id,
            const int64_t *__restrict__ off, int64_t *__restrict__ row_center,
            int64_t *__restrict__ row_first, int64_t *__restrict__ padlen) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T || !flag[k]) return;
  const int64_t r = row_id[k] - 1;
  const int64_t c = tc ? tc[ord[k]] : ord[k];
  row_center[r] = c;
  row_first[r] = k;
  const int64_t len = off[c + 1] - off[c];
  padlen[r] = (len + kRowPad - 1) / kRowPad * kRowPad;
}

// Row r's entries in device numbering, then padding entries N (a block per
// row at a time; the rows are sorted afterwards, and N sorts last).
__global__ void __launch_bounds__(kBlock)
k_fill_rows(int64_t R, const int64_t *__restrict__ row_center, const int64_t *__restrict__ row_off,
            const int64_t *__restrict__ off, const int32_t *__restrict__ list,
            const int32_t *__restrict__ rank, int32_t N, int32_t *__restrict__ buf) {
  for (int64_t r = blockIdx.x; r < R; r += gridDim.x) {
    const int64_t c = row_center[r];
    const int64_t b = off[c], len = off[c + 1] - b;
    const int64_t o = row_off[r], plen = row_off[r + 1] - o;
    for (int64_t j = threadIdx.x; j < plen; j += blockDim.x)
      buf[o + j] = j < len ? rank[list[b + j]] : N;
  }
}

// TargetRec, target normal and list length of each device-order target.
__global__ void __launch_bounds__(kBlock)
k_targets(const int32_t *__restrict__ ord, int64_t T, const int32_t *__restrict__ tc,
          const int32_t *__restrict__ row_id, const int64_t *__restrict__ row_off,
          const int64_t *__restrict__ off, const double *__restrict__ centers,
          const double *__restrict__ targets, const double *__restrict__ tnrm,
          TargetRec *__restrict__ rec, double4 *__restrict__ tnrm_out,
          int64_t *__restrict__ row_len) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= T) return;
  const int64_t t = ord[k];
  const int64_t c = tc ? tc[t] : t;
  const int64_t r = row_id[k] - 1;
  TargetRec x;
  for (int a = 0; a < 3; ++a) {
    x.c[a] = centers[3 * c + a];
    x.d[a] = targets[3 * t + a] - centers[3 * c + a];
  }
  x.row_begin = row_off[r];
  x.row_len = (int32_t)(row_off[r + 1] - row_off[r]);
  x.out_index = (int32_t)t;
  rec[k] = x;
  if (tnrm) tnrm_out[k] = make_double4(tnrm[3 * t], tnrm[3 * t + 1], tnrm[3 * t + 2], 0.0);
  row_len[k] = off[c + 1] - off[c];
}

// CenterRec of each row; the row's targets are the run row_first[r] .. , so
// row_tgts is the identity.
__global__ void __launch_bounds__(kBlock)
k_centers(int64_t R, int64_t T, const int64_t *__restrict__ row_center,
          const int64_t *__restrict__ row_first, const int64_t *__restrict__ row_off,
          const int64_t *__restrict__ off, const double *__restrict__ centers,
          CenterRec *__restrict__ crec, int32_t *__restrict__ row_tgts,
          unsigned *__restrict__ max_count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r < T) row_tgts[r] = (int32_t)r;
  if (r >= R) return;
  const int64_t c = row_center[r];
  CenterRec x;
  for (int a = 0; a < 3; ++a) x.c[a] = centers[3 * c + a];
  x.row_begin = row_off[r];
  x.len = (int32_t)(off[c + 1] - off[c]);
  x.center = (int32_t)c;
  x.tgt_begin = (int32_t)row_first[r];
  x.tgt_count = (int32_t)((r + 1 < R ? row_first[r + 1] : T) - row_first[r]);
  x.pad = 0;
  crec[r] = x;
  atomicMax(max_count, (unsigned)x.tgt_count);
}

unsigned grid_of(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kBlock - 1) / kBlock); }

int bits_for(int64_t v) {  // bits that hold 0..v
  int b = 1;
  while (b < 63 && (int64_t(1) << b) <= v) ++b;
  return b;
}

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

// Device buffers of one build, freed when it ends.
struct Scratch {
  std::vector<void *> ptrs;
  ~Scratch() {
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  hipError_t get(T **p, size_t n) {
    *p = nullptr;
    hipError_t e = hipMalloc((void **)p, std::max<size_t>(n, 1) * sizeof(T));
    if (e == hipSuccess) ptrs.push_back(*p);
    return e;
  }
};

}  // namespace
}  // namespace tsqbx

using namespace tsqbx;

int tsqbx::build_geometry_device(tsqbx_ctx *ctx, const tsqbx_geometry_desc *d, hipStream_t s,
                                 tsqbx_geometry **out) {
  *out = nullptr;
  const int64_t N = d->n_sources, M = d->n_centers, T = d->n_targets;
  if (N < 0 || M < 0 || T < 0) return fail(TSQBX_E_INVALID, "negative count");
  if (N >= TSQBX_MAX_SOURCES)
    return fail(TSQBX_E_RANGE, "n_sources = %lld; a geometry holds fewer than %lld sources",
                (long long)N, (long long)TSQBX_MAX_SOURCES);
  if (T > INT32_MAX || M > INT32_MAX) return fail(TSQBX_E_RANGE, "counts must stay below 2^31");
  if ((N > 0 && (!d->sources || !d->weights)) || (M > 0 && !d->centers) || !d->list_offsets ||
      (T > 0 && !d->targets))
    return fail(TSQBX_E_INVALID, "a required array is NULL");
  if (!d->target_center && T > 0 && T != M)
    return fail(TSQBX_E_INVALID, "target_center is NULL but n_targets (%lld) != n_centers (%lld)",
                (long long)T, (long long)M);
  Guard dg(ctx->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  Scratch sc;
  hipError_t e = hipSuccess;
#define TQ(call)                                  \
  do {                                            \
    e = (call);                                   \
    if (e != hipSuccess) return fail_hip(e, #call); \
  } while (0)

  // the list count and the checks the host path makes
  int64_t nnz = 0;
  TQ(hipMemcpyAsync(&nnz, d->list_offsets + M, sizeof nnz, hipMemcpyDeviceToHost, s));
  TQ(hipStreamSynchronize(s));
  if (nnz > 0 && !d->list_sources) return fail(TSQBX_E_INVALID, "list_sources is NULL");
  unsigned *d_err = nullptr;
  TQ(sc.get(&d_err, 1));
  TQ(hipMemsetAsync(d_err, 0, sizeof(unsigned), s));
  hipLaunchKernelGGL(k_validate, dim3((unsigned)std::min<int64_t>(grid_of(std::max({M, nnz, T})), 4096)),
                     dim3(kBlock), 0, s, d->list_offsets, M, d->list_sources, nnz, N,
                     d->target_center, T, d_err);
  TQ(hipGetLastError());
  unsigned herr = 0;
  TQ(hipMemcpyAsync(&herr, d_err, sizeof herr, hipMemcpyDeviceToHost, s));
  TQ(hipStreamSynchronize(s));
  if (herr & 1u) return fail(TSQBX_E_INVALID, "list_offsets does not start at 0 or decreases");
  if (herr & 2u)
    return fail(TSQBX_E_RANGE, "a list is longer than 2^30 - %d entries", kRowPad);
  if (herr & 4u) return fail(TSQBX_E_RANGE, "a list_sources entry is outside [0, %lld)", (long long)N);
  if (herr & 8u) return fail(TSQBX_E_RANGE, "a target_center entry is outside [0, %lld)", (long long)M);

  auto *g = new tsqbx_geometry;
  g->ctx = ctx;
  g->device = ctx->device;
  g->n_sources = N;
  g->n_centers = M;
  g->n_targets = T;
  g->has_normals = d->normals != nullptr;
  g->has_target_normals = d->target_normals != nullptr;
  struct Own {  // frees the geometry unless the build succeeds
    tsqbx_geometry *g;
    ~Own() { free_geometry(g); }
  } own{g};
  size_t bytes = 0;
  auto keep = [&](auto **p, size_t n) -> hipError_t {
    using T = std::remove_reference_t<decltype(**p)>;
    *p = nullptr;
    if (n == 0) return hipSuccess;
    bytes += n * sizeof(T);
    return hipMalloc((void **)p, n * sizeof(T));
  };
  size_t tmp_bytes = 0, need = 0;
  void *tmp = nullptr;
  auto tmp_for = [&](size_t n) -> hipError_t {  // grow the rocPRIM temporary storage
    if (n <= tmp_bytes) return hipSuccess;
    void *p = nullptr;
    hipError_t er = sc.get((char **)&p, n);
    if (er == hipSuccess) {
      tmp = p;
      tmp_bytes = n;
    }
    return er;
  };

  // sources: Morton keys in their bounding box, a stable sort, the inverse
  const int nbb = (int)std::min<int64_t>(grid_of(std::max(N, M)), 1024);
  double *part = nullptr, *box = nullptr;
  TQ(sc.get(&part, 6 * (size_t)nbb));
  TQ(sc.get(&box, 8));
  int32_t *src_ord = nullptr;
  if (N > 0) {
    uint64_t *k0 = nullptr, *k1 = nullptr;
    int32_t *v0 = nullptr;
    TQ(sc.get(&k0, N));
    TQ(sc.get(&k1, N));
    TQ(sc.get(&v0, N));
    TQ(sc.get(&src_ord, N));
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(kBlock), 0, s, d->sources, N, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBlock), 0, s, part, nbb, box);
    hipLaunchKernelGGL(k_morton, dim3(grid_of(N)), dim3(kBlock), 0, s, d->sources, N, box, k0, v0);
    TQ(hipGetLastError());
    TQ(rocprim::radix_sort_pairs(nullptr, need, k0, k1, v0, src_ord, (size_t)N, 0, 63, s));
    TQ(tmp_for(need));
    TQ(rocprim::radix_sort_pairs(tmp, need, k0, k1, v0, src_ord, (size_t)N, 0, 63, s));
    TQ(keep(&g->src_pos, N));
    TQ(keep(&g->src_w, N));
    if (d->normals) TQ(keep(&g->src_nrm, N));
    TQ(keep(&g->src_perm, N));
    TQ(keep(&g->src_rank, N));
    hipLaunchKernelGGL(k_sources, dim3(grid_of(N)), dim3(kBlock), 0, s, src_ord, N, d->sources,
                       d->weights, d->normals, g->src_pos, g->src_w, g->src_nrm, g->src_perm,
                       g->src_rank);
    TQ(hipGetLastError());
  }

  // targets: by the Morton key of their center, then center, then index
  // (two stable sorts: by center, then by the center's key)
  int32_t *tgt_ord = nullptr, *row_id = nullptr, *flag = nullptr;
  int64_t R = 0;
  if (T > 0) {
    uint64_t *ckey = nullptr, *k0 = nullptr, *k1 = nullptr;
    uint32_t *c0 = nullptr, *c1 = nullptr;
    int32_t *v0 = nullptr, *v1 = nullptr;
    TQ(sc.get(&ckey, M));
    TQ(sc.get(&k0, T));
    TQ(sc.get(&k1, T));
    TQ(sc.get(&c0, T));
    TQ(sc.get(&c1, T));
    TQ(sc.get(&v0, T));
    TQ(sc.get(&v1, T));
    TQ(sc.get(&tgt_ord, T));
    TQ(sc.get(&flag, T));
    TQ(sc.get(&row_id, T));
    hipLaunchKernelGGL(k_bbox_partial, dim3(nbb), dim3(kBlock), 0, s, d->centers, M, part);
    hipLaunchKernelGGL(k_bbox_final, dim3(1), dim3(kBlock), 0, s, part, nbb, box);
    hipLaunchKernelGGL(k_morton, dim3(grid_of(M)), dim3(kBlock), 0, s, d->centers, M, box, ckey,
                       (int32_t *)nullptr);
    hipLaunchKernelGGL(k_target_centers, dim3(grid_of(T)), dim3(kBlock), 0, s, d->target_center, T,
                       c0, v0);
    TQ(hipGetLastError());
    const int cb = bits_for(M);
    TQ(rocprim::radix_sort_pairs(nullptr, need, c0, c1, v0, v1, (size_t)T, 0, cb, s));
    TQ(tmp_for(need));
    TQ(rocprim::radix_sort_pairs(tmp, need, c0, c1, v0, v1, (size_t)T, 0, cb, s));
    hipLaunchKernelGGL(k_gather_center_keys, dim3(grid_of(T)), dim3(kBlock), 0, s, v1, T,
                       d->target_center, ckey, k0);
    TQ(hipGetLastError());
    TQ(rocprim::radix_sort_pairs(nullptr, need, k0, k1, v1, tgt_ord, (size_t)T, 0, 63, s));
    TQ(tmp_for(need));
    TQ(rocprim::radix_sort_pairs(tmp, need, k0, k1, v1, tgt_ord, (size_t)T, 0, 63, s));
    // rows: one per run of targets sharing a center
    hipLaunchKernelGGL(k_row_flags, dim3(grid_of(T)), dim3(kBlock), 0, s, tgt_ord, T,
                       d->target_center, flag);
    TQ(hipGetLastError());
    TQ(rocprim::inclusive_scan(nullptr, need, flag, row_id, (size_t)T, rocprim::plus<int32_t>(), s));
    TQ(tmp_for(need));
    TQ(rocprim::inclusive_scan(tmp, need, flag, row_id, (size_t)T, rocprim::plus<int32_t>(), s));
    int32_t r32 = 0;
    TQ(hipMemcpyAsync(&r32, row_id + (T - 1), sizeof r32, hipMemcpyDeviceToHost, s));
    TQ(hipStreamSynchronize(s));
    R = r32;
  }

  // row offsets (padded lengths, scanned), then the rows
  int64_t *row_center = nullptr, *row_first = nullptr, *padlen = nullptr, *row_off = nullptr;
  TQ(sc.get(&row_center, R));
  TQ(sc.get(&row_first, R));
  TQ(sc.get(&padlen, R));
  TQ(sc.get(&row_off, R + 1));
  TQ(hipMemsetAsync(row_off, 0, sizeof(int64_t), s));
  int64_t nnz_dev = 0, longest = 0;
  if (R > 0) {
    int64_t *d_longest = nullptr;
    TQ(sc.get(&d_longest, 1));
    hipLaunchKernelGGL(k_row_setup, dim3(grid_of(T)), dim3(kBlock), 0, s, tgt_ord, T,
                       d->target_center, flag, row_id, d->list_offsets,
                       row_center, row_first, padlen);
    TQ(hipGetLastError());
    TQ(rocprim::inclusive_scan(nullptr, need, padlen, row_off + 1, (size_t)R,
                               rocprim::plus<int64_t>(), s));
    TQ(tmp_for(need));
    TQ(rocprim::inclusive_scan(tmp, need, padlen, row_off + 1, (size_t)R, rocprim::plus<int64_t>(),
                               s));
    TQ(rocprim::reduce(nullptr, need, padlen, d_longest, int64_t(0), (size_t)R,
                       rocprim::maximum<int64_t>(), s));
    TQ(tmp_for(need));
    TQ(rocprim::reduce(tmp, need, padlen, d_longest, int64_t(0), (size_t)R,
                       rocprim::maximum<int64_t>(), s));
    TQ(hipMemcpyAsync(&nnz_dev, row_off + R, sizeof nnz_dev, hipMemcpyDeviceToHost, s));
    TQ(hipMemcpyAsync(&longest, d_longest, sizeof longest, hipMemcpyDeviceToHost, s));
    TQ(hipStreamSynchronize(s));
  }
  g->nnz = nnz_dev;
  g->n_rows = R;
  TQ(keep(&g->idx, nnz_dev));
  if (nnz_dev > 0) {
    int32_t *buf = nullptr;
    if (!(longest <= kRowSortMax && R <= INT32_MAX)) TQ(sc.get(&buf, nnz_dev));
    if (longest <= kRowSortMax && R <= INT32_MAX) {
      // rows short enough for one workgroup each: filled in place, sorted in LDS
      hipLaunchKernelGGL(k_fill_rows, dim3((unsigned)std::min<int64_t>(R, 1 << 20)),
                         dim3(kBlock), 0, s, R, row_center, row_off, d->list_offsets,
                         d->list_sources, g->src_rank, (int32_t)N, g->idx);
      TQ(hipGetLastError());
      TQ(sort_rows(row_off, g->idx, R, longest, N, s));
    } else {
      hipLaunchKernelGGL(k_fill_rows, dim3((unsigned)std::min<int64_t>(R, 1 << 20)),
                         dim3(kBlock), 0, s, R, row_center, row_off, d->list_offsets,
                         d->list_sources, g->src_rank, (int32_t)N, buf);
      TQ(hipGetLastError());
      // entries lie in [0, N]: sort them as unsigned keys on their low bits
      const int ib = bits_for(N);
      uint32_t *ub = (uint32_t *)buf, *uo = (uint32_t *)g->idx;
      TQ(rocprim::segmented_radix_sort_keys(nullptr, need, ub, uo, (size_t)nnz_dev, (unsigned)R,
                                            row_off, row_off + 1, 0, ib, s));
      TQ(tmp_for(need));
      TQ(rocprim::segmented_radix_sort_keys(tmp, need, ub, uo, (size_t)nnz_dev, (unsigned)R,
                                            row_off, row_off + 1, 0, ib, s));
    }
  }

  // per-target and per-row records
  int64_t *row_len = nullptr;
  TQ(sc.get(&row_len, T));
  TQ(keep(&g->tgt, T));
  if (d->target_normals) TQ(keep(&g->tgt_nrm, T));
  TQ(keep(&g->ctr, R));
  TQ(keep(&g->row_tgts, T));
  unsigned *d_maxc = nullptr, h_maxc = 0;  // most targets in a row
  TQ(sc.get(&d_maxc, 1));
  TQ(hipMemsetAsync(d_maxc, 0, sizeof(unsigned), s));
  if (T > 0) {
    hipLaunchKernelGGL(k_targets, dim3(grid_of(T)), dim3(kBlock), 0, s, tgt_ord, T,
                       d->target_center, row_id, row_off, d->list_offsets, d->centers, d->targets,
                       d->target_normals, g->tgt, g->tgt_nrm, row_len);
    hipLaunchKernelGGL(k_centers, dim3(grid_of(std::max(R, T))), dim3(kBlock), 0, s, R, T,
                       row_center, row_first, row_off, d->list_offsets, d->centers, g->ctr,
                       g->row_tgts, d_maxc);
    TQ(hipGetLastError());
    TQ(hipMemcpyAsync(&h_maxc, d_maxc, sizeof h_maxc, hipMemcpyDeviceToHost, s));
  }
  g->host_row_len.resize(T);
  if (T > 0)
    TQ(hipMemcpyAsync(g->host_row_len.data(), row_len, T * sizeof(int64_t), hipMemcpyDeviceToHost, s));
  // staging arrays of the plain path
  char *spos = nullptr, *snrm = nullptr;
  TQ(keep(&spos, stage_pos_bytes(N)));
  if (d->normals) TQ(keep(&snrm, stage_nrm_bytes(N)));
  g->stage = stage_views(spos, snrm, N);
  // the positions and the padding entry, once: evaluations stage strengths only
  TQ(launch_stage_positions(g, g->stage, s));
  TQ(hipStreamSynchronize(s));  // the scratch buffers are freed on return
  g->max_row_targets = h_maxc;
  for (int64_t v : g->host_row_len) {
    g->pairs += v;
    g->max_list = std::max(g->max_list, v);
  }
  g->device_bytes = bytes;
#undef TQ
  own.g = nullptr;
  *out = g;
  return TSQBX_OK;
}

extern "C" int tsqbx_geometry_create_device(tsqbx_ctx *ctx, const tsqbx_geometry_desc *d,
                                            unsigned flags, void *hip_stream,
                                            tsqbx_geometry **out) {
  TraceRange trace_("tsqbx_geometry_create_device");
  if (!ctx || !out || !d) return fail(TSQBX_E_INVALID, "ctx, desc or out is NULL");
  *out = nullptr;
  if (flags & TSQBX_NO_REORDER)
    return fail(TSQBX_E_INVALID, "geometry_create_device builds the reordered layout only");
  return build_geometry_device(ctx, d, (hipStream_t)hip_stream, out);
}

extern "C" int tsqbx_geometry_read_layout(const tsqbx_geometry *g, int64_t *source_order,
                                          int64_t *target_order, int64_t *target_row,
                                          int64_t *row_offsets, int64_t row_offsets_cap,
                                          int32_t *rows, int64_t rows_cap,
                                          tsqbx_layout_info *info) {
  TraceRange trace_("tsqbx_geometry_read_layout");
  if (!g || !info) return fail(TSQBX_E_INVALID, "geometry or info is NULL");
  const int64_t N = g->n_sources, T = g->n_targets, R = g->n_rows;
  info->n_rows = R;
  info->nnz = g->nnz;
  info->pairs = g->pairs;
  info->max_list = g->max_list;
  if ((row_offsets && row_offsets_cap < R + 1) || (rows && rows_cap < g->nnz))
    return fail(TSQBX_E_RANGE, "geometry_read_layout: %lld rows of %lld entries do not fit the buffers",
                (long long)R, (long long)g->nnz);
  Guard dg(g->device);
  if (dg.err != hipSuccess) return fail_hip(dg.err, "hipSetDevice");
  if (source_order) {
    if (g->src_perm)
      TSQBX_HIP(hipMemcpy(source_order, g->src_perm, N * sizeof(int64_t), hipMemcpyDeviceToHost));
    else
      for (int64_t i = 0; i < N; ++i) source_order[i] = i;
  }
  std::vector<CenterRec> crec(R);
  if (R > 0) TSQBX_HIP(hipMemcpy(crec.data(), g->ctr, R * sizeof(CenterRec), hipMemcpyDeviceToHost));
  if (row_offsets) {
    for (int64_t r = 0; r < R; ++r) row_offsets[r] = crec[r].row_begin;
    row_offsets[R] = g->nnz;
  }
  if (target_order && T > 0) {
    std::vector<TargetRec> rec(T);
    TSQBX_HIP(hipMemcpy(rec.data(), g->tgt, T * sizeof(TargetRec), hipMemcpyDeviceToHost));
    for (int64_t k = 0; k < T; ++k) target_order[k] = rec[k].out_index;
  }
  if (target_row && T > 0) {  // row r holds targets row_tgts[tgt_begin .. + tgt_count)
    std::vector<int32_t> rt(T);
    TSQBX_HIP(hipMemcpy(rt.data(), g->row_tgts, T * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t r = 0; r < R; ++r)
      for (int32_t j = crec[r].tgt_begin; j < crec[r].tgt_begin + crec[r].tgt_count; ++j)
        target_row[rt[j]] = r;
  }
  if (rows && g->nnz > 0)
    TSQBX_HIP(hipMemcpy(rows, g->idx, g->nnz * sizeof(int32_t), hipMemcpyDeviceToHost));
  return TSQBX_OK;
}
