// Near-field list construction on the device: for every QBX center the
// sources inside the closed ball of radius r about it (the near-field source
// set of Sec. 3.3, taken as a ball as in the workloads), as CSR with
// ascending source indices.
//
// Membership is decided in FP64 exactly as written: dx = y_x - c_x (likewise
// y, z), d2 = (dx*dx + dy*dy) + dz*dz with every operation rounded on its own
// (the library is built without FP contraction), member iff d2 <= r*r.
//
// Steps: a bounding box; a uniform grid of cells of size h >= r(1 + 1e-8)
// (so that rounding in the cell coordinates cannot move a member out of the
// 27 cells around its center's cell) hashed into an open-addressing table;
// sources counted per cell, scanned and scattered into cell order; one wave
// per center counts its members in the 27 cells, the counts are scanned into
// the row offsets, a second pass writes the members, and one workgroup per
// row sorts it in LDS.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "tsqbx_internal.h"

namespace tsqbx {
namespace {

constexpr uint64_t kEmpty = ~0ull;
constexpr int kCellBits = 21;
constexpr double kMaxCells = double((1 << kCellBits) - 16);
constexpr int kScanItems = 8;  // elements per thread in a scan block
constexpr int kScanBlock = 256 * kScanItems;

struct GridParams {
  double lo[3];
  double inv_h;
  double r2;
};

__device__ __forceinline__ uint32_t cell_of(double x, double lo, double inv_h) {
  return (uint32_t)floor((x - lo) * inv_h);
}

__device__ __forceinline__ uint64_t cell_key(uint32_t ix, uint32_t iy, uint32_t iz) {
  return ((uint64_t)ix << (2 * kCellBits)) | ((uint64_t)iy << kCellBits) | (uint64_t)iz;
}

__device__ __forceinline__ uint32_t hash_slot(uint64_t key, uint32_t mask) {
  return (uint32_t)((key * 0x9E3779B97F4A7C15ull) >> 32) & mask;
}

// Slot of key in the table, or -1 when the cell holds no source.
__device__ __forceinline__ int64_t find_slot(const uint64_t *__restrict__ keys, uint32_t mask,
                                             uint64_t key) {
  uint32_t s = hash_slot(key, mask);
  for (;;) {
    const uint64_t k = keys[s];
    if (k == key) return s;
    if (k == kEmpty) return -1;
    s = (s + 1) & mask;
  }
}

// ---- bounding box --------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_bbox_partial(const double *__restrict__ src, int64_t n, const double *__restrict__ ctr,
               int64_t m, double *__restrict__ partial) {
  __shared__ double s[6][256];
  double mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n + m;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double *p = i < n ? src + 3 * i : ctr + 3 * (i - n);
    for (int a = 0; a < 3; ++a) {
      mn[a] = fmin(mn[a], p[a]);
      mx[a] = fmax(mx[a], p[a]);
    }
  }
  const int t = threadIdx.x;
  for (int a = 0; a < 3; ++a) {
    s[a][t] = mn[a];
    s[3 + a][t] = mx[a];
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off)
      for (int a = 0; a < 3; ++a) {
        s[a][t] = fmin(s[a][t], s[a][t + off]);
        s[3 + a][t] = fmax(s[3 + a][t], s[3 + a][t + off]);
      }
    __syncthreads();
  }
  if (t < 6) partial[blockIdx.x * 6 + t] = s[t][0];
}

__global__ void __launch_bounds__(256)
k_grid_params(const double *__restrict__ partial, int nb, double r, GridParams *__restrict__ gp) {
  __shared__ double s[6][256];
  const int t = threadIdx.x;
  double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
  for (int b = t; b < nb; b += blockDim.x)
    for (int a = 0; a < 3; ++a) {
      v[a] = fmin(v[a], partial[b * 6 + a]);
      v[3 + a] = fmax(v[3 + a], partial[b * 6 + 3 + a]);
    }
  for (int a = 0; a < 6; ++a) s[a][t] = v[a];
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off)
      for (int a = 0; a < 3; ++a) {
        s[a][t] = fmin(s[a][t], s[a][t + off]);
        s[3 + a][t] = fmax(s[3 + a][t], s[3 + a][t + off]);
      }
    __syncthreads();
  }
  if (t == 0) {
    double ext = 0.0;
    for (int a = 0; a < 3; ++a) ext = fmax(ext, s[3 + a][0] - s[a][0]);
    // cells slightly larger than r; larger still when the box would need
    // more than 2^21 cells along an axis
    const double h = fmax(r * (1.0 + 1e-8), (ext + 4.0 * r) / kMaxCells);
    for (int a = 0; a < 3; ++a) gp->lo[a] = s[a][0] - 2.0 * h;  // cell coordinates >= 1
    gp->inv_h = 1.0 / h;
    gp->r2 = r * r;
  }
}

// ---- cells ---------------------------------------------------------------------
__global__ void __launch_bounds__(256)
k_cell_insert(const double *__restrict__ src, int64_t n, const GridParams *__restrict__ gp,
              uint64_t *__restrict__ keys, int32_t *__restrict__ counts, uint32_t mask,
              int32_t *__restrict__ src_slot) {
  const double lo0 = gp->lo[0], lo1 = gp->lo[1], lo2 = gp->lo[2], ih = gp->inv_h;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = cell_key(cell_of(src[3 * i], lo0, ih), cell_of(src[3 * i + 1], lo1, ih),
                                  cell_of(src[3 * i + 2], lo2, ih));
    uint32_t s = hash_slot(key, mask);
    for (;;) {  // the table is at most half full, so a free or matching slot exists
      const unsigned long long prev =
          atomicCAS((unsigned long long *)&keys[s], (unsigned long long)kEmpty,
                    (unsigned long long)key);
      if (prev == kEmpty || prev == key) break;
      s = (s + 1) & mask;
    }
    atomicAdd(&counts[s], 1);
    src_slot[i] = (int32_t)s;
  }
}

__global__ void __launch_bounds__(256)
k_cell_scatter(const double *__restrict__ src, int64_t n, const int32_t *__restrict__ src_slot,
               int64_t *__restrict__ cursor, double4 *__restrict__ cell_pts) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t pos = atomicAdd((unsigned long long *)&cursor[src_slot[i]], 1ull);
    cell_pts[pos] = make_double4(src[3 * i], src[3 * i + 1], src[3 * i + 2], (double)i);
  }
}

// ---- exclusive scan (int32 or int64 in, int64 out) -------------------------------
template <class T>
__global__ void __launch_bounds__(256)
k_scan_blocks(const T *__restrict__ in, int64_t n, int64_t *__restrict__ out,
              int64_t *__restrict__ block_sums) {
  __shared__ int64_t s[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + (int64_t)t * kScanItems;
  int64_t v[kScanItems];
  int64_t sum = 0;
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = base + j < n ? (int64_t)in[base + j] : 0;
    sum += v[j];
  }
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive Hillis-Steele scan
    const int64_t x = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int64_t run = s[t] - sum;
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) out[base + j] = run;
    run += v[j];
  }
  if (t == 255) block_sums[blockIdx.x] = s[255];
}

// Exclusive scan of the block sums by one workgroup; total -> *total.
__global__ void __launch_bounds__(256)
k_scan_top(int64_t *__restrict__ sums, int64_t nb, int64_t *__restrict__ total) {
  __shared__ int64_t s[256];
  const int t = threadIdx.x;
  const int64_t per = (nb + 255) / 256;
  const int64_t b0 = t * per, b1 = std::min<int64_t>(nb, b0 + per);
  int64_t sum = 0;
  for (int64_t b = b0; b < b1; ++b) sum += sums[b];
  s[t] = sum;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    const int64_t x = t >= off ? s[t - off] : 0;
    __syncthreads();
    s[t] += x;
    __syncthreads();
  }
  int64_t run = s[t] - sum;
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t x = sums[b];
    sums[b] = run;
    run += x;
  }
  if (t == 255) *total = s[255];
}

__global__ void __launch_bounds__(256)
k_scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ block_sums) {
  const int64_t i = (int64_t)blockIdx.x * kScanBlock;
  const int64_t add = block_sums[blockIdx.x];
  for (int j = threadIdx.x; j < kScanBlock; j += blockDim.x)
    if (i + j < n) out[i + j] += add;
}

// ---- per-center passes -------------------------------------------------------------
// One wave per center.  count: row_count[c] = members; fill: members written
// from out_idx + offsets[c] in cell order (sorted afterwards).
template <bool kFill>
__global__ void __launch_bounds__(256)
k_ball_pass(const double *__restrict__ ctr, int64_t m, const GridParams *__restrict__ gp,
            const uint64_t *__restrict__ keys, uint32_t mask,
            const int64_t *__restrict__ cell_start, const int32_t *__restrict__ cell_count,
            const double4 *__restrict__ cell_pts, int64_t *__restrict__ row_count,
            const int64_t *__restrict__ offsets, int32_t *__restrict__ out_idx) {
  const int lane = threadIdx.x & 63;
  const int64_t c = __builtin_amdgcn_readfirstlane(
      (int)((int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)));
  if (c >= m) return;
  const double cx = ctr[3 * c], cy = ctr[3 * c + 1], cz = ctr[3 * c + 2];
  const double ih = gp->inv_h, r2 = gp->r2;
  const uint32_t ix = cell_of(cx, gp->lo[0], ih), iy = cell_of(cy, gp->lo[1], ih),
                 iz = cell_of(cz, gp->lo[2], ih);
  int64_t cnt = 0;
  int32_t *dst = kFill ? out_idx + offsets[c] : nullptr;
  for (int d = 0; d < 27; ++d) {
    const uint64_t key = cell_key(ix + d / 9 - 1, iy + (d / 3) % 3 - 1, iz + d % 3 - 1);
    const int64_t slot = find_slot(keys, mask, key);
    if (slot < 0) continue;
    const int64_t beg = cell_start[slot];
    const int num = cell_count[slot];
    for (int j0 = 0; j0 < num; j0 += 64) {
      const int j = j0 + lane;
      bool hit = false;
      double w = 0.0;
      if (j < num) {
        const double4 p = cell_pts[beg + j];
        const double dx = p.x - cx, dy = p.y - cy, dz = p.z - cz;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        hit = d2 <= r2;
        w = p.w;
      }
      const uint64_t bal = __ballot(hit);
      if constexpr (kFill) {
        if (hit) {
          const uint64_t below = lane ? (bal & (~0ull >> (64 - lane))) : 0ull;
          dst[cnt + __popcll(below)] = (int32_t)w;
        }
      }
      cnt += __popcll(bal);
    }
  }
  if (!kFill && lane == 0) row_count[c] = cnt;
}

// ---- row sort --------------------------------------------------------------------
constexpr int kSortMax = 8192;

// CAP: the LDS capacity, at least the longest row (smaller capacities let
// more workgroups share a CU).
template <int CAP>
__global__ void __launch_bounds__(256)
k_row_sort(const int64_t *__restrict__ offsets, int32_t *__restrict__ idx) {
  __shared__ int32_t s[CAP];
  const int64_t b = offsets[blockIdx.x];
  const int len = (int)(offsets[blockIdx.x + 1] - b);
  if (len <= 1) return;
  int P = 1;
  while (P < len) P <<= 1;
  for (int i = threadIdx.x; i < P; i += blockDim.x) s[i] = i < len ? idx[b + i] : INT32_MAX;
  __syncthreads();
  // bitonic network over the P/2 compare-exchange pairs of each stage
  const int half = P >> 1;
  for (int k = 2; k <= P; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = threadIdx.x; q < half; q += blockDim.x) {
        const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));  // lower index of pair q
        const int l = i | j;
        const int32_t x = s[i], y = s[l];
        const bool up = (i & k) == 0;
        if ((x > y) == up) {
          s[i] = y;
          s[l] = x;
        }
      }
      __syncthreads();
    }
  for (int i = threadIdx.x; i < len; i += blockDim.x) idx[b + i] = s[i];
}

__global__ void __launch_bounds__(256)
k_max_row(const int64_t *__restrict__ offsets, int64_t m, unsigned long long *__restrict__ out) {
  unsigned long long mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    mx = std::max<unsigned long long>(mx, (unsigned long long)(offsets[i + 1] - offsets[i]));
  atomicMax(out, mx);
}

// Exclusive scan of n values into out[0..n], out[n] = total (device).
template <class T>
hipError_t scan_exclusive(const T *in, int64_t n, int64_t *out, int64_t *scratch,
                          hipStream_t s) {
  const int64_t nb = std::max<int64_t>(1, (n + kScanBlock - 1) / kScanBlock);
  hipLaunchKernelGGL(k_scan_blocks<T>, dim3((unsigned)nb), dim3(256), 0, s, in, n, out, scratch);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(256), 0, s, scratch, nb, out + n);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(256), 0, s, out, n, scratch);
  return hipGetLastError();
}

template <class T>
struct DevBuf {
  T *p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  hipError_t alloc(size_t n) { return hipMalloc((void **)&p, std::max<size_t>(n, 1) * sizeof(T)); }
};

}  // namespace
}  // namespace tsqbx

using namespace tsqbx;

extern "C" int tsqbx_ball_lists(tsqbx_ctx *ctx, int64_t n_sources, const double *d_sources,
                                int64_t n_centers, const double *d_centers, double radius,
                                int64_t *d_offsets, int32_t *d_indices, int64_t capacity,
                                int64_t *nnz, void *hip_stream) {
  if (!ctx || !nnz || !d_offsets) return fail(TSQBX_E_INVALID, "ctx, offsets or nnz is NULL");
  if (n_sources < 0 || n_centers < 0 || capacity < 0)
    return fail(TSQBX_E_INVALID, "negative count");
  if (n_sources >= TSQBX_MAX_SOURCES)
    return fail(TSQBX_E_RANGE, "n_sources = %lld; at most %lld", (long long)n_sources,
                (long long)TSQBX_MAX_SOURCES - 1);
  if (n_centers > INT32_MAX) return fail(TSQBX_E_RANGE, "n_centers must stay below 2^31");
  if ((n_sources > 0 && !d_sources) || (n_centers > 0 && !d_centers) ||
      (capacity > 0 && !d_indices))
    return fail(TSQBX_E_INVALID, "sources, centers or indices is NULL");
  if (!(radius > 0.0) || !std::isfinite(radius))
    return fail(TSQBX_E_RANGE, "radius = %g must be positive and finite", radius);
  *nnz = 0;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != ctx->device) TSQBX_HIP(hipSetDevice(ctx->device));
  struct Restore {
    int dev;
    ~Restore() {
      if (dev >= 0) (void)hipSetDevice(dev);
    }
  } restore{prev};
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t N = n_sources, M = n_centers;
  if (M == 0) {
    TSQBX_HIP(hipMemsetAsync(d_offsets, 0, sizeof(int64_t), s));
    TSQBX_HIP(hipStreamSynchronize(s));
    return TSQBX_OK;
  }
  // table of at most half load
  uint32_t cap = 1024;
  while ((int64_t)cap < 2 * N) cap <<= 1;
  const uint32_t mask = cap - 1;
  const int bb_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (N + M + 255) / 256));
  DevBuf<double> partial;
  DevBuf<GridParams> gp;
  DevBuf<uint64_t> keys;
  DevBuf<int32_t> counts, src_slot;
  DevBuf<int64_t> cell_start, cursor, row_count, scan_tmp;
  DevBuf<double4> cell_pts;
  DevBuf<unsigned long long> maxrow;
  const int64_t scan_blocks = std::max<int64_t>((int64_t)cap, M) / kScanBlock + 2;
  TSQBX_HIP(partial.alloc(6 * (size_t)bb_blocks));
  TSQBX_HIP(gp.alloc(1));
  TSQBX_HIP(keys.alloc(cap));
  TSQBX_HIP(counts.alloc(cap));
  TSQBX_HIP(cell_start.alloc((size_t)cap + 1));
  TSQBX_HIP(cursor.alloc((size_t)cap + 1));
  TSQBX_HIP(src_slot.alloc((size_t)N));
  TSQBX_HIP(cell_pts.alloc((size_t)N));
  TSQBX_HIP(row_count.alloc((size_t)M));
  TSQBX_HIP(scan_tmp.alloc((size_t)scan_blocks));
  TSQBX_HIP(maxrow.alloc(1));
  TSQBX_HIP(hipMemsetAsync(keys.p, 0xff, (size_t)cap * sizeof(uint64_t), s));
  TSQBX_HIP(hipMemsetAsync(counts.p, 0, (size_t)cap * sizeof(int32_t), s));
  TSQBX_HIP(hipMemsetAsync(maxrow.p, 0, sizeof(unsigned long long), s));
  hipLaunchKernelGGL(k_bbox_partial, dim3(bb_blocks), dim3(256), 0, s, d_sources, N, d_centers, M,
                     partial.p);
  hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(256), 0, s, partial.p, bb_blocks, radius, gp.p);
  const unsigned gs = (unsigned)std::min<int64_t>(65536, std::max<int64_t>(1, (N + 255) / 256));
  if (N > 0) {
    hipLaunchKernelGGL(k_cell_insert, dim3(gs), dim3(256), 0, s, d_sources, N, gp.p, keys.p,
                       counts.p, mask, src_slot.p);
  }
  TSQBX_HIP(hipGetLastError());
  TSQBX_HIP(scan_exclusive(counts.p, (int64_t)cap, cell_start.p, scan_tmp.p, s));
  TSQBX_HIP(hipMemcpyAsync(cursor.p, cell_start.p, ((size_t)cap + 1) * sizeof(int64_t),
                           hipMemcpyDeviceToDevice, s));
  if (N > 0)
    hipLaunchKernelGGL(k_cell_scatter, dim3(gs), dim3(256), 0, s, d_sources, N, src_slot.p,
                       cursor.p, cell_pts.p);
  const unsigned wb = (unsigned)((M + 3) / 4);  // 4 waves (centers) per block
  hipLaunchKernelGGL(k_ball_pass<false>, dim3(wb), dim3(256), 0, s, d_centers, M, gp.p, keys.p,
                     mask, cell_start.p, counts.p, cell_pts.p, row_count.p, nullptr, nullptr);
  TSQBX_HIP(hipGetLastError());
  TSQBX_HIP(scan_exclusive(row_count.p, M, d_offsets, scan_tmp.p, s));
  hipLaunchKernelGGL(k_max_row, dim3((unsigned)std::min<int64_t>(1024, (M + 255) / 256)),
                     dim3(256), 0, s, d_offsets, M, maxrow.p);
  TSQBX_HIP(hipGetLastError());
  int64_t total = 0;
  unsigned long long longest = 0;
  TSQBX_HIP(hipMemcpyAsync(&total, d_offsets + M, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TSQBX_HIP(hipMemcpyAsync(&longest, maxrow.p, sizeof(longest), hipMemcpyDeviceToHost, s));
  TSQBX_HIP(hipStreamSynchronize(s));
  *nnz = total;
  if ((int64_t)longest > kSortMax)
    return fail(TSQBX_E_RANGE, "a ball holds %llu sources; at most %d per center", longest,
                kSortMax);
  if (total > capacity)
    return fail(TSQBX_E_RANGE, "the lists need %lld entries; capacity is %lld", (long long)total,
                (long long)capacity);
  if (total > 0) {
    hipLaunchKernelGGL(k_ball_pass<true>, dim3(wb), dim3(256), 0, s, d_centers, M, gp.p, keys.p,
                       mask, cell_start.p, counts.p, cell_pts.p, nullptr, d_offsets, d_indices);
    if (longest <= 512)
      hipLaunchKernelGGL(k_row_sort<512>, dim3((unsigned)M), dim3(256), 0, s, d_offsets, d_indices);
    else if (longest <= 2048)
      hipLaunchKernelGGL(k_row_sort<2048>, dim3((unsigned)M), dim3(256), 0, s, d_offsets, d_indices);
    else
      hipLaunchKernelGGL(k_row_sort<kSortMax>, dim3((unsigned)M), dim3(256), 0, s, d_offsets,
                         d_indices);
    TSQBX_HIP(hipGetLastError());
  }
  TSQBX_HIP(hipStreamSynchronize(s));
  return TSQBX_OK;
}
