// Near-field list construction on the device: for every QBX center the
// sources inside the closed ball of radius r about it, or the k_c sources
// nearest to it (the near-field source set of Sec. 3.3, taken as a ball or as
// nearest neighbours as in the workloads), as CSR with ascending source
// indices.
//
// Distances are formed in FP64 exactly as written: dx = y_x - c_x (likewise
// y, z), d2 = (dx*dx + dy*dy) + dz*dz with every operation rounded on its own
// (the library is built without FP contraction).  Ball: member iff d2 <= r*r.
// Nearest: the k_c smallest sources in the order of the 96-bit key
// (bits of d2, source index), so equal distances go to the smaller index.
//
// Both start from a uniform grid hashed into an open-addressing table: a
// bounding box, cells of size h, sources counted per cell, scanned and
// scattered into cell order.  Ball: h >= r(1 + 1e-8), so that rounding in the
// cell coordinates cannot move a member out of the 27 cells around its
// center's cell; one wave per center counts its members, the counts are
// scanned into the row offsets, a second pass writes the members, and one
// workgroup per row sorts it in LDS.  Nearest: h from the source density; one
// workgroup per center grows rings of cells until they hold k_c sources,
// bounds the k_c-th distance from the cells' far corners, gathers the cells
// that can hold a closer source and selects the k_c smallest keys among their
// sources by a most-significant-digit radix select; the rows are then sorted
// as for balls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include <rocprim/block/block_radix_sort.hpp>

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
  double h;
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

// r > 0: cells for balls of radius r.  r = 0: cells for nearest-neighbour
// search over n_src sources, h = ext (4 / n_src)^(1/3) (a few sources per
// occupied cell of a surface, about 4 per cell of a uniform volume).
__global__ void __launch_bounds__(256)
k_grid_params(const double *__restrict__ partial, int nb, double r, int64_t n_src,
              GridParams *__restrict__ gp) {
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
    // ball cells slightly larger than r; larger still when the box would need
    // more than 2^21 cells along an axis
    double h0 = r * (1.0 + 1e-8);
    if (!(r > 0.0)) h0 = ext > 0.0 ? ext * cbrt(4.0 / (double)(n_src > 0 ? n_src : 1)) : 1.0;
    const double h = fmax(h0, (ext + 4.0 * h0) / kMaxCells);
    for (int a = 0; a < 3; ++a) gp->lo[a] = s[a][0] - 2.0 * h;  // cell coordinates >= 1
    gp->inv_h = 1.0 / h;
    gp->r2 = r * r;
    gp->h = h;
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

// ---- k nearest ---------------------------------------------------------------------
constexpr int kKnnCells = 4096;  // cells a center keeps in LDS
constexpr int kKnnRank = 256;    // keys ranked one against another at the end

// Cell offset (a, b, e) of entry q of ring r, the cells with
// max(|a|, |b|, |e|) = r: the two z faces, then the two y faces without their
// z edges, then the two x faces without their y and z edges.  The ring has
// 24 r^2 + 2 cells (1 for r = 0).
__device__ __forceinline__ void ring_cell(int r, int q, int &a, int &b, int &e) {
  if (r == 0) {
    a = b = e = 0;
    return;
  }
  const int w = 2 * r + 1, v = 2 * r - 1;
  const int f1 = w * w, f2 = w * v, f3 = v * v;
  if (q < 2 * f1) {
    e = q < f1 ? -r : r;
    const int x = q % f1;
    a = x / w - r;
    b = x % w - r;
  } else if ((q -= 2 * f1) < 2 * f2) {
    b = q < f2 ? -r : r;
    const int x = q % f2;
    a = x / v - r;
    e = x % v - (r - 1);
  } else {
    q -= 2 * f2;
    a = q < f3 ? -r : r;
    const int x = q % f3;
    b = x / v - (r - 1);
    e = x % v - (r - 1);
  }
}

__device__ __forceinline__ int ring_size(int r) { return r == 0 ? 1 : 24 * r * r + 2; }

// Slot of cell (jx, jy, jz) in the table, or -1 (empty or outside the grid).
__device__ __forceinline__ int64_t cell_slot(const uint64_t *__restrict__ keys, uint32_t mask,
                                             int jx, int jy, int jz) {
  constexpr int lim = 1 << kCellBits;
  if (jx < 0 || jy < 0 || jz < 0 || jx >= lim || jy >= lim || jz >= lim) return -1;
  return find_slot(keys, mask, cell_key((uint32_t)jx, (uint32_t)jy, (uint32_t)jz));
}

// Nearest (q = 0) and farthest (q = 1) squared distance from (cx, cy, cz) to
// the cell (jx, jy, jz), from its corner coordinates lo + j h.
__device__ __forceinline__ double cell_dist2(const GridParams &g, double cx, double cy, double cz,
                                             int jx, int jy, int jz, bool far) {
  const double c[3] = {cx, cy, cz};
  const int j[3] = {jx, jy, jz};
  double d2 = 0.0;
  for (int a = 0; a < 3; ++a) {
    const double lo = g.lo[a] + (double)j[a] * g.h, hi = lo + g.h;
    const double t = far ? fmax(c[a] - lo, hi - c[a]) : fmax(0.0, fmax(lo - c[a], c[a] - hi));
    d2 += t * t;
  }
  return d2;
}

__device__ __forceinline__ bool key_matches(uint64_t hi, uint32_t lo, int nbits, uint64_t p_hi,
                                            uint32_t p_lo) {
  if (nbits == 0) return true;
  if (nbits <= 64) return (hi >> (64 - nbits)) == p_hi;
  return hi == p_hi && (lo >> (96 - nbits)) == p_lo;
}

__device__ __forceinline__ uint32_t key_digit(uint64_t hi, uint32_t lo, int nbits) {
  return nbits < 64 ? (uint32_t)(hi >> (56 - nbits)) & 255u : (lo >> (88 - nbits)) & 255u;
}

__device__ __forceinline__ bool key_less(uint64_t ah, uint32_t al, uint64_t bh, uint32_t bl) {
  return ah < bh || (ah == bh && al < bl);
}

// One workgroup (256 threads) per center c with k = counts[c] > 0: writes
// the k nearest sources to out_idx[offsets[c] ...] in arbitrary order.  A
// count that does not come out at k sets *err (never expected).
__global__ void __launch_bounds__(256)
k_knn(const double *__restrict__ ctr, const int32_t *__restrict__ counts,
      const int64_t *__restrict__ offsets, const GridParams *__restrict__ gpp,
      const uint64_t *__restrict__ keys, uint32_t mask, const int64_t *__restrict__ cell_start,
      const int32_t *__restrict__ cell_count, const double4 *__restrict__ cell_pts,
      int32_t *__restrict__ out_idx, int *__restrict__ err) {
  __shared__ int32_t cells[kKnnCells];
  __shared__ uint32_t hist[256];
  __shared__ uint64_t rank_hi[kKnnRank];
  __shared__ uint32_t rank_lo[kKnnRank];
  __shared__ int n_cells, n_rank, n_out;
  __shared__ unsigned long long found, kmin, kmax;
  __shared__ uint64_t p_hi, t_hi;
  __shared__ uint32_t p_lo, t_lo;
  __shared__ int nbits, need, done;
  __shared__ double bound;

  const int64_t c = blockIdx.x;
  const int k = counts[c];
  if (k <= 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const GridParams g = *gpp;
  const double cx = ctr[3 * c], cy = ctr[3 * c + 1], cz = ctr[3 * c + 2];
  const int ix = (int)cell_of(cx, g.lo[0], g.inv_h), iy = (int)cell_of(cy, g.lo[1], g.inv_h),
            iz = (int)cell_of(cz, g.lo[2], g.inv_h);
  // slack for rounding in cell coordinates and distances: 1e-9 of the
  // largest coordinate magnitude the grid can hold
  const double mu = 1e-9 * (g.h * (double)(1 << kCellBits) + fabs(g.lo[0]) + fabs(g.lo[1]) +
                            fabs(g.lo[2]) + fabs(cx) + fabs(cy) + fabs(cz));

  // 1. rings of cells around the center's cell until they hold k sources
  if (tid == 0) {
    n_cells = 0;
    found = 0;
  }
  __syncthreads();
  int rings = 0;
  for (;; ++rings) {
    unsigned long long local = 0;
    for (int q = tid; q < ring_size(rings); q += 256) {
      int a, b, e;
      ring_cell(rings, q, a, b, e);
      const int64_t slot = cell_slot(keys, mask, ix + a, iy + b, iz + e);
      if (slot < 0) continue;
      local += (unsigned long long)cell_count[slot];
      const int pos = atomicAdd(&n_cells, 1);
      if (pos < kKnnCells) cells[pos] = (int32_t)slot;
    }
    if (local) atomicAdd(&found, local);
    __syncthreads();
    const bool enough = found >= (unsigned long long)k;
    __syncthreads();
    if (enough) break;
  }

  // 2. a bound on the k-th distance: the cells' farthest corners, weighted
  // by their counts, in 64 bins up to the rings' corner radius
  const double dmax = sqrt(3.0) * (double)(rings + 1) * g.h + 4.0 * mu;
  if (tid < 64) hist[tid] = 0;
  if (tid == 0) bound = dmax;
  __syncthreads();
  const int nc1 = n_cells;
  if (nc1 <= kKnnCells) {
    for (int i = tid; i < nc1; i += 256) {
      const int slot = cells[i];
      const uint64_t key = keys[slot];
      const int jx = (int)(key >> (2 * kCellBits)), jy = (int)((key >> kCellBits) & ((1u << kCellBits) - 1)),
                jz = (int)(key & ((1u << kCellBits) - 1));
      const double df = sqrt(cell_dist2(g, cx, cy, cz, jx, jy, jz, true)) + mu;
      const int bin = min(63, (int)(df * (64.0 / dmax)));
      atomicAdd(&hist[bin], (uint32_t)cell_count[slot]);
    }
    __syncthreads();
    if (tid == 0) {
      uint64_t cum = 0;
      for (int b = 0; b < 64; ++b) {
        cum += hist[b];
        if (cum >= (uint64_t)k) {
          bound = fmin(dmax, (double)(b + 1) * (dmax / 64.0) * (1.0 + 1e-12) + mu);
          break;
        }
      }
    }
  }
  __syncthreads();
  const double D = bound + mu;              // every one of the k lies within D
  const double lim2 = D * D;                // candidates: d2 <= lim2
  const double cell_lim2 = (D + mu) * (D + mu);

  // 3. the cells that can hold a source with d2 <= lim2
  const int M = (int)ceil(D * g.inv_h) + 1;
  if (tid == 0) n_cells = 0;
  __syncthreads();
  for (int r = 0; r <= M; ++r)
    for (int q = tid; q < ring_size(r); q += 256) {
      int a, b, e;
      ring_cell(r, q, a, b, e);
      if (cell_dist2(g, cx, cy, cz, ix + a, iy + b, iz + e, false) > cell_lim2) continue;
      const int64_t slot = cell_slot(keys, mask, ix + a, iy + b, iz + e);
      if (slot < 0) continue;
      const int pos = atomicAdd(&n_cells, 1);
      if (pos < kKnnCells) cells[pos] = (int32_t)slot;
    }
  __syncthreads();
  const int nc = n_cells;
  const bool cached = nc <= kKnnCells;
  const int64_t w_box = 2 * (int64_t)M + 1;
  const int64_t n_box = w_box * w_box * w_box;

  // every candidate (d2 <= lim2) once: a wave per cell, its lanes over the
  // cell's sources (from the cached cells, else from the whole box)
  auto for_each = [&](auto &&fn) {
    const int64_t n_iter = cached ? nc : n_box;
    for (int64_t i = wave; i < n_iter; i += 4) {
      int64_t slot;
      if (cached) {
        slot = cells[i];
      } else {
        const int a = (int)(i / (w_box * w_box)) - M, b = (int)((i / w_box) % w_box) - M,
                  e = (int)(i % w_box) - M;
        if (cell_dist2(g, cx, cy, cz, ix + a, iy + b, iz + e, false) > cell_lim2) continue;
        slot = cell_slot(keys, mask, ix + a, iy + b, iz + e);
        if (slot < 0) continue;
      }
      const int64_t beg = cell_start[slot];
      const int num = cell_count[slot];
      for (int j = lane; j < num; j += 64) {
        const double4 pt = cell_pts[beg + j];
        const double dx = pt.x - cx, dy = pt.y - cy, dz = pt.z - cz;
        const double d2 = (dx * dx + dy * dy) + dz * dz;
        if (d2 <= lim2) fn((uint64_t)__double_as_longlong(d2), (uint32_t)pt.w);
      }
    }
  };

  // 4. radix select of the k-th smallest key, from the first digit where the
  // candidates' distances differ
  if (tid == 0) {
    kmin = ~0ull;
    kmax = 0;
  }
  __syncthreads();
  for_each([&](uint64_t hi, uint32_t) {
    atomicMin(&kmin, (unsigned long long)hi);
    atomicMax(&kmax, (unsigned long long)hi);
  });
  __syncthreads();
  if (tid == 0) {
    const uint64_t x = kmin ^ kmax;
    const int nb0 = x ? (__clzll((long long)x) / 8) * 8 : 64;
    nbits = nb0;
    p_hi = nb0 ? (uint64_t)kmin >> (64 - nb0) : 0;
    p_lo = 0;
    need = k;
    done = 0;
  }
  __syncthreads();
  for (;;) {
    hist[tid] = 0;
    __syncthreads();
    const int nb = nbits;
    const uint64_t ph = p_hi;
    const uint32_t pl = p_lo;
    for_each([&](uint64_t hi, uint32_t lo) {
      if (key_matches(hi, lo, nb, ph, pl)) atomicAdd(&hist[key_digit(hi, lo, nb)], 1u);
    });
    __syncthreads();
    if (tid == 0) {
      int cum = 0, d = 0;
      for (; d < 255; ++d) {
        if (cum + (int)hist[d] >= need) break;
        cum += (int)hist[d];
      }
      need -= cum;
      if (nb < 64)
        p_hi = (p_hi << 8) | d;
      else
        p_lo = (p_lo << 8) | (uint32_t)d;
      nbits = nb + 8;
      done = (int)hist[d] <= kKnnRank || nb + 8 == 96;
    }
    __syncthreads();
    if (done) break;
  }
  if (tid == 0) n_rank = 0;
  __syncthreads();
  {
    const int nb = nbits;
    const uint64_t ph = p_hi;
    const uint32_t pl = p_lo;
    for_each([&](uint64_t hi, uint32_t lo) {
      if (key_matches(hi, lo, nb, ph, pl)) {
        const int pos = atomicAdd(&n_rank, 1);
        if (pos < kKnnRank) {
          rank_hi[pos] = hi;
          rank_lo[pos] = lo;
        }
      }
    });
  }
  __syncthreads();
  const int nr = min(n_rank, kKnnRank);
  if (tid < nr) {
    int below = 0;
    for (int j = 0; j < nr; ++j) below += key_less(rank_hi[j], rank_lo[j], rank_hi[tid], rank_lo[tid]);
    if (below == need - 1) {
      t_hi = rank_hi[tid];
      t_lo = rank_lo[tid];
    }
  }
  if (tid == 0) n_out = 0;
  __syncthreads();

  // 5. the k keys up to the threshold
  int32_t *row = out_idx + offsets[c];
  const uint64_t th = t_hi;
  const uint32_t tl = t_lo;
  for_each([&](uint64_t hi, uint32_t lo) {
    if (!key_less(th, tl, hi, lo)) {
      const int pos = atomicAdd(&n_out, 1);
      if (pos < k) row[pos] = (int32_t)lo;
    }
  });
  __syncthreads();
  if (tid == 0 && (n_out != k || n_rank > kKnnRank || n_rank < need)) atomicExch(err, 1);
}

// ---- row sort --------------------------------------------------------------------
// One workgroup per row whose length lies in (min_len, ITEMS x 256]: a
// block-wide LSD radix sort of the row's entries in registers and LDS
// (rocPRIM's block radix sort, 4 bits per pass), on the end_bit low bits
// that hold every entry; padding keys (2^end_bit - 1, above every entry) sort
// last and are not written back.  Rows of other lengths are left to the
// launches of the other length classes.
template <int ITEMS>
__global__ void __launch_bounds__(256)
k_row_sort(const int64_t *__restrict__ offsets, int32_t *__restrict__ idx, int end_bit,
           int min_len) {
  using Sort = rocprim::block_radix_sort<uint32_t, 256, ITEMS>;
  __shared__ typename Sort::storage_type storage;
  const int64_t b = offsets[blockIdx.x];
  const int64_t len64 = offsets[blockIdx.x + 1] - b;
  if (len64 <= min_len || len64 <= 1 || len64 > 256 * ITEMS) return;
  const int len = (int)len64;
  const uint32_t pad = (1u << end_bit) - 1u;
  uint32_t k[ITEMS];
  for (int j = 0; j < ITEMS; ++j) {  // blocked: thread t holds entries t ITEMS ..
    const int i = (int)threadIdx.x * ITEMS + j;
    k[j] = i < len ? (uint32_t)idx[b + i] : pad;
  }
  Sort().sort(k, storage, 0, (unsigned)end_bit);
  for (int j = 0; j < ITEMS; ++j) {
    const int i = (int)threadIdx.x * ITEMS + j;
    if (i < len) idx[b + i] = (int32_t)k[j];
  }
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

// The hashed grid of the sources, in cell order (cell_pts = (x, y, z, index)).
struct Grid {
  uint32_t cap = 0, mask = 0;
  int bb_blocks = 1;
  DevBuf<double> partial;
  DevBuf<GridParams> gp;
  DevBuf<uint64_t> keys;
  DevBuf<int32_t> counts, src_slot;
  DevBuf<int64_t> cell_start, cursor, scan_tmp;
  DevBuf<double4> cell_pts;
};

// r > 0: cells for balls of radius r; r = 0: cells for nearest neighbours.
// scan_items: the longest scan the caller will run on g.scan_tmp.
hipError_t build_grid(Grid &g, int64_t N, const double *d_sources, int64_t M,
                      const double *d_centers, double r, int64_t scan_items, hipStream_t s) {
  g.cap = 1024;  // a table of at most half load
  while ((int64_t)g.cap < 2 * N) g.cap <<= 1;
  g.mask = g.cap - 1;
  g.bb_blocks = (int)std::min<int64_t>(1024, std::max<int64_t>(1, (N + M + 255) / 256));
  const int64_t scan_blocks = std::max<int64_t>((int64_t)g.cap, scan_items) / kScanBlock + 2;
  hipError_t e;
  if ((e = g.partial.alloc(6 * (size_t)g.bb_blocks)) != hipSuccess) return e;
  if ((e = g.gp.alloc(1)) != hipSuccess) return e;
  if ((e = g.keys.alloc(g.cap)) != hipSuccess) return e;
  if ((e = g.counts.alloc(g.cap)) != hipSuccess) return e;
  if ((e = g.cell_start.alloc((size_t)g.cap + 1)) != hipSuccess) return e;
  if ((e = g.cursor.alloc((size_t)g.cap + 1)) != hipSuccess) return e;
  if ((e = g.src_slot.alloc((size_t)N)) != hipSuccess) return e;
  if ((e = g.cell_pts.alloc((size_t)N)) != hipSuccess) return e;
  if ((e = g.scan_tmp.alloc((size_t)scan_blocks)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(g.keys.p, 0xff, (size_t)g.cap * sizeof(uint64_t), s)) != hipSuccess)
    return e;
  if ((e = hipMemsetAsync(g.counts.p, 0, (size_t)g.cap * sizeof(int32_t), s)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_bbox_partial, dim3(g.bb_blocks), dim3(256), 0, s, d_sources, N, d_centers,
                     M, g.partial.p);
  hipLaunchKernelGGL(k_grid_params, dim3(1), dim3(256), 0, s, g.partial.p, g.bb_blocks, r, N,
                     g.gp.p);
  const unsigned gs = (unsigned)std::min<int64_t>(65536, std::max<int64_t>(1, (N + 255) / 256));
  if (N > 0)
    hipLaunchKernelGGL(k_cell_insert, dim3(gs), dim3(256), 0, s, d_sources, N, g.gp.p, g.keys.p,
                       g.counts.p, g.mask, g.src_slot.p);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  if ((e = scan_exclusive(g.counts.p, (int64_t)g.cap, g.cell_start.p, g.scan_tmp.p, s)) !=
      hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(g.cursor.p, g.cell_start.p, ((size_t)g.cap + 1) * sizeof(int64_t),
                          hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return e;
  if (N > 0)
    hipLaunchKernelGGL(k_cell_scatter, dim3(gs), dim3(256), 0, s, d_sources, N, g.src_slot.p,
                       g.cursor.p, g.cell_pts.p);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
k_count_range(const int32_t *__restrict__ counts, int64_t m, int *__restrict__ out) {
  int mn = INT32_MAX, mx = INT32_MIN;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    mn = min(mn, counts[i]);
    mx = max(mx, counts[i]);
  }
  atomicMin(&out[0], mn);
  atomicMax(&out[1], mx);
}

struct RestoreDevice {
  int dev;
  ~RestoreDevice() {
    if (dev >= 0) (void)hipSetDevice(dev);
  }
};

}  // namespace

hipError_t sort_rows(const int64_t *d_offsets, int32_t *d_indices, int64_t M,
                     int64_t longest, int64_t max_value, hipStream_t s) {
  if (M <= 0 || longest <= 1) return hipSuccess;
  if (longest > kRowSortMax || M > INT32_MAX || max_value >= INT32_MAX) return hipErrorInvalidValue;
  int end_bit = 1;  // 2^end_bit - 1 > max_value: the padding key sorts after every entry
  while ((int64_t(1) << end_bit) - 1 <= max_value) ++end_bit;
  // one launch per length class up to the longest row
  hipLaunchKernelGGL(k_row_sort<2>, dim3((unsigned)M), dim3(256), 0, s, d_offsets, d_indices,
                     end_bit, 0);
  if (longest > 512)
    hipLaunchKernelGGL(k_row_sort<8>, dim3((unsigned)M), dim3(256), 0, s, d_offsets, d_indices,
                       end_bit, 512);
  if (longest > 2048)
    hipLaunchKernelGGL(k_row_sort<(int)(kRowSortMax / 256)>, dim3((unsigned)M), dim3(256), 0, s, d_offsets,
                       d_indices, end_bit, 2048);
  return hipGetLastError();
}

}  // namespace tsqbx

using namespace tsqbx;

extern "C" int tsqbx_ball_lists(tsqbx_ctx *ctx, int64_t n_sources, const double *d_sources,
                                int64_t n_centers, const double *d_centers, double radius,
                                int64_t *d_offsets, int32_t *d_indices, int64_t capacity,
                                int64_t *nnz, void *hip_stream) {
  TraceRange trace_("tsqbx_ball_lists");
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
  RestoreDevice restore{prev};
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t N = n_sources, M = n_centers;
  if (M == 0) {
    TSQBX_HIP(hipMemsetAsync(d_offsets, 0, sizeof(int64_t), s));
    TSQBX_HIP(hipStreamSynchronize(s));
    return TSQBX_OK;
  }
  Grid g;
  TSQBX_HIP(build_grid(g, N, d_sources, M, d_centers, radius, M, s));
  DevBuf<int64_t> row_count;
  DevBuf<unsigned long long> maxrow;
  TSQBX_HIP(row_count.alloc((size_t)M));
  TSQBX_HIP(maxrow.alloc(1));
  TSQBX_HIP(hipMemsetAsync(maxrow.p, 0, sizeof(unsigned long long), s));
  const unsigned wb = (unsigned)((M + 3) / 4);  // 4 waves (centers) per block
  hipLaunchKernelGGL(k_ball_pass<false>, dim3(wb), dim3(256), 0, s, d_centers, M, g.gp.p, g.keys.p,
                     g.mask, g.cell_start.p, g.counts.p, g.cell_pts.p, row_count.p, nullptr,
                     nullptr);
  TSQBX_HIP(hipGetLastError());
  TSQBX_HIP(scan_exclusive(row_count.p, M, d_offsets, g.scan_tmp.p, s));
  hipLaunchKernelGGL(k_max_row, dim3((unsigned)std::min<int64_t>(1024, (M + 255) / 256)),
                     dim3(256), 0, s, d_offsets, M, maxrow.p);
  TSQBX_HIP(hipGetLastError());
  int64_t total = 0;
  unsigned long long longest = 0;
  TSQBX_HIP(hipMemcpyAsync(&total, d_offsets + M, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TSQBX_HIP(hipMemcpyAsync(&longest, maxrow.p, sizeof(longest), hipMemcpyDeviceToHost, s));
  TSQBX_HIP(hipStreamSynchronize(s));
  *nnz = total;
  if ((int64_t)longest > kRowSortMax)
    return fail(TSQBX_E_RANGE, "a ball holds %llu sources; at most %d per center", longest,
                (int)kRowSortMax);
  if (total > capacity)
    return fail(TSQBX_E_RANGE, "the lists need %lld entries; capacity is %lld", (long long)total,
                (long long)capacity);
  if (total > 0) {
    hipLaunchKernelGGL(k_ball_pass<true>, dim3(wb), dim3(256), 0, s, d_centers, M, g.gp.p,
                       g.keys.p, g.mask, g.cell_start.p, g.counts.p, g.cell_pts.p, nullptr,
                       d_offsets, d_indices);
    TSQBX_HIP(hipGetLastError());
    TSQBX_HIP(sort_rows(d_offsets, d_indices, M, (int64_t)longest, N - 1, s));
  }
  TSQBX_HIP(hipStreamSynchronize(s));
  return TSQBX_OK;
}

extern "C" int tsqbx_knn_lists(tsqbx_ctx *ctx, int64_t n_sources, const double *d_sources,
                               int64_t n_centers, const double *d_centers, const int32_t *d_counts,
                               int64_t *d_offsets, int32_t *d_indices, int64_t capacity,
                               int64_t *nnz, void *hip_stream) {
  TraceRange trace_("tsqbx_knn_lists");
  if (!ctx || !nnz || !d_offsets) return fail(TSQBX_E_INVALID, "ctx, offsets or nnz is NULL");
  if (n_sources < 0 || n_centers < 0 || capacity < 0)
    return fail(TSQBX_E_INVALID, "negative count");
  if (n_sources >= TSQBX_MAX_SOURCES)
    return fail(TSQBX_E_RANGE, "n_sources = %lld; at most %lld", (long long)n_sources,
                (long long)TSQBX_MAX_SOURCES - 1);
  if (n_centers > INT32_MAX) return fail(TSQBX_E_RANGE, "n_centers must stay below 2^31");
  if ((n_sources > 0 && !d_sources) || (n_centers > 0 && (!d_centers || !d_counts)) ||
      (capacity > 0 && !d_indices))
    return fail(TSQBX_E_INVALID, "sources, centers, counts or indices is NULL");
  *nnz = 0;
  int prev = -1;
  (void)hipGetDevice(&prev);
  if (prev != ctx->device) TSQBX_HIP(hipSetDevice(ctx->device));
  RestoreDevice restore{prev};
  hipStream_t s = (hipStream_t)hip_stream;
  const int64_t N = n_sources, M = n_centers;
  if (M == 0) {
    TSQBX_HIP(hipMemsetAsync(d_offsets, 0, sizeof(int64_t), s));
    TSQBX_HIP(hipStreamSynchronize(s));
    return TSQBX_OK;
  }
  // the counts: 0 <= k <= min(N, kRowSortMax)
  DevBuf<int> range;
  TSQBX_HIP(range.alloc(3));
  const int init[3] = {INT32_MAX, INT32_MIN, 0};
  TSQBX_HIP(hipMemcpyAsync(range.p, init, sizeof(init), hipMemcpyHostToDevice, s));
  hipLaunchKernelGGL(k_count_range, dim3((unsigned)std::min<int64_t>(1024, (M + 255) / 256)),
                     dim3(256), 0, s, d_counts, M, range.p);
  TSQBX_HIP(hipGetLastError());
  int got[2] = {0, 0};
  TSQBX_HIP(hipMemcpyAsync(got, range.p, sizeof(got), hipMemcpyDeviceToHost, s));
  TSQBX_HIP(hipStreamSynchronize(s));
  if (got[0] < 0) return fail(TSQBX_E_RANGE, "a count is negative (%d)", got[0]);
  if ((int64_t)got[1] > N)
    return fail(TSQBX_E_RANGE, "a count (%d) exceeds n_sources = %lld", got[1], (long long)N);
  if (got[1] > kRowSortMax)
    return fail(TSQBX_E_RANGE, "a count (%d) exceeds %d per center", got[1], (int)kRowSortMax);
  Grid g;
  if (got[1] > 0) TSQBX_HIP(build_grid(g, N, d_sources, M, d_centers, 0.0, M, s));
  else TSQBX_HIP(g.scan_tmp.alloc((size_t)(M / kScanBlock + 2)));
  TSQBX_HIP(scan_exclusive(d_counts, M, d_offsets, g.scan_tmp.p, s));
  int64_t total = 0;
  TSQBX_HIP(hipMemcpyAsync(&total, d_offsets + M, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TSQBX_HIP(hipStreamSynchronize(s));
  *nnz = total;
  if (total > capacity)
    return fail(TSQBX_E_RANGE, "the lists need %lld entries; capacity is %lld", (long long)total,
                (long long)capacity);
  if (total > 0) {
    hipLaunchKernelGGL(k_knn, dim3((unsigned)M), dim3(256), 0, s, d_centers, d_counts, d_offsets,
                       g.gp.p, g.keys.p, g.mask, g.cell_start.p, g.counts.p, g.cell_pts.p,
                       d_indices, range.p + 2);
    TSQBX_HIP(hipGetLastError());
    TSQBX_HIP(sort_rows(d_offsets, d_indices, M, (int64_t)got[1], N - 1, s));
    int bad = 0;
    TSQBX_HIP(hipMemcpyAsync(&bad, range.p + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    TSQBX_HIP(hipStreamSynchronize(s));
    if (bad) return fail(TSQBX_E_DEVICE, "nearest-neighbour selection did not close");
  }
  TSQBX_HIP(hipStreamSynchronize(s));
  return TSQBX_OK;
}
