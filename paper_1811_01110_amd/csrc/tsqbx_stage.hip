// Staging of the strengths (q = w sigma, and q times the normal for the
// double layer) into the arrays the evaluation kernels gather from, for one
// geometry or for many in one launch, and the multi-item copy kernel of the
// served path.  Staging arrays that persist (a geometry's own, a plan's)
// receive the positions and the padding entry once, when they are made;
// each evaluation then writes only the strengths (q into the second half of
// zq, and the double layer's q-weighted normals), a third to a half of the
// bytes of a full staging.  Staging arrays made per request (the served
// path, the caller-free scratch) are staged in full.
#include <algorithm>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

// Staging of one source: (x, y), (z, q) with q = w sigma and, for the double
// layer, (q nx, q ny) and q nz, at device index j; pw holds (x, y, z, w) and
// nv (nx, ny, nz, 0) per source, w the weights alone.  Full: positions too;
// else the strengths only.
template <bool Full, class PR, class PD>
__device__ __forceinline__ void stage_one(int64_t j, PR pw, PR w, PR nv, double sg, PD xy, PD zq,
                                          PD nxy, PD nz, int want_dlp) {
  const double q = (Full ? pw[4 * j + 3] : w[j]) * sg;
  if (Full) {
    xy[2 * j] = pw[4 * j];
    xy[2 * j + 1] = pw[4 * j + 1];
    zq[2 * j] = pw[4 * j + 2];
  }
  zq[2 * j + 1] = q;
  if (want_dlp) {
    nxy[2 * j] = q * nv[4 * j];
    nxy[2 * j + 1] = q * nv[4 * j + 1];
    nz[j] = q * nv[4 * j + 2];
  }
}

// Entry n, the padding record: finite and far from every center, q = 0, so
// a padded list entry contributes exactly zero.
template <class PD>
__device__ __forceinline__ void stage_pad(int64_t n, PD xy, PD zq, PD nxy, PD nz, int want_dlp) {
  xy[2 * n] = 1e100;
  xy[2 * n + 1] = 1e100;
  zq[2 * n] = 1e100;
  zq[2 * n + 1] = 0.0;
  if (want_dlp) {
    nxy[2 * n] = 0.0;
    nxy[2 * n + 1] = 0.0;
    nz[n] = 0.0;
  }
}

// Staging in device source order (the padding entry too when Full).
template <bool Full>
__global__ void __launch_bounds__(256)
k_stage(int64_t n, const double4 *__restrict__ pos_w, const double *__restrict__ w_dev,
        const double4 *__restrict__ nrm, const int64_t *__restrict__ perm,
        const double *__restrict__ sigma, double2 *xy2, double2 *zq2, double2 *nxy2, double *nz,
        int want_dlp) {
  typedef TSQBX_GLOBAL double *GD;
  typedef const TSQBX_GLOBAL double *GR;
  const GR pw = (GR)pos_w, w = (GR)w_dev, nv = (GR)nrm;
  const GD xy = (GD)xy2, zq = (GD)zq2, nxy = (GD)nxy2, nzg = (GD)nz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {
      if (Full) stage_pad(n, xy, zq, nxy, nzg, want_dlp);
      continue;
    }
    stage_one<Full>(i, pw, w, nv, sigma[perm ? perm[i] : i], xy, zq, nxy, nzg, want_dlp);
  }
}

// The positions of persistent staging arrays, q = 0, and the padding entry
// (with the double layer's zeros when nxy is given).
__global__ void __launch_bounds__(256)
k_stage_positions(int64_t n, const double4 *__restrict__ pos_w, double2 *xy2, double2 *zq2,
                  double2 *nxy2, double *nz) {
  typedef TSQBX_GLOBAL double *GD;
  typedef const TSQBX_GLOBAL double *GR;
  const GR pw = (GR)pos_w;
  const GD xy = (GD)xy2, zq = (GD)zq2, nxy = (GD)nxy2, nzg = (GD)nz;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {
      stage_pad(n, xy, zq, nxy, nzg, nxy2 != nullptr);
      continue;
    }
    xy[2 * i] = pw[4 * i];
    xy[2 * i + 1] = pw[4 * i + 1];
    zq[2 * i] = pw[4 * i + 2];
    zq[2 * i + 1] = 0.0;
  }
}

// The same staging for many items in one launch.  The items' elements lie
// end to end, each item starting at a multiple of kStageBlock (begin), and
// block b takes elements [b kStageBlock, (b + 1) kStageBlock) of the one
// item they fall in (one per thread), found by a binary search on the block
// index (uniform across the block, so its loads are scalar).  A density in
// device memory is gathered while walking the sources in device order; a
// density in pinned host memory is read contiguously, walking the sources in
// the caller's order, since every read then crosses PCIe.
__global__ void __launch_bounds__(256) k_stage_multi(const StageItem *__restrict__ items,
                                                     int n_items) {
  typedef TSQBX_GLOBAL double *GD;
  typedef const TSQBX_GLOBAL double *GR;
  const TSQBX_GLOBAL StageItem *all = (const TSQBX_GLOBAL StageItem *)items;
  const int64_t base = (int64_t)blockIdx.x * kStageBlock;
  int lo = 0, hi = n_items - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (all[mid].begin <= base) lo = mid;
    else hi = mid - 1;
  }
  const TSQBX_GLOBAL StageItem *gi = all + lo;
  const int64_t n = gi->n;
  const int want_dlp = gi->want_dlp;
  const int host_sigma = gi->host_sigma;
  const int full = !gi->strengths_only;
  const GR pw = (GR)gi->pos_w;  // (x, y, z, w)
  const GR w = (GR)gi->w;       // w alone
  const GR nv = (GR)gi->nrm;    // (nx, ny, nz, 0)
  const TSQBX_GLOBAL int32_t *rank = (const TSQBX_GLOBAL int32_t *)gi->order;
  const TSQBX_GLOBAL int64_t *perm = (const TSQBX_GLOBAL int64_t *)gi->order;
  const double *sigma = gi->sigma;  // device or pinned host memory
  const GD xy = (GD)gi->xy, zq = (GD)gi->zq, nxy = (GD)gi->nxy, nz = (GD)gi->nz;
  const int64_t i = base - gi->begin + threadIdx.x;  // one source per thread
  if (i > n) return;
  if (i == n) {
    if (full) stage_pad(n, xy, zq, nxy, nz, want_dlp);
    return;
  }
  int64_t j;  // device index
  double sg;
  if (host_sigma) {
    j = rank ? (int64_t)rank[i] : i;
    sg = sigma[i];
  } else {
    j = i;
    sg = sigma[perm ? perm[i] : i];
  }
  if (full)
    stage_one<true>(j, pw, w, nv, sg, xy, zq, nxy, nz, want_dlp);
  else
    stage_one<false>(j, pw, w, nv, sg, xy, zq, nxy, nz, want_dlp);
}

// Contiguous copies, blockIdx.y selects the item.
__global__ void __launch_bounds__(256) k_copy_multi(const CopyItem *__restrict__ items) {
  const TSQBX_GLOBAL CopyItem *ci = (const TSQBX_GLOBAL CopyItem *)items + blockIdx.y;
  const int64_t n = ci->n;
  const double *src = ci->src;
  double *dst = ci->dst;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

hipError_t launch_stage(const tsqbx_geometry *g, const double *d_sigma, unsigned layers,
                        const SourceStage &st, bool positions_ready, hipStream_t s) {
  const int64_t n = g->n_sources;
  if (n < 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 1 + 255) / 256, 65536);
  if (positions_ready)
    hipLaunchKernelGGL(k_stage<false>, dim3((unsigned)blocks), dim3(256), 0, s, n, g->src_pos,
                       g->src_w, g->src_nrm, g->src_perm, d_sigma, st.xy, st.zq, st.nxy, st.nz,
                       (layers & TSQBX_DLP) ? 1 : 0);
  else
    hipLaunchKernelGGL(k_stage<true>, dim3((unsigned)blocks), dim3(256), 0, s, n, g->src_pos,
                       g->src_w, g->src_nrm, g->src_perm, d_sigma, st.xy, st.zq, st.nxy, st.nz,
                       (layers & TSQBX_DLP) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_stage_positions(const tsqbx_geometry *g, const SourceStage &st, hipStream_t s) {
  const int64_t n = g->n_sources;
  if (n < 0 || !st.xy) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 1 + 255) / 256, 65536);
  hipLaunchKernelGGL(k_stage_positions, dim3((unsigned)blocks), dim3(256), 0, s, n, g->src_pos,
                     st.xy, st.zq, st.nxy, st.nz);
  return hipGetLastError();
}

StageItem make_stage_item(const tsqbx_geometry *g, const double *sigma, unsigned layers,
                          const SourceStage &st, bool sigma_on_host, bool positions_ready) {
  StageItem it{};
  it.pos_w = g->src_pos;
  it.w = g->src_w;
  it.strengths_only = positions_ready ? 1 : 0;
  it.nrm = g->src_nrm;
  it.host_sigma = sigma_on_host ? 1 : 0;
  it.order = sigma_on_host ? (const void *)g->src_rank : (const void *)g->src_perm;
  it.sigma = sigma;
  it.xy = st.xy;
  it.zq = st.zq;
  it.nxy = st.nxy;
  it.nz = st.nz;
  it.n = g->n_sources;
  it.want_dlp = (layers & TSQBX_DLP) ? 1 : 0;
  return it;
}

int64_t assign_stage_blocks(StageItem *items, int n_items) {
  int64_t at = 0;
  for (int i = 0; i < n_items; ++i) {
    items[i].begin = at;
    at += (items[i].n + 1 + kStageBlock - 1) / kStageBlock * kStageBlock;
  }
  return at;
}

hipError_t launch_stage_multi(const StageItem *d_items, int n_items, int64_t total,
                              hipStream_t s) {
  if (n_items <= 0 || total <= 0) return hipSuccess;
  if (n_items > 65535 || total / kStageBlock > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_stage_multi, dim3((unsigned)(total / kStageBlock)), dim3(kStageBlock), 0, s,
                     d_items, n_items);
  return hipGetLastError();
}


hipError_t launch_copy_multi(const CopyItem *d_items, int n_items, int64_t max_n,
                             hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (n_items > 65535) return hipErrorInvalidValue;
  const int64_t bx = std::min<int64_t>((max_n + 255) / 256, 256);
  hipLaunchKernelGGL(k_copy_multi, dim3((unsigned)std::max<int64_t>(bx, 1), (unsigned)n_items),
                     dim3(256), 0, s, d_items);
  return hipGetLastError();
}

}  // namespace tsqbx
