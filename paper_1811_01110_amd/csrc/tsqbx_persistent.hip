// The persistent kernel of the batched and served paths: resident waves
// work through a static schedule of units (runs of consecutive targets of
// one item), each target summed by the same device routine as the plain path.
#include <algorithm>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

// ---- persistent batched kernel ---------------------------------------------
// A unit is a run of
// consecutive targets of one item; p and the layer mask are wave-uniform.
// The single layer alone always takes the table-driven Clenshaw loop here:
// the unit loop around it leaves no registers for unrolled constants.
template <int P, int L, int G, int U>
__device__ __forceinline__ void unit_body(const WorkItem &it, int first, int count, int lane) {
  constexpr int TPW = 64 / G;
  const TSQBX_GLOBAL TargetRec *tgt = (const TSQBX_GLOBAL TargetRec *)it.tgt;
  const TSQBX_GLOBAL double4 *tnrm = (const TSQBX_GLOBAL double4 *)it.tnrm;
  for (int k = 0; k < count; k += TPW) {
    int slot = k + lane / G;
    if constexpr (G == 64) slot = __builtin_amdgcn_readfirstlane(slot);
    if (slot >= count) break;  // whole groups leave together
    const TargetRec tr = load_target(tgt + first + slot);
    double v[3];
    const SrcView src{it.xy, it.zq, it.nxy, it.nz};
    target_sum<P, L, G, U, false>(it.p, lane % G, tr, tnrm + first + slot, it.idx, src, v);
    if (lane % G == 0)
      store_out<L>(tr, v, (TSQBX_GLOBAL double *)it.out_s, (TSQBX_GLOBAL double *)it.out_d,
                   (TSQBX_GLOBAL double *)it.out_t, it.accumulate);
  }
}

// PF >= 0: every item has order PF.  PF < 0: switch over the compiled
// orders, with the remaining orders on the run-time loop (one pair in flight,
// which keeps the kernel's register budget that of the compiled orders).
template <int L, int PF, int G, int U>
__device__ __forceinline__ void unit_dispatch_p(const WorkItem &it, int first, int count,
                                                int lane) {
  if constexpr (PF >= 0) {
    unit_body<PF, L, G, U>(it, first, count, lane);
  } else {
    switch (it.p) {
      case 4: unit_body<4, L, G, U>(it, first, count, lane); break;
      case 8: unit_body<8, L, G, U>(it, first, count, lane); break;
      case 12: unit_body<12, L, G, U>(it, first, count, lane); break;
      case 16: unit_body<16, L, G, U>(it, first, count, lane); break;
      case 24: unit_body<24, L, G, U>(it, first, count, lane); break;
      default: unit_body<-1, L, G, 1>(it, first, count, lane); break;
    }
  }
}

// LC = layer class: 1, 2 or 3 (every item has that mask), kLayersSingle
// (masks 1 and 2), kLayersMixed (any of masks 1..3) or kLayersAny (any mask,
// S' included).
// Each wave works through its own range of units (a static schedule built
// on the host), so no wave waits on another and no atomics are needed.
template <int LC, int PF, int G, int U>
__global__ void __launch_bounds__(256) k_persistent(PersistentArgs a) {
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int w = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * wpb +
                                               (int)(threadIdx.x >> 6));
  if (w >= a.n_waves) return;
  const TSQBX_GLOBAL int32_t *wb = (const TSQBX_GLOBAL int32_t *)a.wave_begin;
  const int ub = wb[w], ue = wb[w + 1];
  const TSQBX_GLOBAL WorkUnit *units = (const TSQBX_GLOBAL WorkUnit *)a.units;
  const TSQBX_GLOBAL WorkItem *items = (const TSQBX_GLOBAL WorkItem *)a.items;
  for (int u = ub; u < ue; ++u) {
    const int item = __builtin_amdgcn_readfirstlane(units[u].item);
    const int first = __builtin_amdgcn_readfirstlane(units[u].first);
    const int count = __builtin_amdgcn_readfirstlane(units[u].count);
    WorkItem it;
    it.tgt = items[item].tgt;
    it.idx = items[item].idx;
    it.xy = items[item].xy;
    it.zq = items[item].zq;
    it.nxy = items[item].nxy;
    it.nz = items[item].nz;
    it.out_s = items[item].out_s;
    it.out_d = items[item].out_d;
    it.p = items[item].p;
    it.layers = items[item].layers;
    it.accumulate = items[item].accumulate;
    it.tnrm = items[item].tnrm;
    it.out_t = items[item].out_t;
    if constexpr (LC == kLayersSingle) {
      if (it.layers == 1)
        unit_dispatch_p<1, PF, G, U>(it, first, count, lane);
      else
        unit_dispatch_p<2, PF, G, U>(it, first, count, lane);
    } else if constexpr (LC == kLayersMixed) {
      switch (it.layers) {
        case 1: unit_dispatch_p<1, PF, G, U>(it, first, count, lane); break;
        case 2: unit_dispatch_p<2, PF, G, U>(it, first, count, lane); break;
        default: unit_dispatch_p<3, PF, G, U>(it, first, count, lane); break;
      }
    } else if constexpr (LC == kLayersAny) {
      switch (it.layers) {
        case 1: unit_dispatch_p<1, PF, G, U>(it, first, count, lane); break;
        case 2: unit_dispatch_p<2, PF, G, U>(it, first, count, lane); break;
        case 3: unit_dispatch_p<3, PF, G, U>(it, first, count, lane); break;
        case 4: unit_dispatch_p<4, PF, G, U>(it, first, count, lane); break;
        case 5: unit_dispatch_p<5, PF, G, U>(it, first, count, lane); break;
        case 6: unit_dispatch_p<6, PF, G, U>(it, first, count, lane); break;
        default: unit_dispatch_p<7, PF, G, U>(it, first, count, lane); break;
      }
    } else {
      unit_dispatch_p<LC, PF, G, U>(it, first, count, lane);
    }
  }
}


}  // namespace

int persistent_max_waves(int num_cus, int oversub) {
  // oversub times the waves that fit at six per SIMD: the dispatcher hands
  // out blocks as others finish, which evens out differences in speed
  return std::max(1, num_cus) * 4 * 6 * std::max(1, oversub);
}

namespace {
template <int LC, int PF>
hipError_t launch_persistent_lp(const PersistentArgs &a, const Tuning &tn, hipStream_t s) {
  const dim3 block(64 * tn.waves_per_block);
  const int grid = (a.n_waves + tn.waves_per_block - 1) / tn.waves_per_block;
  const int G = tn.group_lanes, U = tn.unroll;
  if (G == 64 && U == 1)
    hipLaunchKernelGGL((k_persistent<LC, PF, 64, 1>), dim3(grid), block, 0, s, a);
  else if (G == 64)
    hipLaunchKernelGGL((k_persistent<LC, PF, 64, 2>), dim3(grid), block, 0, s, a);
  else if (G == 32)
    hipLaunchKernelGGL((k_persistent<LC, PF, 32, 2>), dim3(grid), block, 0, s, a);
  else
    hipLaunchKernelGGL((k_persistent<LC, PF, 16, 2>), dim3(grid), block, 0, s, a);
  return hipGetLastError();
}

template <int LC>
hipError_t launch_persistent_l(const PersistentArgs &a, int p_all, const Tuning &tn,
                               hipStream_t s) {
  switch (p_all) {
    case 4: return launch_persistent_lp<LC, 4>(a, tn, s);
    case 8: return launch_persistent_lp<LC, 8>(a, tn, s);
    case 12: return launch_persistent_lp<LC, 12>(a, tn, s);
    case 16: return launch_persistent_lp<LC, 16>(a, tn, s);
    case 24: return launch_persistent_lp<LC, 24>(a, tn, s);
    default: return launch_persistent_lp<LC, -1>(a, tn, s);
  }
}
}  // namespace

hipError_t launch_persistent(const PersistentArgs &a, unsigned layer_class, int p_all,
                             const Tuning &tn, hipStream_t s) {
  if (!tuning_supported(tn) || a.n_waves <= 0) return hipErrorInvalidValue;
  switch (layer_class) {
    case 1: return launch_persistent_l<1>(a, p_all, tn, s);
    case 2: return launch_persistent_l<2>(a, p_all, tn, s);
    case 3: return launch_persistent_l<3>(a, p_all, tn, s);
    case kLayersMixed: return launch_persistent_l<kLayersMixed>(a, p_all, tn, s);
    case kLayersSingle: return launch_persistent_l<kLayersSingle>(a, p_all, tn, s);
    default: return launch_persistent_l<kLayersAny>(a, p_all, tn, s);
  }
}

}  // namespace tsqbx
