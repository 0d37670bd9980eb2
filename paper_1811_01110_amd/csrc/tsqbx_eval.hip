// The evaluation kernel of the plain path (one launch per evaluation, a
// group of G lanes per target) and its launch helpers.  The per-target
// device routines are in tsqbx_device.h.
#include <algorithm>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

template <int P, int L, int G, int U>
__global__ void __launch_bounds__(512)
k_eval(const TargetRec *__restrict__ tgt, const double4 *__restrict__ tnrm, int64_t n_targets,
       const int32_t *__restrict__ idx, SrcView src, double *__restrict__ out_s,
       double *__restrict__ out_d, double *__restrict__ out_t, int accumulate, int p_rt,
       int remap) {
  constexpr int TPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int blk = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  int64_t t = ((int64_t)blk * wpb + wave) * TPW + lane / G;
  if constexpr (G == 64) t = __builtin_amdgcn_readfirstlane((int)t);
  if (t >= n_targets) return;
  const TargetRec tr = tgt[t];
  double v[3];
  target_sum<P, L, G, U, G == 64>(p_rt, lane % G, tr, tnrm + t, idx, src, v);
  if (lane % G == 0) store_out<L>(tr, v, out_s, out_d, out_t, accumulate);
}

// ---- launch helpers -----------------------------------------------------------
template <int P, int L, int G, int U>
hipError_t launch_one(const tsqbx_geometry *g, int p, const SourceStage &st, const Outputs &o,
                      bool acc, const Tuning &tn, hipStream_t s) {
  constexpr int TPW = 64 / G;
  const int64_t per_block = (int64_t)tn.waves_per_block * TPW;
  const int64_t blocks = (g->n_targets + per_block - 1) / per_block;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const SrcView src{st.xy, st.zq, st.nxy, st.nz};
  hipLaunchKernelGGL((k_eval<P, L, G, U>), dim3((unsigned)blocks), dim3(64 * tn.waves_per_block),
                     0, s, g->tgt, g->tgt_nrm, g->n_targets, g->idx, src, o.s, o.d, o.t,
                     acc ? 1 : 0, p, tn.xcd_remap);
  return hipGetLastError();
}

template <int L, int G, int U>
hipError_t launch_p(const tsqbx_geometry *g, int p, const SourceStage &st, const Outputs &o,
                    bool acc, const Tuning &tn, hipStream_t s) {
  switch (p) {
    case 4: return launch_one<4, L, G, U>(g, p, st, o, acc, tn, s);
    case 8: return launch_one<8, L, G, U>(g, p, st, o, acc, tn, s);
    case 12: return launch_one<12, L, G, U>(g, p, st, o, acc, tn, s);
    case 16: return launch_one<16, L, G, U>(g, p, st, o, acc, tn, s);
    case 24: return launch_one<24, L, G, U>(g, p, st, o, acc, tn, s);
    default: return launch_one<-1, L, G, U>(g, p, st, o, acc, tn, s);
  }
}

template <int G, int U>
hipError_t launch_l(const tsqbx_geometry *g, int p, unsigned layers, const SourceStage &st,
                    const Outputs &o, bool acc, const Tuning &tn, hipStream_t s) {
  switch (layers) {
    case 1: return launch_p<1, G, U>(g, p, st, o, acc, tn, s);
    case 2: return launch_p<2, G, U>(g, p, st, o, acc, tn, s);
    case 3: return launch_p<3, G, U>(g, p, st, o, acc, tn, s);
    case 4: return launch_p<4, G, U>(g, p, st, o, acc, tn, s);
    case 5: return launch_p<5, G, U>(g, p, st, o, acc, tn, s);
    case 6: return launch_p<6, G, U>(g, p, st, o, acc, tn, s);
    case 7: return launch_p<7, G, U>(g, p, st, o, acc, tn, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

static bool group_supported(const Tuning &tn) {
  if (!(tn.xcd_remap == 0 || tn.xcd_remap == 1)) return false;
  const int G = tn.group_lanes, U = tn.unroll;
  return (G == 64 && (U == 1 || U == 2 || U == 4)) || (G == 32 && U == 2) || (G == 16 && U == 2);
}

bool tuning_supported(const Tuning &tn) {
  const int w = tn.waves_per_block;
  return (w == 1 || w == 2 || w == 4) && group_supported(tn);
}

bool eval_tuning_supported(const Tuning &tn) {
  const int w = tn.waves_per_block;
  return (w == 1 || w == 2 || w == 4 || w == 8) && group_supported(tn);
}

hipError_t launch_eval(const tsqbx_geometry *g, int p, unsigned layers, const SourceStage &st,
                       const Outputs &o, bool accumulate, const Tuning &tn, hipStream_t s) {
  if (!eval_tuning_supported(tn)) return hipErrorInvalidValue;
  const int G = tn.group_lanes, U = tn.unroll;
  if (G == 64 && U == 1) return launch_l<64, 1>(g, p, layers, st, o, accumulate, tn, s);
  if (G == 64 && U == 2) return launch_l<64, 2>(g, p, layers, st, o, accumulate, tn, s);
  if (G == 64 && U == 4) return launch_l<64, 4>(g, p, layers, st, o, accumulate, tn, s);
  if (G == 32 && U == 2) return launch_l<32, 2>(g, p, layers, st, o, accumulate, tn, s);
  return launch_l<16, 2>(g, p, layers, st, o, accumulate, tn, s);
}

}  // namespace tsqbx
