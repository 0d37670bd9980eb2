// The plain path for geometries whose targets share centers: one wave per
// row (a center and its list) walks the list once for several of the row's
// targets (four at a time, then two; two at a time where rows hold fewer
// than 3.5 targets on average), so each source record is gathered once per
// walk and the source's offset from the center, its distance and 1/R are
// formed once.  Each target's terms are the same operations in the same
// order as in the one-target-per-wave kernel (lane l adds the entries l,
// l + 64, ... of the list, then the same butterfly), so the results equal
// that kernel's bit for bit.
#include <algorithm>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

// The terms of one source for K targets of one center: pair_terms with the
// source held and the target varying (same expressions, per target).
template <int P, int L, int K>
__device__ __forceinline__ void source_terms(int p_rt, uint32_t s, const SrcView &src,
                                             const TargetGeom (&tg)[K], double (&acc_s)[K],
                                             double (&acc_d)[K], double (&acc_t)[K]) {
  const double2 a = load2(src.xy, s);
  const double2 aq = load2(src.zq, s);
  double2 b = make_double2(0.0, 0.0);
  double bz = 0.0;
  if constexpr (L & 2) {
    b = load2(src.nxy, s);
    bz = load1(src.nz, s);
  }
  const int p = P >= 0 ? P : p_rt;
  // the center is the row's: the same for every target
  const double dx = a.x - tg[0].cx;
  const double dy = a.y - tg[0].cy;
  const double dz = aq.x - tg[0].cz;
  const double R2 = fma(dz, dz, fma(dy, dy, dx * dx));
  const double rinv = rsqrt_nr(R2);
  const double inv = rinv * rinv;
  PairState<K> st;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double dd = fma(tg[k].tz, dz, fma(tg[k].ty, dy, tg[k].tx * dx));
    st.beta[k] = dd * inv;
    st.g2[k] = tg[k].rho2 * inv;
  }
  if constexpr (L == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      st.fm1[k] = 0.0;
      st.f[k] = 0.0;
    }
    if constexpr (P >= 0)
      slp_clenshaw<P, K, P>(st);
    else
      slp_clenshaw_rt<K>(p, st);
    constexpr double kap1 = kap_c(1);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double S = p >= 1 ? fma(st.beta[k], st.f[k], fma(-st.g2[k], kap1 * st.fm1[k], 1.0))
                              : 1.0;
      acc_s[k] = fma(aq.y * rinv, S, acc_s[k]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      st.fm1[k] = p >= 1 ? 1.0 : 0.0;
      st.f[k] = p >= 1 ? st.beta[k] : 1.0;
      st.S[k] = p >= 2 ? fma(3.0, st.beta[k], 1.0) : (p == 1 ? 1.0 : 0.0);
    }
    if constexpr (P >= 0)
      dlp_steps<P, K, 2>(st);
    else
      dlp_steps_rt<K>(p, st);
    const double mu_p1 = P >= 0 ? mu_c(P + 1) : d_coef.mu[p + 1];
    const double mu_p = P >= 0 ? (P >= 1 ? mu_c(P) : 0.0) : (p >= 1 ? d_coef.mu[p] : 0.0);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double S2 = st.S[k];
      const double Ep1 = mu_p1 * st.f[k];
      const double Ep = mu_p * st.fm1[k];
      if constexpr (L & 1) {
        const double w = fma(-2.0, st.beta[k], 1.0 + st.g2[k]);
        const double S0 = fma(w, S2, fma(-st.g2[k], Ep, Ep1));
        acc_s[k] = fma(aq.y * rinv, S0, acc_s[k]);
      }
      if constexpr (L & 2) {
        const double nd = fma(bz, dz, fma(b.y, dy, b.x * dx));
        const double nt = fma(bz, tg[k].tz, fma(b.y, tg[k].ty, b.x * tg[k].tx));
        const double val = fma(nt, S2, -nd * (S2 + Ep1));
        acc_d[k] = fma(val, rinv * inv, acc_d[k]);
      }
      if constexpr (L & 4) {
        const double ndt = fma(tg[k].nz, dz, fma(tg[k].ny, dy, tg[k].nx * dx));
        const double vt = fma(ndt, S2, -tg[k].ntd * (S2 - Ep));
        acc_t[k] = fma(aq.y * (rinv * inv), vt, acc_t[k]);
      }
    }
  }
}

template <int L>
__device__ __forceinline__ TargetGeom geom_of(const TargetRec &tr, const double4 *tn) {
  TargetGeom tg;
  tg.cx = tr.c[0];
  tg.cy = tr.c[1];
  tg.cz = tr.c[2];
  tg.tx = tr.d[0];
  tg.ty = tr.d[1];
  tg.tz = tr.d[2];
  tg.rho2 = fma(tg.tz, tg.tz, fma(tg.ty, tg.ty, tg.tx * tg.tx));
  tg.nx = tg.ny = tg.nz = tg.ntd = 0.0;
  if constexpr (L & 4) {
    tg.nx = tn->x;
    tg.ny = tn->y;
    tg.nz = tn->z;
    tg.ntd = fma(tg.nz, tg.tz, fma(tg.ny, tg.ty, tg.nx * tg.tx));
  }
  return tg;
}

// K targets of one row (all with the row's row_begin): lane gl adds the
// entries gl, gl + 64, ... (the next entry's index loaded a step ahead),
// then the 64 lanes' sums are folded by the butterfly of target_sum.
template <int P, int L, int K>
__device__ __forceinline__ void row_sumK(int p_rt, int gl, const TargetRec (&tr)[K],
                                         const double4 *tnrm, const int (&t)[K],
                                         const int32_t *__restrict__ idx, const SrcView &src,
                                         double (&out)[K][3]) {
  constexpr int G = 64;
  TargetGeom tg[K];
#pragma unroll
  for (int k = 0; k < K; ++k) tg[k] = geom_of<L>(tr[k], tnrm + t[k]);
  const int32_t *__restrict__ row = idx + tr[0].row_begin;
  const int len = tr[0].row_len;
  double acc_s[K], acc_d[K], acc_t[K];
#pragma unroll
  for (int k = 0; k < K; ++k) acc_s[k] = acc_d[k] = acc_t[k] = 0.0;
  const int full = len - len % G;
  int c0 = 0;
  uint32_t s = 0;
  if (full > 0) s = load_idx(row, (uint32_t)gl);
  for (; c0 < full; c0 += G) {
    const uint32_t sn = load_idx(row, (uint32_t)min(c0 + G + gl, len - 1));
    source_terms<P, L, K>(p_rt, s, src, tg, acc_s, acc_d, acc_t);
    s = sn;
  }
  if (c0 + gl < len) source_terms<P, L, K>(p_rt, load_idx(row, (uint32_t)(c0 + gl)), src, tg,
                                           acc_s, acc_d, acc_t);
#pragma unroll
  for (int k = 0; k < K; ++k) {
#pragma unroll
    for (int off = G / 2; off >= 1; off >>= 1) {
      if constexpr (L & 1) acc_s[k] += __shfl_xor(acc_s[k], off, 64);
      if constexpr (L & 2) acc_d[k] += __shfl_xor(acc_d[k], off, 64);
      if constexpr (L & 4) acc_t[k] += __shfl_xor(acc_t[k], off, 64);
    }
    out[k][0] = acc_s[k] * kInv4Pi;
    out[k][1] = acc_d[k] * kInv4Pi;
    out[k][2] = acc_t[k] * kInv4Pi;
  }
}

// The row's targets first + k .. first + k + K - 1: sums and stores.
template <int P, int L, int K>
__device__ __forceinline__ void do_group(int p_rt, int lane, int first, int k,
                                         const int32_t *__restrict__ row_tgts,
                                         const TargetRec *__restrict__ tgt,
                                         const double4 *__restrict__ tnrm,
                                         const int32_t *__restrict__ idx, const SrcView &src,
                                         double *out_s, double *out_d, double *out_t,
                                         int accumulate) {
  int t[K];
  TargetRec tr[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    t[j] = __builtin_amdgcn_readfirstlane(row_tgts[first + k + j]);
    tr[j] = tgt[t[j]];
  }
  double v[K][3];
  row_sumK<P, L, K>(p_rt, lane, tr, tnrm, t, idx, src, v);
  if (lane == 0)
#pragma unroll
    for (int j = 0; j < K; ++j) store_out<L>(tr[j], v[j], out_s, out_d, out_t, accumulate);
}

// One wave per row; its targets four at a time (KMAX = 4), then two, and a
// last odd one through the one-target routine.  The four-target walk takes
// more VGPRs (half the waves per SIMD), so rows of two or three targets run
// the KMAX = 2 kernel.
template <int P, int L, int KMAX>
__global__ void __launch_bounds__(512)
k_eval_rows(const CenterRec *__restrict__ ctr, int64_t n_rows, const int32_t *__restrict__ row_tgts,
            const TargetRec *__restrict__ tgt, const double4 *__restrict__ tnrm,
            const int32_t *__restrict__ idx, SrcView src, double *__restrict__ out_s,
            double *__restrict__ out_d, double *__restrict__ out_t, int accumulate, int p_rt,
            int remap) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int blk = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  const int64_t r = __builtin_amdgcn_readfirstlane((int)((int64_t)blk * wpb + wave));
  if (r >= n_rows) return;
  const int first = __builtin_amdgcn_readfirstlane(ctr[r].tgt_begin);
  const int count = __builtin_amdgcn_readfirstlane(ctr[r].tgt_count);
  int k = 0;
  if constexpr (KMAX >= 4)
    for (; k + 3 < count; k += 4)
      do_group<P, L, 4>(p_rt, lane, first, k, row_tgts, tgt, tnrm, idx, src, out_s, out_d, out_t,
                        accumulate);
  for (; k + 1 < count; k += 2)
    do_group<P, L, 2>(p_rt, lane, first, k, row_tgts, tgt, tnrm, idx, src, out_s, out_d, out_t,
                      accumulate);
  if (k < count) {
    const int t0 = __builtin_amdgcn_readfirstlane(row_tgts[first + k]);
    const TargetRec tr = tgt[t0];
    double v[3];
    target_sum<P, L, 64, 2, true>(p_rt, lane, tr, tnrm + t0, idx, src, v);
    if (lane == 0) store_out<L>(tr, v, out_s, out_d, out_t, accumulate);
  }
}

template <int P, int L>
hipError_t launch_rows_one(const tsqbx_geometry *g, int p, const SourceStage &st,
                           const Outputs &o, bool acc, const Tuning &tn, hipStream_t s) {
  const int64_t blocks = (g->n_rows + tn.waves_per_block - 1) / tn.waves_per_block;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  const SrcView src{st.xy, st.zq, st.nxy, st.nz};
  // four targets per walk where rows hold 3.5 or more on average
  if (2 * g->n_targets >= 7 * g->n_rows)
    hipLaunchKernelGGL((k_eval_rows<P, L, 4>), dim3((unsigned)blocks),
                       dim3(64 * tn.waves_per_block), 0, s, g->ctr, g->n_rows, g->row_tgts, g->tgt,
                       g->tgt_nrm, g->idx, src, o.s, o.d, o.t, acc ? 1 : 0, p, tn.xcd_remap);
  else
    hipLaunchKernelGGL((k_eval_rows<P, L, 2>), dim3((unsigned)blocks),
                       dim3(64 * tn.waves_per_block), 0, s, g->ctr, g->n_rows, g->row_tgts, g->tgt,
                       g->tgt_nrm, g->idx, src, o.s, o.d, o.t, acc ? 1 : 0, p, tn.xcd_remap);
  return hipGetLastError();
}

template <int L>
hipError_t launch_rows_p(const tsqbx_geometry *g, int p, const SourceStage &st, const Outputs &o,
                         bool acc, const Tuning &tn, hipStream_t s) {
  switch (p) {
    case 4: return launch_rows_one<4, L>(g, p, st, o, acc, tn, s);
    case 8: return launch_rows_one<8, L>(g, p, st, o, acc, tn, s);
    case 12: return launch_rows_one<12, L>(g, p, st, o, acc, tn, s);
    case 16: return launch_rows_one<16, L>(g, p, st, o, acc, tn, s);
    case 24: return launch_rows_one<24, L>(g, p, st, o, acc, tn, s);
    default: return launch_rows_one<-1, L>(g, p, st, o, acc, tn, s);
  }
}

}  // namespace

bool rows_kernel_pays(const tsqbx_geometry *g, const Tuning &tn) {
  // one wave per target group, on average 1.5 targets or more per row, and
  // at most 16 in any row: a wave takes a whole row, so a row with many more
  // targets than the others would hold one wave while the GPU idles
  return tn.group_lanes == 64 && g->n_rows > 0 && 2 * g->n_targets >= 3 * g->n_rows &&
         g->max_row_targets <= 16;
}

hipError_t launch_eval_plain(const tsqbx_geometry *g, int p, unsigned layers,
                             const SourceStage &st, const Outputs &o, bool accumulate,
                             const Tuning &tn, bool per_target, hipStream_t s) {
  if (per_target || !rows_kernel_pays(g, tn)) return launch_eval(g, p, layers, st, o, accumulate, tn, s);
  if (!eval_tuning_supported(tn)) return hipErrorInvalidValue;
  switch (layers) {
    case 1: return launch_rows_p<1>(g, p, st, o, accumulate, tn, s);
    case 2: return launch_rows_p<2>(g, p, st, o, accumulate, tn, s);
    case 3: return launch_rows_p<3>(g, p, st, o, accumulate, tn, s);
    case 4: return launch_rows_p<4>(g, p, st, o, accumulate, tn, s);
    case 5: return launch_rows_p<5>(g, p, st, o, accumulate, tn, s);
    case 6: return launch_rows_p<6>(g, p, st, o, accumulate, tn, s);
    case 7: return launch_rows_p<7>(g, p, st, o, accumulate, tn, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tsqbx
