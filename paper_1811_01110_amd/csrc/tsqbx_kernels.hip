// Device code of libtsqbx.so: target-specific QBX near-field kernels for
// gfx950 (CDNA4), FP64 on the vector ALUs.
//
// Per pair (target t, center c, listed source y) the kernels evaluate the
// p-th order target-specific expansion of App. A,
//   G^(p)(t, y) = 1/(4 pi) sum_{n=0..p} |t-c|^n / |y-c|^{n+1} P_n(cos gamma),
// and the double-layer kernel nu . grad_y G^(p), through a scaled form of
// Bonnet's recurrence that needs no division and no angle:
//
//   d = y - c, delta = t - c, R^2 = d.d, beta = delta.d / R^2, g2 = |delta|^2 / R^2
//   b_n = (|delta|/R)^n P_n(cos gamma):  b_0 = 1, b_1 = beta,
//   (n+1) b_{n+1} = (2n+1) beta b_n - n g2 b_{n-1}
//
// (Bonnet's (n+1)P_{n+1} = (2n+1)xP_n - nP_{n-1} times (|delta|/R)^{n+1}),
// so that G^(p) = (1/(4 pi R)) sum_n b_n.  Writing b_n = lam_n e_n with
// lam_{n+1} = lam_n (2n+1)/(n+1) leaves
//   e_{n+1} = beta e_n - kap_n g2 e_{n-1},  kap_n = (n/(n+1)) lam_{n-1}/lam_{n+1},
// two multiplies and one FMA per order, plus one FMA for the sum.
//
// Double layer (App. A, gradient with respect to the source): with
// E_n = R |delta|^{n-1} P_n'(x) / R^n, the derivative recurrence
// P_{n+1}' = x P_n' + (n+1) P_n becomes E_{n+1} = beta E_n + (n+1) b_n, and
//   nu . grad_y G^(p) = (1/(4 pi R^3)) [ -(nu.d) S1 + (nu.delta - beta nu.d) S2 ],
//   S1 = sum_{n<=p} (n+1) b_n = (1 - beta) S2 + E_{p+1},  S2 = sum_{n<=p} E_n.
// (The identity for S1 follows from summing the E recurrence.)
//
// 1/R comes from v_rsq_f64 refined by two Newton-Raphson steps on x^{-1/2}.
// Sums within a target run in a fixed order (lane-strided over the list,
// then a fixed xor-butterfly across the lanes of the group), so a target's
// result depends only on its list and the group width.
#include "tsqbx_internal.h"

namespace tsqbx {
namespace {

constexpr double kInv4Pi = 1.0 / (4.0 * 3.14159265358979323846);

// ---- recurrence constants (compile-time; a __constant__ copy serves the
// runtime-order kernels, with identical values) ------------------------------
constexpr double lam_c(int n) {
  double l = 1.0;
  for (int k = 1; k <= n; ++k) l = l * double(2 * k - 1) / double(k);
  return l;
}
constexpr double kap_c(int n) { return (double(n) / double(n + 1)) * lam_c(n - 1) / lam_c(n + 1); }
constexpr double cn_c(int n) { return double(n + 1) * lam_c(n); }

struct CoefTable {
  double lam[TSQBX_P_MAX + 2];
  double kap[TSQBX_P_MAX + 2];
  double cn[TSQBX_P_MAX + 2];
};
constexpr CoefTable make_coef_table() {
  CoefTable t{};
  for (int n = 0; n < TSQBX_P_MAX + 2; ++n) {
    t.lam[n] = lam_c(n);
    t.kap[n] = n >= 1 ? kap_c(n) : 0.0;
    t.cn[n] = cn_c(n);
  }
  return t;
}
__constant__ CoefTable d_coef = make_coef_table();

// 1/sqrt(x) for normal x > 0: hardware estimate, then two Newton-Raphson
// steps y <- y (3 - x y^2)/2; the second in residual form for ~1 ulp.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double hx = 0.5 * x;
  y = y * fma(-hx, y * y, 1.5);
  double e = x * y;
  double h = fma(-e, y, 1.0);
  return fma(0.5 * y, h, y);
}

// Orders 1..P-1 of the scaled recurrence, fully unrolled.
template <int P, int L, int N>
__device__ __forceinline__ void legendre_steps(double beta, double g2, double em1, double e,
                                               double &S0, double &E, double &S2) {
  if constexpr (N < P) {
    constexpr double kap = kap_c(N);
    constexpr double lam1 = lam_c(N + 1);
    constexpr double c1 = cn_c(N + 1);
    double en1 = fma(-kap, g2 * em1, beta * e);
    if constexpr (L & 1) S0 = fma(lam1, en1, S0);
    if constexpr (L & 2) {
      S2 = S2 + E;
      E = fma(beta, E, c1 * en1);
    }
    legendre_steps<P, L, N + 1>(beta, g2, e, en1, S0, E, S2);
  }
}

// The same orders for a run-time p (constants from the table).
template <int L>
__device__ __forceinline__ void legendre_steps_rt(int p, double beta, double g2, double em1,
                                                  double e, double &S0, double &E, double &S2) {
  for (int n = 1; n < p; ++n) {
    double en1 = fma(-d_coef.kap[n], g2 * em1, beta * e);
    if constexpr (L & 1) S0 = fma(d_coef.lam[n + 1], en1, S0);
    if constexpr (L & 2) {
      S2 = S2 + E;
      E = fma(beta, E, d_coef.cn[n + 1] * en1);
    }
    em1 = e;
    e = en1;
  }
}

// One pair.  (dx, dy, dz) = y - c; (tx, ty, tz) = t - c; rho2 = |t - c|^2;
// q = w sigma; (nx, ny, nz) = q nu.  cs, cd: contributions without 1/(4 pi).
template <int P, int L>
__device__ __forceinline__ void pair_terms(int p_rt, double dx, double dy, double dz, double tx,
                                           double ty, double tz, double rho2, double q, double nx,
                                           double ny, double nz, double &cs, double &cd) {
  double R2 = fma(dz, dz, fma(dy, dy, dx * dx));
  double dd = fma(tz, dz, fma(ty, dy, tx * dx));
  double rinv = rsqrt_nr(R2);
  double inv = rinv * rinv;
  double beta = dd * inv;
  double g2 = rho2 * inv;
  const int p = P >= 0 ? P : p_rt;
  double S0 = 1.0;  // sum_n lam_n e_n
  double S2 = 0.0;  // sum_{n<=order} E_n
  double E = 1.0;   // E_{order+1}
  if (p >= 1) {
    S0 = 1.0 + beta;
    S2 = 1.0;
    E = 3.0 * beta;
    if constexpr (P >= 0)
      legendre_steps<P, L, 1>(beta, g2, 1.0, beta, S0, E, S2);
    else
      legendre_steps_rt<L>(p, beta, g2, 1.0, beta, S0, E, S2);
  }
  if constexpr (L & 1) cs = (q * rinv) * S0;
  if constexpr (L & 2) {
    double S1 = fma(1.0 - beta, S2, E);
    double nd = fma(nz, dz, fma(ny, dy, nx * dx));
    double nt = fma(nz, tz, fma(ny, ty, nx * tx));
    double br = fma(-nd, beta, nt);
    double val = fma(br, S2, -nd * S1);
    cd = val * (rinv * inv);
  }
}

// Sum over one target's list by the G lanes of its group (lane gl of G),
// U independent pairs in flight per lane, accumulated in list order.
template <int P, int L, int G, int U>
__device__ __forceinline__ void target_sum(int p_rt, int gl, const TargetRec &tr,
                                           const int32_t *__restrict__ idx,
                                           const double4 *__restrict__ posq,
                                           const double4 *__restrict__ qn, double &out_s,
                                           double &out_d) {
  const double cx = tr.c[0], cy = tr.c[1], cz = tr.c[2];
  const double tx = tr.d[0], ty = tr.d[1], tz = tr.d[2];
  const double rho2 = fma(tz, tz, fma(ty, ty, tx * tx));
  const int32_t *row = idx + tr.row_begin;
  const int len = tr.row_len;
  double acc_s = 0.0, acc_d = 0.0;
  for (int j0 = gl; j0 < len; j0 += G * U) {
    double cs[U], cd[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int j = j0 + u * G;
      ok[u] = j < len;
      int s = row[ok[u] ? j : j0];
      double4 a = posq[s];
      double4 b = make_double4(0.0, 0.0, 0.0, 0.0);
      if constexpr (L & 2) b = qn[s];
      pair_terms<P, L>(p_rt, a.x - cx, a.y - cy, a.z - cz, tx, ty, tz, rho2, a.w, b.x, b.y, b.z,
                       cs[u], cd[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (L & 1) acc_s += ok[u] ? cs[u] : 0.0;
      if constexpr (L & 2) acc_d += ok[u] ? cd[u] : 0.0;
    }
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    if constexpr (L & 1) acc_s += __shfl_xor(acc_s, off, 64);
    if constexpr (L & 2) acc_d += __shfl_xor(acc_d, off, 64);
  }
  out_s = acc_s * kInv4Pi;
  out_d = acc_d * kInv4Pi;
}

template <int L>
__device__ __forceinline__ void store_out(const TargetRec &tr, double vs, double vd,
                                          double *__restrict__ out_s, double *__restrict__ out_d,
                                          int accumulate) {
  const int o = tr.out_index;
  if constexpr (L & 1) out_s[o] = accumulate ? out_s[o] + vs : vs;
  if constexpr (L & 2) out_d[o] = accumulate ? out_d[o] + vd : vd;
}

// Blocks are dealt to the 8 XCDs round-robin; renumber them so that each XCD
// works through one contiguous range of (Morton-ordered) targets and its L2
// holds one region of the source array.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int xcd = b % X, local = b / X;
  const int per = nb / X, rem = nb % X;
  return xcd * per + min(xcd, rem) + local;
}

template <int P, int L, int G, int U>
__global__ void __launch_bounds__(1024)
k_eval(const TargetRec *__restrict__ tgt, int64_t n_targets, const int32_t *__restrict__ idx,
       const double4 *__restrict__ posq, const double4 *__restrict__ qn,
       double *__restrict__ out_s, double *__restrict__ out_d, int accumulate, int p_rt,
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
  double vs = 0.0, vd = 0.0;
  target_sum<P, L, G, U>(p_rt, lane % G, tr, idx, posq, qn, vs, vd);
  if (lane % G == 0) store_out<L>(tr, vs, vd, out_s, out_d, accumulate);
}

// Staging: q = w sigma in device source order, and q nu for the double layer.
__global__ void __launch_bounds__(256)
k_stage(int64_t n, const double4 *__restrict__ pos_w, const double4 *__restrict__ nrm,
        const int64_t *__restrict__ perm, const double *__restrict__ sigma,
        double4 *__restrict__ posq, double4 *__restrict__ qn, int want_dlp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double4 a = pos_w[i];
    const double q = a.w * sigma[perm ? perm[i] : i];
    posq[i] = make_double4(a.x, a.y, a.z, q);
    if (want_dlp) {
      const double4 v = nrm[i];
      qn[i] = make_double4(q * v.x, q * v.y, q * v.z, 0.0);
    }
  }
}

// ---- persistent batched kernel ---------------------------------------------
// Each wave takes work units from a global ticket counter until none remain
// (every wave reaches the exit: tickets only grow).  A unit is a run of
// consecutive targets of one item; p and the layer mask are wave-uniform.
template <int P, int L, int G, int U>
__device__ __forceinline__ void unit_body(const WorkItem &it, int first, int count, int lane) {
  constexpr int TPW = 64 / G;
  for (int k = 0; k < count; k += TPW) {
    const int slot = k + lane / G;
    if (slot >= count) break;  // whole groups leave together
    const TargetRec tr = it.tgt[first + slot];
    double vs = 0.0, vd = 0.0;
    target_sum<P, L, G, U>(it.p, lane % G, tr, it.idx, it.posq, it.qn, vs, vd);
    if (lane % G == 0) store_out<L>(tr, vs, vd, it.out_s, it.out_d, it.accumulate);
  }
}

template <int L, int G, int U>
__device__ __forceinline__ void unit_dispatch_p(const WorkItem &it, int first, int count,
                                                int lane) {
  switch (it.p) {
    case 4: unit_body<4, L, G, U>(it, first, count, lane); break;
    case 8: unit_body<8, L, G, U>(it, first, count, lane); break;
    case 12: unit_body<12, L, G, U>(it, first, count, lane); break;
    case 16: unit_body<16, L, G, U>(it, first, count, lane); break;
    case 24: unit_body<24, L, G, U>(it, first, count, lane); break;
    default: unit_body<-1, L, G, U>(it, first, count, lane); break;
  }
}

template <int G, int U>
__global__ void __launch_bounds__(1024) k_persistent(PersistentArgs a) {
  const int lane = threadIdx.x & 63;
  for (;;) {
    unsigned int u = 0;
    if (lane == 0) u = atomicAdd(a.ticket, 1u);
    u = __builtin_amdgcn_readfirstlane(__shfl(u, 0, 64));
    if ((int64_t)u >= a.n_units) break;
    const WorkUnit wu = a.units[u];
    const WorkItem it = a.items[wu.item];
    switch (it.layers) {
      case 1: unit_dispatch_p<1, G, U>(it, wu.first, wu.count, lane); break;
      case 2: unit_dispatch_p<2, G, U>(it, wu.first, wu.count, lane); break;
      default: unit_dispatch_p<3, G, U>(it, wu.first, wu.count, lane); break;
    }
  }
}

__global__ void k_reset(unsigned int *ticket) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *ticket = 0u;
}

// ---- launch helpers -----------------------------------------------------------
template <int P, int L, int G, int U>
hipError_t launch_one(const tsqbx_geometry *g, int p, const SourceStage &st, double *out_s,
                      double *out_d, bool acc, const Tuning &tn, hipStream_t s) {
  constexpr int TPW = 64 / G;
  const int64_t per_block = (int64_t)tn.waves_per_block * TPW;
  const int64_t blocks = (g->n_targets + per_block - 1) / per_block;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_eval<P, L, G, U>), dim3((unsigned)blocks), dim3(64 * tn.waves_per_block),
                     0, s, g->tgt, g->n_targets, g->idx, st.posq, st.qn, out_s, out_d, acc ? 1 : 0,
                     p, tn.xcd_remap);
  return hipGetLastError();
}

template <int L, int G, int U>
hipError_t launch_p(const tsqbx_geometry *g, int p, const SourceStage &st, double *out_s,
                    double *out_d, bool acc, const Tuning &tn, hipStream_t s) {
  switch (p) {
    case 4: return launch_one<4, L, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    case 8: return launch_one<8, L, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    case 12: return launch_one<12, L, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    case 16: return launch_one<16, L, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    case 24: return launch_one<24, L, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    default: return launch_one<-1, L, G, U>(g, p, st, out_s, out_d, acc, tn, s);
  }
}

template <int G, int U>
hipError_t launch_l(const tsqbx_geometry *g, int p, unsigned layers, const SourceStage &st,
                    double *out_s, double *out_d, bool acc, const Tuning &tn, hipStream_t s) {
  switch (layers) {
    case 1: return launch_p<1, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    case 2: return launch_p<2, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    case 3: return launch_p<3, G, U>(g, p, st, out_s, out_d, acc, tn, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool tuning_supported(const Tuning &tn) {
  const int w = tn.waves_per_block;
  if (!(w == 1 || w == 2 || w == 4 || w == 8 || w == 16)) return false;
  if (!(tn.xcd_remap == 0 || tn.xcd_remap == 1)) return false;
  const int G = tn.group_lanes, U = tn.unroll;
  return (G == 64 && (U == 1 || U == 2 || U == 4)) || (G == 32 && U == 2) || (G == 16 && U == 2);
}

hipError_t launch_eval(const tsqbx_geometry *g, int p, unsigned layers, const SourceStage &st,
                       double *out_s, double *out_d, bool accumulate, const Tuning &tn,
                       hipStream_t s) {
  if (!tuning_supported(tn)) return hipErrorInvalidValue;
  const int G = tn.group_lanes, U = tn.unroll;
  if (G == 64 && U == 1) return launch_l<64, 1>(g, p, layers, st, out_s, out_d, accumulate, tn, s);
  if (G == 64 && U == 2) return launch_l<64, 2>(g, p, layers, st, out_s, out_d, accumulate, tn, s);
  if (G == 64 && U == 4) return launch_l<64, 4>(g, p, layers, st, out_s, out_d, accumulate, tn, s);
  if (G == 32 && U == 2) return launch_l<32, 2>(g, p, layers, st, out_s, out_d, accumulate, tn, s);
  return launch_l<16, 2>(g, p, layers, st, out_s, out_d, accumulate, tn, s);
}

hipError_t launch_stage(const tsqbx_geometry *g, const double *d_sigma, unsigned layers,
                        const SourceStage &st, hipStream_t s) {
  const int64_t n = g->n_sources;
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 65536);
  hipLaunchKernelGGL(k_stage, dim3((unsigned)blocks), dim3(256), 0, s, n, g->src_pos, g->src_nrm,
                     g->src_perm, d_sigma, st.posq, st.qn, (layers & TSQBX_DLP) ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_reset(unsigned int *ticket, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(1), dim3(64), 0, s, ticket);
  return hipGetLastError();
}

int persistent_max_grid(int num_cus, const Tuning &tn) {
  // enough resident waves to cover every SIMD several times over
  const int waves = num_cus * 4 * 6;
  return std::max(1, waves / tn.waves_per_block);
}

hipError_t launch_persistent(const PersistentArgs &a, int grid, const Tuning &tn, hipStream_t s) {
  if (!tuning_supported(tn) || grid <= 0) return hipErrorInvalidValue;
  const dim3 block(64 * tn.waves_per_block);
  const int G = tn.group_lanes, U = tn.unroll;
  if (G == 64 && U == 1)
    hipLaunchKernelGGL((k_persistent<64, 1>), dim3(grid), block, 0, s, a);
  else if (G == 64 && U == 2)
    hipLaunchKernelGGL((k_persistent<64, 2>), dim3(grid), block, 0, s, a);
  else if (G == 64 && U == 4)
    hipLaunchKernelGGL((k_persistent<64, 4>), dim3(grid), block, 0, s, a);
  else if (G == 32 && U == 2)
    hipLaunchKernelGGL((k_persistent<32, 2>), dim3(grid), block, 0, s, a);
  else
    hipLaunchKernelGGL((k_persistent<16, 2>), dim3(grid), block, 0, s, a);
  return hipGetLastError();
}

}  // namespace tsqbx
