// Device code of libtsqbx.so: target-specific QBX near-field kernels for
// gfx950 (CDNA4), FP64 on the vector ALUs.
//
// Per pair (target t, center c, listed source y) the kernels evaluate the
// p-th order target-specific expansion of App. A,
//   G^(p)(t, y) = 1/(4 pi) sum_{n=0..p} |t-c|^n / |y-c|^{n+1} P_n(cos gamma),
// and the double-layer kernel nu . grad_y G^(p) (App. A, source gradient),
// through scaled recurrences that need neither the angle nor a division:
//
//   d = y - c, delta = t - c, beta = delta.d / |d|^2, g2 = |delta|^2 / |d|^2,
//   b_n = (|delta|/|d|)^n P_n(cos gamma),  E_n = (|delta|/|d|)^(n-1) P_n'(cos gamma)
//   G^(p) = (1/(4 pi |d|)) sum_n b_n
//   nu . grad_y G^(p) = (1/(4 pi |d|^3)) [ -(nu.d) sum_n (n+1) b_n
//                                          + (nu.delta - beta nu.d) sum_n E_n ]
//
// (the second line is App. A's gradient with P_n' written through E_n).
// Bonnet's recurrence times (|delta|/|d|)^(n+1) gives
//   (n+1) b_{n+1} = (2n+1) beta b_n - n g2 b_{n-1},
// and the derivative recurrence n P_{n+1}' = (2n+1) x P_n' - (n+1) P_{n-1}'
//   n E_{n+1} = (2n+1) beta E_n - (n+1) g2 E_{n-1}.
// Both are rescaled by per-order constants so that one order costs two
// multiplies and one FMA, plus one FMA for the running sum.  When the double
// layer is requested only the E_n are generated; the sums of b_n and
// (n+1) b_n then follow in closed form (see pair_terms), so the single and
// double layer together cost one recurrence.
//
// 1/|d| comes from v_rsq_f64 and a second-order correction.  Sums within a
// target run in a fixed order (lane-strided over the list, then a fixed
// xor-butterfly across the lanes of the group), so a target's result depends
// only on its list and the group width.
#include "tsqbx_internal.h"

namespace tsqbx {
namespace {

constexpr double kInv4Pi = 1.0 / (4.0 * 3.14159265358979323846);

// ---- recurrence constants (compile-time; a __constant__ copy serves the
// runtime-order kernels, with identical values) ------------------------------
// single layer: b_n = lam_n e_n, lam_{n+1} = lam_n (2n+1)/(n+1),
//   e_{n+1} = beta e_n - kap_n g2 e_{n-1},  kap_n = (n/(n+1)) lam_{n-1}/lam_{n+1}
constexpr double lam_c(int n) {
  double l = 1.0;
  for (int k = 1; k <= n; ++k) l = l * double(2 * k - 1) / double(k);
  return l;
}
constexpr double kap_c(int n) { return (double(n) / double(n + 1)) * lam_c(n - 1) / lam_c(n + 1); }
// double layer: E_n = mu_n F_n, mu_1 = 1, mu_{n+1} = mu_n (2n+1)/n,
//   F_{n+1} = beta F_n - kapd_n g2 F_{n-1},  kapd_n = ((n+1)/n) mu_{n-1}/mu_{n+1}
constexpr double mu_c(int n) {
  double m = 1.0;
  for (int k = 1; k < n; ++k) m = m * double(2 * k + 1) / double(k);
  return m;
}
constexpr double kapd_c(int n) { return (double(n + 1) / double(n)) * mu_c(n - 1) / mu_c(n + 1); }

struct CoefTable {
  double lam[TSQBX_P_MAX + 3];
  double kap[TSQBX_P_MAX + 3];
  double mu[TSQBX_P_MAX + 3];
  double kapd[TSQBX_P_MAX + 3];
};
constexpr CoefTable make_coef_table() {
  CoefTable t{};
  for (int n = 0; n < TSQBX_P_MAX + 3; ++n) {
    t.lam[n] = lam_c(n);
    t.kap[n] = n >= 1 ? kap_c(n) : 0.0;
    t.mu[n] = mu_c(n);
    t.kapd[n] = n >= 2 ? kapd_c(n) : 0.0;
  }
  return t;
}
__constant__ CoefTable d_coef = make_coef_table();

// 1/sqrt(x) for normal x > 0: the hardware estimate y0 (relative error about
// 2^-24) corrected by the second-order series of (1 - h)^(-1/2),
// h = 1 - x y0^2: y = y0 (1 + h/2 + 3h^2/8); the dropped term is ~h^3.
__device__ __forceinline__ double rsqrt_nr(double x) {
  const double y0 = __builtin_amdgcn_rsq(x);
  const double h = fma(-(x * y0), y0, 1.0);
  return fma(y0 * h, fma(h, 0.375, 0.5), y0);
}

// State of U independent pairs advanced in lockstep, so that the U
// dependency chains interleave in the instruction stream.
template <int U>
struct PairState {
  double beta[U], g2[U];  // per-pair recurrence coefficients
  double fm1[U], f[U];    // two consecutive scaled terms
  double S[U];            // running sum
};

// Single layer only: e_{n+1} for n = N..P-1 and S += lam_{n+1} e_{n+1}.
template <int P, int U, int N>
__device__ __forceinline__ void slp_steps(PairState<U> &st) {
  if constexpr (N < P) {
    constexpr double kap = kap_c(N);
    constexpr double lam1 = lam_c(N + 1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double en1 = fma(-kap, st.g2[u] * st.fm1[u], st.beta[u] * st.f[u]);
      st.S[u] = fma(lam1, en1, st.S[u]);
      st.fm1[u] = st.f[u];
      st.f[u] = en1;
    }
    slp_steps<P, U, N + 1>(st);
  }
}

// Derivative terms: F_{n+1} for n = N..P and S += mu_{n+1} F_{n+1} while
// n + 1 <= P; leaves (fm1, f) = (F_P, F_{P+1}).
template <int P, int U, int N>
__device__ __forceinline__ void dlp_steps(PairState<U> &st) {
  if constexpr (N <= P) {
    constexpr double kap = kapd_c(N);
    constexpr double mu1 = mu_c(N + 1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double fn1 = fma(-kap, st.g2[u] * st.fm1[u], st.beta[u] * st.f[u]);
      if constexpr (N + 1 <= P) st.S[u] = fma(mu1, fn1, st.S[u]);
      st.fm1[u] = st.f[u];
      st.f[u] = fn1;
    }
    dlp_steps<P, U, N + 1>(st);
  }
}

// The same steps for a run-time order p (constants from the table).
template <int U>
__device__ __forceinline__ void slp_steps_rt(int p, PairState<U> &st) {
  for (int n = 1; n < p; ++n) {
    const double kap = d_coef.kap[n], lam1 = d_coef.lam[n + 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double en1 = fma(-kap, st.g2[u] * st.fm1[u], st.beta[u] * st.f[u]);
      st.S[u] = fma(lam1, en1, st.S[u]);
      st.fm1[u] = st.f[u];
      st.f[u] = en1;
    }
  }
}

template <int U>
__device__ __forceinline__ void dlp_steps_rt(int p, PairState<U> &st) {
  for (int n = 2; n <= p; ++n) {
    const double kap = d_coef.kapd[n], mu1 = d_coef.mu[n + 1];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double fn1 = fma(-kap, st.g2[u] * st.fm1[u], st.beta[u] * st.f[u]);
      if (n + 1 <= p) st.S[u] = fma(mu1, fn1, st.S[u]);
      st.fm1[u] = st.f[u];
      st.f[u] = fn1;
    }
  }
}

// Loads through global-address-space pointers: pointers that reach a kernel
// through a device-side table would otherwise be treated as generic (flat).
#define TSQBX_GLOBAL __attribute__((address_space(1)))

__device__ __forceinline__ uint32_t load_idx(const int32_t *__restrict__ row, uint32_t j) {
  const TSQBX_GLOBAL char *base = (const TSQBX_GLOBAL char *)row;
  return *(const TSQBX_GLOBAL uint32_t *)(base + (size_t)(j * 4u));
}

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double4 load4(const double4 *__restrict__ base, uint32_t i) {
  const TSQBX_GLOBAL char *b = (const TSQBX_GLOBAL char *)base;
  const f64x4 v = *(const TSQBX_GLOBAL f64x4 *)(b + (size_t)(i * 32u));
  return make_double4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ TargetRec load_target(const TSQBX_GLOBAL TargetRec *p) {
  TargetRec t;
  for (int a = 0; a < 3; ++a) {
    t.c[a] = p->c[a];
    t.d[a] = p->d[a];
  }
  t.row_begin = p->row_begin;
  t.row_len = p->row_len;
  t.out_index = p->out_index;
  return t;
}

// U pairs of one target, added to acc_s / acc_d in the order u = 0..U-1.
// Source records come from posq / qn at indices s[u] (q = w sigma and q nu);
// (cx, cy, cz) = c; (tx, ty, tz) = t - c; rho2 = |t - c|^2.  The sums leave
// out the factor 1/(4 pi).
//
// Single layer alone: S = sum_n b_n from the Legendre recurrence.
// With the double layer, only the derivative terms E_n = (|delta|/R)^{n-1}
// P_n'(x) are generated, by the three-term recurrence
//   n P_{n+1}' = (2n+1) x P_n' - (n+1) P_{n-1}',
// giving S2 = sum_{n<=p} E_n, E_p and E_{p+1}.  Summing
// P_{n+1}' = x P_n' + (n+1) P_n and P_{n+1}' - P_{n-1}' = (2n+1) P_n over
// n = 0..p yields, without division,
//   sum_n (n+1) b_n = (1 - beta) S2 + E_{p+1}
//   sum_n b_n       = (1 - 2 beta + g2) S2 + E_{p+1} - g2 E_p,
// and the double layer bracket becomes (nu.delta) S2 - (nu.d)(S2 + E_{p+1}).
template <int P, int L, int U>
__device__ __forceinline__ void pair_terms(int p_rt, const uint32_t (&s)[U],
                                           const double4 *__restrict__ posq,
                                           const double4 *__restrict__ qn, double cx, double cy,
                                           double cz, double tx, double ty, double tz, double rho2,
                                           double &acc_s, double &acc_d) {
  double4 a[U], b[U];
#pragma unroll
  for (int u = 0; u < U; ++u) a[u] = load4(posq, s[u]);
  if constexpr (L & 2) {
#pragma unroll
    for (int u = 0; u < U; ++u) b[u] = load4(qn, s[u]);
  }
  const int p = P >= 0 ? P : p_rt;
  PairState<U> st;
  double dx[U], dy[U], dz[U], rinv[U], inv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    dx[u] = a[u].x - cx;
    dy[u] = a[u].y - cy;
    dz[u] = a[u].z - cz;
    const double R2 = fma(dz[u], dz[u], fma(dy[u], dy[u], dx[u] * dx[u]));
    const double dd = fma(tz, dz[u], fma(ty, dy[u], tx * dx[u]));
    rinv[u] = rsqrt_nr(R2);
    inv[u] = rinv[u] * rinv[u];
    st.beta[u] = dd * inv[u];
    st.g2[u] = rho2 * inv[u];
  }
  if constexpr (L == 1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      st.fm1[u] = 1.0;
      st.f[u] = st.beta[u];
      st.S[u] = p >= 1 ? 1.0 + st.beta[u] : 1.0;
    }
    if constexpr (P >= 0)
      slp_steps<P, U, 1>(st);
    else
      slp_steps_rt<U>(p, st);
#pragma unroll
    for (int u = 0; u < U; ++u) acc_s = fma(a[u].w * rinv[u], st.S[u], acc_s);
  } else {
    // (fm1, f) = (F_0, F_1) for p = 0, else (F_1, F_2) = (1, beta)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      st.fm1[u] = p >= 1 ? 1.0 : 0.0;
      st.f[u] = p >= 1 ? st.beta[u] : 1.0;
      st.S[u] = p >= 2 ? fma(3.0, st.beta[u], 1.0) : (p == 1 ? 1.0 : 0.0);
    }
    if constexpr (P >= 0)
      dlp_steps<P, U, 2>(st);
    else
      dlp_steps_rt<U>(p, st);
    const double mu_p1 = P >= 0 ? mu_c(P + 1) : d_coef.mu[p + 1];
    const double mu_p = P >= 0 ? (P >= 1 ? mu_c(P) : 0.0) : (p >= 1 ? d_coef.mu[p] : 0.0);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double S2 = st.S[u];
      const double Ep1 = mu_p1 * st.f[u];
      if constexpr (L & 1) {
        const double Ep = mu_p * st.fm1[u];
        const double w = fma(-2.0, st.beta[u], 1.0 + st.g2[u]);
        const double S0 = fma(w, S2, fma(-st.g2[u], Ep, Ep1));
        acc_s = fma(a[u].w * rinv[u], S0, acc_s);
      }
      const double nd = fma(b[u].z, dz[u], fma(b[u].y, dy[u], b[u].x * dx[u]));
      const double nt = fma(b[u].z, tz, fma(b[u].y, ty, b[u].x * tx));
      const double val = fma(nt, S2, -nd * (S2 + Ep1));
      acc_d = fma(val, rinv[u] * inv[u], acc_d);
    }
  }
}

// Sum over one target's list by the G lanes of its group (lane gl of G).
// Lane gl takes the entries gl, gl + G, gl + 2G, ... in list order and adds
// them in that order: U at a time over the full chunks of G*U entries, then
// one at a time over the rest.  The chunk loop's bounds are the same for the
// whole group, so only the tail runs with idle lanes.
template <int P, int L, int G, int U>
__device__ __forceinline__ void target_sum(int p_rt, int gl, const TargetRec &tr,
                                           const int32_t *__restrict__ idx,
                                           const double4 *__restrict__ posq,
                                           const double4 *__restrict__ qn, double &out_s,
                                           double &out_d) {
  const double cx = tr.c[0], cy = tr.c[1], cz = tr.c[2];
  const double tx = tr.d[0], ty = tr.d[1], tz = tr.d[2];
  const double rho2 = fma(tz, tz, fma(ty, ty, tx * tx));
  const int32_t *__restrict__ row = idx + tr.row_begin;
  const int len = tr.row_len;
  double acc_s = 0.0, acc_d = 0.0;
  int c0 = 0;
  if constexpr (U > 1) {
    const int full = len - len % (G * U);
    uint32_t s[U];
    if (full > 0) {
#pragma unroll
      for (int u = 0; u < U; ++u) s[u] = load_idx(row, (uint32_t)(gl + u * G));
    }
    for (; c0 < full; c0 += G * U) {
      // indices of the next chunk (clamped into the row; unused past its end)
      uint32_t sn[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        sn[u] = load_idx(row, (uint32_t)min(c0 + G * U + gl + u * G, len - 1));
      pair_terms<P, L, U>(p_rt, s, posq, qn, cx, cy, cz, tx, ty, tz, rho2, acc_s, acc_d);
#pragma unroll
      for (int u = 0; u < U; ++u) s[u] = sn[u];
    }
  }
  for (; c0 < len; c0 += G) {
    const int j = c0 + gl;
    if (j < len) {
      const uint32_t s1[1] = {load_idx(row, (uint32_t)j)};
      pair_terms<P, L, 1>(p_rt, s1, posq, qn, cx, cy, cz, tx, ty, tz, rho2, acc_s, acc_d);
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

template <int L, class Ptr>
__device__ __forceinline__ void store_out(const TargetRec &tr, double vs, double vd, Ptr out_s,
                                          Ptr out_d, int accumulate) {
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
__global__ void __launch_bounds__(256)
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
// Entry n is the padding record: finite and far from every center, q = 0, so
// a padded list entry contributes exactly zero.
__global__ void __launch_bounds__(256)
k_stage(int64_t n, const double4 *__restrict__ pos_w, const double4 *__restrict__ nrm,
        const int64_t *__restrict__ perm, const double *__restrict__ sigma,
        double4 *__restrict__ posq, double4 *__restrict__ qn, int want_dlp) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {
      posq[n] = make_double4(1e100, 1e100, 1e100, 0.0);
      if (want_dlp) qn[n] = make_double4(0.0, 0.0, 0.0, 0.0);
      continue;
    }
    const double4 a = pos_w[i];
    const double q = a.w * sigma[perm ? perm[i] : i];
    posq[i] = make_double4(a.x, a.y, a.z, q);
    if (want_dlp) {
      const double4 v = nrm[i];
      qn[i] = make_double4(q * v.x, q * v.y, q * v.z, 0.0);
    }
  }
}

// The same staging for many items: blockIdx.y selects the item.
// The same staging for many items (blockIdx.y selects the item).  A density
// in device memory is gathered while walking the sources in device order; a
// density in pinned host memory is read contiguously, walking the sources in
// the caller's order, since every read then crosses PCIe.
__global__ void __launch_bounds__(256) k_stage_multi(const StageItem *__restrict__ items) {
  const TSQBX_GLOBAL StageItem *gi = (const TSQBX_GLOBAL StageItem *)items + blockIdx.y;
  const int64_t n = gi->n;
  const int want_dlp = gi->want_dlp;
  const int host_sigma = gi->host_sigma;
  const TSQBX_GLOBAL double *pw = (const TSQBX_GLOBAL double *)gi->pos_w;  // (x, y, z, w)
  const TSQBX_GLOBAL double *nv = (const TSQBX_GLOBAL double *)gi->nrm;    // (nx, ny, nz, 0)
  const TSQBX_GLOBAL int32_t *rank = (const TSQBX_GLOBAL int32_t *)gi->order;
  const TSQBX_GLOBAL int64_t *perm = (const TSQBX_GLOBAL int64_t *)gi->order;
  const double *sigma = gi->sigma;
  TSQBX_GLOBAL double *posq = (TSQBX_GLOBAL double *)gi->posq;
  TSQBX_GLOBAL double *qn = (TSQBX_GLOBAL double *)gi->qn;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == n) {  // the padding record
      posq[4 * n] = 1e100;
      posq[4 * n + 1] = 1e100;
      posq[4 * n + 2] = 1e100;
      posq[4 * n + 3] = 0.0;
      if (want_dlp) {
        qn[4 * n] = 0.0;
        qn[4 * n + 1] = 0.0;
        qn[4 * n + 2] = 0.0;
        qn[4 * n + 3] = 0.0;
      }
      continue;
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
    const double q = pw[4 * j + 3] * sg;
    posq[4 * j] = pw[4 * j];
    posq[4 * j + 1] = pw[4 * j + 1];
    posq[4 * j + 2] = pw[4 * j + 2];
    posq[4 * j + 3] = q;
    if (want_dlp) {
      qn[4 * j] = q * nv[4 * j];
      qn[4 * j + 1] = q * nv[4 * j + 1];
      qn[4 * j + 2] = q * nv[4 * j + 2];
      qn[4 * j + 3] = 0.0;
    }
  }
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

// ---- persistent batched kernel ---------------------------------------------
// A unit is a run of
// consecutive targets of one item; p and the layer mask are wave-uniform.
template <int P, int L, int G, int U>
__device__ __forceinline__ void unit_body(const WorkItem &it, int first, int count, int lane) {
  constexpr int TPW = 64 / G;
  const TSQBX_GLOBAL TargetRec *tgt = (const TSQBX_GLOBAL TargetRec *)it.tgt;
  for (int k = 0; k < count; k += TPW) {
    int slot = k + lane / G;
    if constexpr (G == 64) slot = __builtin_amdgcn_readfirstlane(slot);
    if (slot >= count) break;  // whole groups leave together
    const TargetRec tr = load_target(tgt + first + slot);
    double vs = 0.0, vd = 0.0;
    target_sum<P, L, G, U>(it.p, lane % G, tr, it.idx, it.posq, it.qn, vs, vd);
    if (lane % G == 0)
      store_out<L>(tr, vs, vd, (TSQBX_GLOBAL double *)it.out_s, (TSQBX_GLOBAL double *)it.out_d,
                   it.accumulate);
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

// LC = layer class: 1 or 2 (every item has that mask) or 3 (any mask).
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
    it.posq = items[item].posq;
    it.qn = items[item].qn;
    it.out_s = items[item].out_s;
    it.out_d = items[item].out_d;
    it.p = items[item].p;
    it.layers = items[item].layers;
    it.accumulate = items[item].accumulate;
    if constexpr (LC == 3) {
      switch (it.layers) {
        case 1: unit_dispatch_p<1, PF, G, U>(it, first, count, lane); break;
        case 2: unit_dispatch_p<2, PF, G, U>(it, first, count, lane); break;
        default: unit_dispatch_p<3, PF, G, U>(it, first, count, lane); break;
      }
    } else {
      unit_dispatch_p<LC, PF, G, U>(it, first, count, lane);
    }
  }
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
  if (!(w == 1 || w == 2 || w == 4)) return false;
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
  if (n < 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 1 + 255) / 256, 65536);
  hipLaunchKernelGGL(k_stage, dim3((unsigned)blocks), dim3(256), 0, s, n, g->src_pos, g->src_nrm,
                     g->src_perm, d_sigma, st.posq, st.qn, (layers & TSQBX_DLP) ? 1 : 0);
  return hipGetLastError();
}

StageItem make_stage_item(const tsqbx_geometry *g, const double *sigma, unsigned layers,
                          const SourceStage &st, bool sigma_on_host) {
  StageItem it{};
  it.pos_w = g->src_pos;
  it.nrm = g->src_nrm;
  it.host_sigma = sigma_on_host ? 1 : 0;
  it.order = sigma_on_host ? (const void *)g->src_rank : (const void *)g->src_perm;
  it.sigma = sigma;
  it.posq = st.posq;
  it.qn = st.qn;
  it.n = g->n_sources;
  it.want_dlp = (layers & TSQBX_DLP) ? 1 : 0;
  return it;
}

hipError_t launch_stage_multi(const StageItem *d_items, int n_items, int64_t max_n,
                              hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (n_items > 65535) return hipErrorInvalidValue;
  const int64_t bx = std::min<int64_t>((max_n + 1 + 255) / 256, 1024);
  hipLaunchKernelGGL(k_stage_multi, dim3((unsigned)std::max<int64_t>(bx, 1), (unsigned)n_items),
                     dim3(256), 0, s, d_items);
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

int persistent_max_waves(int num_cus) {
  // eight times the waves that fit at six per SIMD: the dispatcher hands out
  // blocks as others finish, which evens out differences in speed
  return std::max(1, num_cus) * 4 * 6 * 8;
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
    default: return launch_persistent_l<3>(a, p_all, tn, s);
  }
}

}  // namespace tsqbx
