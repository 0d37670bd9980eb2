// Device routines shared by the kernels of libtsqbx.so (tsqbx_eval.hip,
// tsqbx_stage.hip, tsqbx_persistent.hip): target-specific QBX near-field sums
// for gfx950 (CDNA4), FP64 on the vector ALUs.  Everything here has internal linkage,
// so each kernel file compiles its own copy.
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
// (the second line is App. A's gradient with P_n' written through E_n), and
// S', the target normal derivative of the single layer (App. A, gradient
// with respect to t, dotted with the target normal nu_t):
//   nu_t . grad_t G^(p) = (1/(4 pi |d|^3)) [ (nu_t.d) sum_{n<=p} E_n
//                                            - (nu_t.delta) sum_{n<p} E_n ].
// The last line follows from grad_delta (rho^n P_n) = rho^(n-1) P_n' d/|d|
// - rho^(n-2) P_{n-1}' delta, which is App. A's target gradient after
// x P_n' - n P_n = P_{n-1}'.
// Bonnet's recurrence times (|delta|/|d|)^(n+1) gives
//   (n+1) b_{n+1} = (2n+1) beta b_n - n g2 b_{n-1},
// and the derivative recurrence n P_{n+1}' = (2n+1) x P_n' - (n+1) P_{n-1}'
//   n E_{n+1} = (2n+1) beta E_n - (n+1) g2 E_{n-1}.
// Both are rescaled by per-order constants.  The single layer alone sums the
// b_n by Clenshaw's backward recurrence: a multiply and two FMAs per order.
// When the double layer or S' is requested only the E_n are generated
// forward (two multiplies and one FMA per order, plus one FMA for their
// running sum), and the sums of b_n and (n+1) b_n follow in closed form (see
// pair_terms), so all three layers together cost one recurrence.
//
// 1/|d| comes from v_rsq_f64 and a second-order correction.  Sums within a
// target run in a fixed order (lane-strided over the list, then a fixed
// xor-butterfly across the lanes of the group), so a target's result depends
// only on its list and the group width.
#pragma once

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
  double2 clen[TSQBX_P_MAX + 3];  // (lam_k, kap_{k+1}): one Clenshaw step's pair
};
constexpr CoefTable make_coef_table() {
  CoefTable t{};
  for (int n = 0; n < TSQBX_P_MAX + 3; ++n) {
    t.lam[n] = lam_c(n);
    t.kap[n] = n >= 1 ? kap_c(n) : 0.0;
    t.mu[n] = mu_c(n);
    t.kapd[n] = n >= 2 ? kapd_c(n) : 0.0;
    t.clen[n] = double2{lam_c(n), kap_c(n + 1)};
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

// Single layer only, by Clenshaw's backward recurrence for
// S = sum_{n=0..p} lam_n e_n with e_{n+1} = beta e_n - kap_n g2 e_{n-1},
// e_0 = 1, e_1 = beta:
//   c_k = lam_k + beta c_{k+1} - kap_{k+1} g2 c_{k+2}  (k = p..1, c_{p+1} = c_{p+2} = 0),
//   S = 1 + beta c_1 - kap_1 g2 c_2.
// One order costs a multiply and two FMAs (the sum needs no accumulator).
// On entry (fm1, f) = (c_{K+2}, c_{K+1}); after K = 1 they hold (c_2, c_1).
// This fully unrolled form keeps the constants in registers; the run-time
// form below reads them from a table.  The first two steps meet zeros, which
// the run-time form passes through exactly, so both give the same values.
template <int P, int U, int K>
__device__ __forceinline__ void slp_clenshaw(PairState<U> &st) {
  if constexpr (K >= 1) {
    constexpr double lam = lam_c(K);
    constexpr double kap = kap_c(K + 1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      double ck;
      if constexpr (K == P)
        ck = lam;
      else if constexpr (K == P - 1)
        ck = fma(st.beta[u], st.f[u], lam);
      else
        ck = fma(st.beta[u], st.f[u], fma(-st.g2[u], kap * st.fm1[u], lam));
      st.fm1[u] = st.f[u];
      st.f[u] = ck;
    }
    slp_clenshaw<P, U, K - 1>(st);
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

// The same recurrences for a run-time order p (constants from the table).
template <int U>
__device__ __forceinline__ void clenshaw_step(const double2 c, PairState<U> &st) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double ck = fma(st.beta[u], st.f[u], fma(-st.g2[u], c.y * st.fm1[u], c.x));
    st.fm1[u] = st.f[u];
    st.f[u] = ck;
  }
}

template <int U>
__device__ __forceinline__ void slp_clenshaw_rt(int p, PairState<U> &st) {
  // two steps per iteration, each step's constants read with one scalar load
  // an iteration ahead: they stay out of vector registers (which would cost
  // occupancy) and their latency hides behind the previous steps
  if (p < 1) return;
  int k = p;
  double2 c0 = d_coef.clen[k];
  double2 c1 = d_coef.clen[k - 1];  // k - 1 >= 0: entry 0 exists
#pragma unroll 1
  for (; k >= 3; k -= 2) {
    const double2 n0 = d_coef.clen[k - 2];
    const double2 n1 = d_coef.clen[k - 3];
    clenshaw_step<U>(c0, st);
    clenshaw_step<U>(c1, st);
    c0 = n0;
    c1 = n1;
  }
  if (k >= 1) clenshaw_step<U>(c0, st);
  if (k >= 2) clenshaw_step<U>(c1, st);
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

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// Element i of a staging array (byte offsets stay within 32 bits: a geometry
// holds fewer than 2^27 sources).
__device__ __forceinline__ double2 load2(const double2 *__restrict__ base, uint32_t i) {
  const TSQBX_GLOBAL char *b = (const TSQBX_GLOBAL char *)base;
  const f64x2 v = *(const TSQBX_GLOBAL f64x2 *)(b + (size_t)(i * 16u));
  return make_double2(v.x, v.y);
}
__device__ __forceinline__ double load1(const double *__restrict__ base, uint32_t i) {
  const TSQBX_GLOBAL char *b = (const TSQBX_GLOBAL char *)base;
  return *(const TSQBX_GLOBAL double *)(b + (size_t)(i * 8u));
}

// The staged sources of one evaluation as the pair loops read them (the
// arrays of SourceStage).
struct SrcView {
  const double2 *xy;   // (x, y)
  const double2 *zq;   // (z, q)
  const double2 *nxy;  // (q nx, q ny), double layer
  const double *nz;    // q nz, double layer
};

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

// Per-target values the pair loop reads: the center c, delta = t - c,
// |delta|^2 and, for S', the target normal nu_t and nu_t . delta.
struct TargetGeom {
  double cx, cy, cz;
  double tx, ty, tz;
  double rho2;
  double nx, ny, nz;
  double ntd;
};

// U pairs of one target, added to acc_s / acc_d / acc_t in the order
// u = 0..U-1.  Sources come from the staged arrays at indices s[u]
// (q = w sigma and q nu).  The sums leave out the factor 1/(4 pi).
//
// Single layer alone: S = sum_n b_n by Clenshaw's backward recurrence.
// With the double layer or S', only the derivative terms E_n = (|delta|/R)^{n-1}
// P_n'(x) are generated, by the three-term recurrence
//   n P_{n+1}' = (2n+1) x P_n' - (n+1) P_{n-1}',
// giving S2 = sum_{n<=p} E_n, E_p and E_{p+1}.  Summing
// P_{n+1}' = x P_n' + (n+1) P_n and P_{n+1}' - P_{n-1}' = (2n+1) P_n over
// n = 0..p yields, without division,
//   sum_n (n+1) b_n = (1 - beta) S2 + E_{p+1}
//   sum_n b_n       = (1 - 2 beta + g2) S2 + E_{p+1} - g2 E_p,
// the double layer bracket becomes (nu.delta) S2 - (nu.d)(S2 + E_{p+1}) and
// the S' bracket (nu_t.d) S2 - (nu_t.delta)(S2 - E_p).
// UNROLLED_SLP: the single layer alone uses the fully unrolled Clenshaw steps
// (constants in registers) instead of the table-driven loop; the plain kernel
// sets it for one target per wave, where the registers are available.
template <int P, int L, int U, bool UNROLLED_SLP>
__device__ __forceinline__ void pair_terms(int p_rt, const uint32_t (&s)[U], const SrcView &src,
                                           const TargetGeom &tg, double &acc_s, double &acc_d,
                                           double &acc_t) {
  double2 a[U], aq[U], b[U];
  double bz[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    a[u] = load2(src.xy, s[u]);
    aq[u] = load2(src.zq, s[u]);
  }
  if constexpr (L & 2) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      b[u] = load2(src.nxy, s[u]);
      bz[u] = load1(src.nz, s[u]);
    }
  }
  const int p = P >= 0 ? P : p_rt;
  PairState<U> st;
  double dx[U], dy[U], dz[U], rinv[U], inv[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    dx[u] = a[u].x - tg.cx;
    dy[u] = a[u].y - tg.cy;
    dz[u] = aq[u].x - tg.cz;
    const double R2 = fma(dz[u], dz[u], fma(dy[u], dy[u], dx[u] * dx[u]));
    const double dd = fma(tg.tz, dz[u], fma(tg.ty, dy[u], tg.tx * dx[u]));
    rinv[u] = rsqrt_nr(R2);
    inv[u] = rinv[u] * rinv[u];
    st.beta[u] = dd * inv[u];
    st.g2[u] = tg.rho2 * inv[u];
  }
  if constexpr (L == 1) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      st.fm1[u] = 0.0;
      st.f[u] = 0.0;
    }
    if constexpr (P >= 0 && UNROLLED_SLP)
      slp_clenshaw<P, U, P>(st);
    else
      slp_clenshaw_rt<U>(p, st);
    constexpr double kap1 = kap_c(1);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double S = p >= 1 ? fma(st.beta[u], st.f[u], fma(-st.g2[u], kap1 * st.fm1[u], 1.0))
                              : 1.0;
      acc_s = fma(aq[u].y * rinv[u], S, acc_s);
    }
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
      const double Ep = mu_p * st.fm1[u];
      if constexpr (L & 1) {
        const double w = fma(-2.0, st.beta[u], 1.0 + st.g2[u]);
        const double S0 = fma(w, S2, fma(-st.g2[u], Ep, Ep1));
        acc_s = fma(aq[u].y * rinv[u], S0, acc_s);
      }
      if constexpr (L & 2) {
        const double nd = fma(bz[u], dz[u], fma(b[u].y, dy[u], b[u].x * dx[u]));
        const double nt = fma(bz[u], tg.tz, fma(b[u].y, tg.ty, b[u].x * tg.tx));
        const double val = fma(nt, S2, -nd * (S2 + Ep1));
        acc_d = fma(val, rinv[u] * inv[u], acc_d);
      }
      if constexpr (L & 4) {
        const double ndt = fma(tg.nz, dz[u], fma(tg.ny, dy[u], tg.nx * dx[u]));
        const double vt = fma(ndt, S2, -tg.ntd * (S2 - Ep));
        acc_t = fma(aq[u].y * (rinv[u] * inv[u]), vt, acc_t);
      }
    }
  }
}

// Sum over one target's list by the G lanes of its group (lane gl of G).
// Lane gl takes the entries gl, gl + G, gl + 2G, ... in list order and adds
// them in that order: U at a time over the full chunks of G*U entries, then
// one at a time over the rest.  The chunk loop's bounds are the same for the
// whole group, so only the tail runs with idle lanes.  tn is the target's
// normal (read for S' only).
template <int P, int L, int G, int U, bool UNROLLED_SLP, class NrmPtr>
__device__ __forceinline__ void target_sum(int p_rt, int gl, const TargetRec &tr, NrmPtr tn,
                                           const int32_t *__restrict__ idx, const SrcView &src,
                                           double (&out)[3]) {
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
  const int32_t *__restrict__ row = idx + tr.row_begin;
  const int len = tr.row_len;
  double acc_s = 0.0, acc_d = 0.0, acc_t = 0.0;
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
      pair_terms<P, L, U, UNROLLED_SLP>(p_rt, s, src, tg, acc_s, acc_d, acc_t);
#pragma unroll
      for (int u = 0; u < U; ++u) s[u] = sn[u];
    }
  }
  for (; c0 < len; c0 += G) {
    const int j = c0 + gl;
    if (j < len) {
      const uint32_t s1[1] = {load_idx(row, (uint32_t)j)};
      pair_terms<P, L, 1, UNROLLED_SLP>(p_rt, s1, src, tg, acc_s, acc_d, acc_t);
    }
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1) {
    if constexpr (L & 1) acc_s += __shfl_xor(acc_s, off, 64);
    if constexpr (L & 2) acc_d += __shfl_xor(acc_d, off, 64);
    if constexpr (L & 4) acc_t += __shfl_xor(acc_t, off, 64);
  }
  out[0] = acc_s * kInv4Pi;
  out[1] = acc_d * kInv4Pi;
  out[2] = acc_t * kInv4Pi;
}

template <int L, class Ptr>
__device__ __forceinline__ void store_out(const TargetRec &tr, const double (&v)[3], Ptr out_s,
                                          Ptr out_d, Ptr out_t, int accumulate) {
  const int o = tr.out_index;
  if constexpr (L & 1) out_s[o] = accumulate ? out_s[o] + v[0] : v[0];
  if constexpr (L & 2) out_d[o] = accumulate ? out_d[o] + v[1] : v[1];
  if constexpr (L & 4) out_t[o] = accumulate ? out_t[o] + v[2] : v[2];
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

}  // namespace
}  // namespace tsqbx
