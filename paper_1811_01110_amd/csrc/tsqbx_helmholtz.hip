// Helmholtz target-specific expansions (App. A, Helmholtz case) on gfx950,
// FP64, real wavenumber k > 0 and complex densities:
//
//   G_k^(p)(t, y) = (i k / 4 pi) sum_{n=0..p} (2n+1) j_n(k rho) h_n(k R) P_n(x),
//   nu . grad_y G_k^(p) = (i k / 4 pi) sum_n (2n+1) j_n(k rho) / R
//                          [ k (nu.d) h_n'(k R) P_n(x) + (nu.delta/rho - (nu.d) x / R) h_n(k R) P_n'(x) ],
//   nu_t . grad_t G_k^(p) = (i k / 4 pi) sum_n (2n+1) h_n(k R)
//                          [ (nu_t.delta/rho) k j_n'(k rho) P_n(x)
//                            + (nu_t.d / R - (nu_t.delta/rho) x) (j_n(k rho) / rho) P_n'(x) ],
//
// d = y - c, delta = t - c, R = |d|, rho = |delta|, x = cos gamma (the last
// line is S', App. A's target gradient dotted with the target normal).  The
// j_n(k rho) terms depend on the target only, so a pre-pass (k_helm_table)
// stores (2n+1) j_n(k rho) per target and, for S', (2n+1) k j_n'(k rho) and
// (2n+1) j_n(k rho) / rho (finite at rho = 0); the pair kernel runs three recurrences per
// pair: Bonnet's for P_n (rescaled so that one order costs a multiply and an
// FMA), the upward recurrence h_{n+1} = (2n+1)/z h_n - h_{n-1} for the
// spherical Hankel functions (stable upward, DLMF 10.51.1), and
// P_{n+1}' = x P_n' + (n+1) P_n.  The derivative h_n' = h_{n-1} - (n+1)/z h_n
// (DLMF 10.51.2, with h_{-1} = h_0/z - h_1) turns the double layer's first
// sum into sum m_n h_{n-1} - (1/z) sum (n+1) m_n h_n with m_n = (2n+1) j_n P_n,
// so no h_n' is formed.
//
// Sums within a target run in a fixed order (lane-strided over the list, then
// a fixed xor butterfly), as in the Laplace kernels.
#include <algorithm>
#include <cmath>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

// Per-target table: tab[n] = (2n+1) j_n(k rho), n = 0..p.  For z = k rho > p
// every order is in the oscillatory range where the upward recurrence
// j_{n+1} = (2n+1)/z j_n - j_{n-1} is stable (DLMF 10.51.1).  Otherwise
// Miller's downward recurrence f_{n-1} = (2n+1)/z f_n - f_{n+1} from
// n = p + 32 + z (where the minimal solution dominates), rescaled on the way,
// is normalised by whichever of j_0 = sin z / z and j_1 = sin z / z^2 - cos z / z
// is larger in magnitude (their zeros interlace, so one is well away from 0).
// With tabs (S'), the row of 2 (p + 1) entries after it holds
// (2n+1) k j_n'(z), from j_n' = (n/z) j_n - j_{n+1} (DLMF 10.51.2; no
// cancellation for small z), then (2n+1) j_n(z) / rho = (2n+1) k j_n(z) / z.
// At z = 0 these are their limits: k for n = 1 and 0 otherwise.
__device__ __forceinline__ void helm_table_row(const TargetRec *__restrict__ tgt, int64_t t,
                                               double k, int p, double *__restrict__ tab,
                                               double *__restrict__ tabs) {
  const TargetRec tr = tgt[t];
  const double rho2 = fma(tr.d[2], tr.d[2], fma(tr.d[1], tr.d[1], tr.d[0] * tr.d[0]));
  const double z = k * sqrt(rho2);
  double *row = tab + t * (int64_t)(p + 1);
  double *rows = tabs ? tabs + t * (int64_t)(2 * (p + 1)) : nullptr;
  if (!(z > 0.0)) {
    row[0] = 1.0;
    for (int n = 1; n <= p; ++n) row[n] = 0.0;
    if (rows)
      for (int n = 0; n <= p; ++n) rows[n] = rows[p + 1 + n] = n == 1 ? k : 0.0;
    return;
  }
  const double zinv = 1.0 / z;
  double sn, cs;
  sincos(z, &sn, &cs);
  const double j0 = sn * zinv;
  const double j1 = (j0 - cs) * zinv;
  // row[] first receives j_n (times a common factor `scale` for Miller's
  // recurrence), jp1 the same for j_{p+1}
  double scale = 1.0, jp1;
  if (z > (double)(p + 1)) {
    double jm1 = j0, jn = j1;
    row[0] = j0;
    for (int n = 1; n <= p; ++n) {
      row[n] = jn;
      const double jnext = (double)(2 * n + 1) * zinv * jn - jm1;
      jm1 = jn;
      jn = jnext;
    }
    jp1 = jn;
  } else {
    const int N = p + 32 + (int)z;
    double fp1 = 0.0, f = 1.0e-280;  // f_{n+1}, f_n
    double f0 = 0.0, f1 = 0.0;
    jp1 = 0.0;
    for (int n = N; n >= 1; --n) {
      const double fm1 = (double)(2 * n + 1) * zinv * f - fp1;
      if (n - 1 <= p) row[n - 1] = fm1;
      if (n - 1 == p + 1) jp1 = fm1;
      if (n == 2) f1 = fm1;
      if (n == 1) f0 = fm1;
      fp1 = f;
      f = fm1;
      if (fabs(f) > 1.0e250) {  // rescale everything kept so far
        fp1 *= 1.0e-250;
        f *= 1.0e-250;
        f0 *= 1.0e-250;
        f1 *= 1.0e-250;
        jp1 *= 1.0e-250;
        for (int m = n - 1; m <= p; ++m) row[m] *= 1.0e-250;
      }
    }
    scale = fabs(j0) >= fabs(j1) ? j0 / f0 : j1 / f1;
  }
  for (int n = 0; n <= p; ++n) {
    const double jn = row[n] * scale;
    if (rows) {
      const double jn1 = (n < p ? row[n + 1] : jp1) * scale;
      const double w = (double)(2 * n + 1) * k;
      rows[n] = w * fma((double)n * zinv, jn, -jn1);
      rows[p + 1 + n] = w * (jn * zinv);
    }
    row[n] = (double)(2 * n + 1) * jn;
  }
}

__global__ void __launch_bounds__(256)
k_helm_table(const TargetRec *__restrict__ tgt, int64_t n_targets, double k, int p,
             double *__restrict__ tab, double *__restrict__ tabs) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n_targets) helm_table_row(tgt, t, k, p, tab, tabs);
}

// Staging: rec[2i] = (x, y, z, Re q), rec[2i+1] = (Im q, nu) with q = w sigma
// and sigma complex in the caller's order; entry n is the padding record
// (q = 0, far from every center).
__device__ __forceinline__ void helm_stage_one(int64_t i, int64_t n,
                                               const double4 *__restrict__ pos_w,
                                               const double4 *__restrict__ nrm,
                                               const int64_t *__restrict__ perm,
                                               const double *__restrict__ sigma,
                                               double4 *__restrict__ rec) {
  if (i == n) {
    rec[2 * n] = make_double4(1e100, 1e100, 1e100, 0.0);
    rec[2 * n + 1] = make_double4(0.0, 0.0, 0.0, 0.0);
    return;
  }
  const double4 a = pos_w[i];
  const int64_t c = perm ? perm[i] : i;
  const double sr = sigma[2 * c], si = sigma[2 * c + 1];
  rec[2 * i] = make_double4(a.x, a.y, a.z, a.w * sr);
  const double4 v = nrm ? nrm[i] : make_double4(0.0, 0.0, 0.0, 0.0);
  rec[2 * i + 1] = make_double4(a.w * si, v.x, v.y, v.z);
}

__global__ void __launch_bounds__(256)
k_helm_stage(int64_t n, const double4 *__restrict__ pos_w, const double4 *__restrict__ nrm,
             const int64_t *__restrict__ perm, const double *__restrict__ sigma,
             double4 *__restrict__ rec) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x)
    helm_stage_one(i, n, pos_w, nrm, perm, sigma, rec);
}

// Staging and tables of many evaluations in one launch each: item
// blockIdx.y, its sources (or targets) strided over blockIdx.x.
__global__ void __launch_bounds__(256) k_helm_stage_multi(const HelmPrepItem *__restrict__ items) {
  const HelmPrepItem it = items[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= it.n;
       i += (int64_t)gridDim.x * blockDim.x)
    helm_stage_one(i, it.n, it.pos_w, it.nrm, it.perm, it.sigma, it.rec);
}

__global__ void __launch_bounds__(256) k_helm_table_multi(const HelmPrepItem *__restrict__ items) {
  const HelmPrepItem it = items[blockIdx.y];
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < it.n_targets;
       t += (int64_t)gridDim.x * blockDim.x)
    helm_table_row(it.tgt, t, it.k, it.p, it.tab, it.tabs);
}

__device__ __forceinline__ double4 load_rec(const double4 *__restrict__ base, uint32_t i,
                                            int half) {
  const TSQBX_GLOBAL char *b = (const TSQBX_GLOBAL char *)base;
  const f64x4 v = *(const TSQBX_GLOBAL f64x4 *)(b + ((size_t)i * 64u + (size_t)half * 32u));
  return make_double4(v.x, v.y, v.z, v.w);
}

struct HelmTarget {
  double cx, cy, cz;
  double tx, ty, tz;
  double rho_inv;  // 1/|t - c|, or 0 at t = c (then only n = 0 survives)
  double nx, ny, nz;  // target normal nu_t (S')
  double ntt;         // nu_t . delta / rho (0 at t = c)
};

// U pairs of one target; acc = (Re, Im) of the single layer, of the double
// layer and of S', without the factor i k / (4 pi).  tabs: the target's S'
// rows (k (2n+1) j_n', then (2n+1) j_n / rho).
template <int L, int U>
__device__ __forceinline__ void helm_pairs(int p, double k, double kinv, uint32_t n_src,
                                           const uint32_t (&s)[U],
                                           const double4 *__restrict__ rec,
                                           const double *__restrict__ tab,
                                           const double *__restrict__ tabs, const HelmTarget &tg,
                                           double (&acc)[6]) {
  double4 a[U], b[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    a[u] = load_rec(rec, s[u], 0);
    b[u] = load_rec(rec, s[u], 1);
  }
  double x[U], zi[U], rinv[U], nd[U], nts[U];
  double em1[U], e[U], g[U];           // P_{n-1}/lam_{n-1}, P_n/lam_n, P_n'
  double hm1r[U], hm1i[U], hr[U], hi[U];  // h_{n-1}, h_n
  double Sr[U], Si[U], Ar[U], Ai[U], Br[U], Bi[U], Cr[U], Ci[U];
  double Tr[U], Ti[U], Er[U], Ei[U];  // S': sum k (2n+1) j_n' P_n h_n, sum (2n+1) (j_n/rho) P_n' h_n
  const double A0 = tab[0];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double dx = a[u].x - tg.cx, dy = a[u].y - tg.cy, dz = a[u].z - tg.cz;
    const double R2 = fma(dz, dz, fma(dy, dy, dx * dx));
    rinv[u] = rsqrt_nr(R2);
    const double dd = fma(tg.tz, dz, fma(tg.ty, dy, tg.tx * dx));
    x[u] = dd * rinv[u] * tg.rho_inv;
    // padding entries (q = 0) get a harmless argument instead of k * 1e100
    const double z = s[u] == n_src ? 1.0 : k * (R2 * rinv[u]);
    zi[u] = kinv * rinv[u];
    if constexpr (L & 2) nd[u] = fma(b[u].w, dz, fma(b[u].z, dy, b[u].y * dx));
    if constexpr (L & 4) nts[u] = fma(tg.nz, dz, fma(tg.ny, dy, tg.nx * dx));
    double sn, cs;
    sincos(z, &sn, &cs);
    // h_0 = -i e^{iz} / z, h_1 = -(z + i) e^{iz} / z^2
    const double h0r = zi[u] * sn, h0i = -zi[u] * cs;
    const double h1r = zi[u] * fma(zi[u], sn, -cs), h1i = -zi[u] * fma(zi[u], cs, sn);
    // n = 0: m_0 = A_0 (P_0 = 1)
    Sr[u] = A0 * h0r;
    Si[u] = A0 * h0i;
    if constexpr (L & 2) {
      // sum m_n h_{n-1} starts with h_{-1} = h_0 / z - h_1; sum (n+1) m_n h_n
      Ar[u] = A0 * fma(zi[u], h0r, -h1r);
      Ai[u] = A0 * fma(zi[u], h0i, -h1i);
      Br[u] = A0 * h0r;
      Bi[u] = A0 * h0i;
      Cr[u] = 0.0;  // sum (2n+1) j_n P_n' h_n (P_0' = 0)
      Ci[u] = 0.0;
    }
    if constexpr (L & 4) {
      Tr[u] = tabs[0] * h0r;
      Ti[u] = tabs[0] * h0i;
      Er[u] = 0.0;  // P_0' = 0
      Ei[u] = 0.0;
    }
    em1[u] = 1.0;
    e[u] = x[u];
    g[u] = 1.0;
    hm1r[u] = h0r;
    hm1i[u] = h0i;
    hr[u] = h1r;
    hi[u] = h1i;
  }
  if (p >= 1) {
    const double A1 = tab[1];  // lam_1 = 1
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double m = A1 * e[u];
      Sr[u] = fma(m, hr[u], Sr[u]);
      Si[u] = fma(m, hi[u], Si[u]);
      if constexpr (L & 2) {
        Ar[u] = fma(m, hm1r[u], Ar[u]);
        Ai[u] = fma(m, hm1i[u], Ai[u]);
        const double m2 = 2.0 * m;
        Br[u] = fma(m2, hr[u], Br[u]);
        Bi[u] = fma(m2, hi[u], Bi[u]);
        Cr[u] = fma(A1, hr[u], Cr[u]);  // P_1' = 1
        Ci[u] = fma(A1, hi[u], Ci[u]);
      }
      if constexpr (L & 4) {
        const double mt = tabs[1] * e[u];
        Tr[u] = fma(mt, hr[u], Tr[u]);
        Ti[u] = fma(mt, hi[u], Ti[u]);
        Er[u] = fma(tabs[p + 2], hr[u], Er[u]);  // P_1' = 1
        Ei[u] = fma(tabs[p + 2], hi[u], Ei[u]);
      }
    }
  }
  // unrolled by two so that the three-term recurrences rotate their
  // registers without moves
#pragma unroll 2
  for (int n = 1; n < p; ++n) {
    // step to order n + 1
    const double kap = d_coef.kap[n];
    const double lam1 = d_coef.lam[n + 1];
    const double cn = (double)(n + 1) * d_coef.lam[n];
    const double tn = tab[n + 1];
    const double An = tn * lam1;
    const double w2 = (double)(2 * n + 1);
    const double np2 = (double)(n + 2);
    double Bt = 0.0, Et = 0.0;
    if constexpr (L & 4) {
      Bt = tabs[n + 1] * lam1;
      Et = tabs[p + 2 + n];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double ep1 = fma(x[u], e[u], -kap * em1[u]);
      const double w = w2 * zi[u];
      const double hp1r = fma(w, hr[u], -hm1r[u]);
      const double hp1i = fma(w, hi[u], -hm1i[u]);
      const double m = An * ep1;
      if constexpr (L & 1) {
        Sr[u] = fma(m, hp1r, Sr[u]);
        Si[u] = fma(m, hp1i, Si[u]);
      }
      double gp1 = 0.0;
      if constexpr (L & 6) gp1 = fma(x[u], g[u], cn * e[u]);
      if constexpr (L & 2) {
        Ar[u] = fma(m, hr[u], Ar[u]);
        Ai[u] = fma(m, hi[u], Ai[u]);
        const double mb = np2 * m;
        Br[u] = fma(mb, hp1r, Br[u]);
        Bi[u] = fma(mb, hp1i, Bi[u]);
        const double mc = tn * gp1;
        Cr[u] = fma(mc, hp1r, Cr[u]);
        Ci[u] = fma(mc, hp1i, Ci[u]);
      }
      if constexpr (L & 4) {
        const double mt = Bt * ep1;
        Tr[u] = fma(mt, hp1r, Tr[u]);
        Ti[u] = fma(mt, hp1i, Ti[u]);
        const double me = Et * gp1;
        Er[u] = fma(me, hp1r, Er[u]);
        Ei[u] = fma(me, hp1i, Ei[u]);
      }
      if constexpr (L & 6) g[u] = gp1;
      em1[u] = e[u];
      e[u] = ep1;
      hm1r[u] = hr[u];
      hm1i[u] = hi[u];
      hr[u] = hp1r;
      hi[u] = hp1i;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double qr = a[u].w, qi = b[u].x;
    if constexpr (L & 1) {
      acc[0] = fma(qr, Sr[u], fma(-qi, Si[u], acc[0]));
      acc[1] = fma(qr, Si[u], fma(qi, Sr[u], acc[1]));
    }
    if constexpr (L & 2) {
      // sum (2n+1) j_n P_n h_n' = A - (1/z) B
      const double T1r = fma(-zi[u], Br[u], Ar[u]);
      const double T1i = fma(-zi[u], Bi[u], Ai[u]);
      const double ntd = fma(b[u].w, tg.tz, fma(b[u].z, tg.ty, b[u].y * tg.tx));
      const double c1 = k * nd[u];
      const double c2 = fma(ntd, tg.rho_inv, -nd[u] * rinv[u] * x[u]);
      const double Dr = rinv[u] * fma(c1, T1r, c2 * Cr[u]);
      const double Di = rinv[u] * fma(c1, T1i, c2 * Ci[u]);
      acc[2] = fma(qr, Dr, fma(-qi, Di, acc[2]));
      acc[3] = fma(qr, Di, fma(qi, Dr, acc[3]));
    }
    if constexpr (L & 4) {
      // (nu_t.delta/rho) T + (nu_t.d / R - (nu_t.delta/rho) x) E
      const double c2 = fma(nts[u], rinv[u], -tg.ntt * x[u]);
      const double Vr = fma(tg.ntt, Tr[u], c2 * Er[u]);
      const double Vi = fma(tg.ntt, Ti[u], c2 * Ei[u]);
      acc[4] = fma(qr, Vr, fma(-qi, Vi, acc[4]));
      acc[5] = fma(qr, Vi, fma(qi, Vr, acc[5]));
    }
  }
}

// One target t (device order) of evaluation v, summed by the G lanes of its
// group (lane gl of G), and its outputs written.  The plain and the batched
// kernels both run this, so their results agree bit for bit.
template <int L, int G, int U>
__device__ __forceinline__ void helm_target(const HelmWorkItem &v, int64_t t, int gl) {
  const TargetRec tr = v.tgt[t];
  HelmTarget tg;
  tg.cx = tr.c[0];
  tg.cy = tr.c[1];
  tg.cz = tr.c[2];
  tg.tx = tr.d[0];
  tg.ty = tr.d[1];
  tg.tz = tr.d[2];
  const double rho = sqrt(fma(tg.tz, tg.tz, fma(tg.ty, tg.ty, tg.tx * tg.tx)));
  tg.rho_inv = rho > 0.0 ? 1.0 / rho : 0.0;
  tg.nx = tg.ny = tg.nz = tg.ntt = 0.0;
  if constexpr (L & 4) {
    const double4 nv = v.tnrm[t];
    tg.nx = nv.x;
    tg.ny = nv.y;
    tg.nz = nv.z;
    tg.ntt = fma(tg.nz, tg.tz, fma(tg.ny, tg.ty, tg.nx * tg.tx)) * tg.rho_inv;
  }
  const int p = v.p;
  const double k = v.k;
  const double kinv = 1.0 / k;
  const double *row_tab = v.tab + t * (int64_t)(p + 1);
  const double *row_tabs = (L & 4) ? v.tabs + t * (int64_t)(2 * (p + 1)) : nullptr;
  const int32_t *__restrict__ row = v.idx + tr.row_begin;
  const int len = tr.row_len;
  double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  int c0 = 0;
  if constexpr (U > 1) {
    const int full = len - len % (G * U);
    for (; c0 < full; c0 += G * U) {
      uint32_t s[U];
#pragma unroll
      for (int u = 0; u < U; ++u) s[u] = load_idx(row, (uint32_t)(c0 + gl + u * G));
      helm_pairs<L, U>(p, k, kinv, v.n_src, s, v.rec, row_tab, row_tabs, tg, acc);
    }
  }
  for (; c0 < len; c0 += G) {
    const int j = c0 + gl;
    if (j < len) {
      const uint32_t s1[1] = {load_idx(row, (uint32_t)j)};
      helm_pairs<L, 1>(p, k, kinv, v.n_src, s1, v.rec, row_tab, row_tabs, tg, acc);
    }
  }
#pragma unroll
  for (int off = G / 2; off >= 1; off >>= 1)
#pragma unroll
    for (int c = 0; c < 6; ++c)
      if (L & (1 << (c / 2))) acc[c] += __shfl_xor(acc[c], off, 64);
  if (gl != 0) return;
  // times i k / (4 pi): (re, im) -> (-im, re) k / (4 pi)
  const double f = k * kInv4Pi;
  const int o = tr.out_index;
  double *const outs[3] = {v.out_s, v.out_d, v.out_t};
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    if (!(L & (1 << l))) continue;
    double *out = outs[l];
    const double vr = -acc[2 * l + 1] * f, vi = acc[2 * l] * f;
    out[2 * o] = v.accumulate ? out[2 * o] + vr : vr;
    out[2 * o + 1] = v.accumulate ? out[2 * o + 1] + vi : vi;
  }
}

template <int L, int G, int U>
__global__ void __launch_bounds__(256)
k_helm_eval(HelmWorkItem v, int64_t n_targets, int remap) {
  constexpr int TPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int wpb = blockDim.x >> 6;
  const int blk = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  int64_t t = ((int64_t)blk * wpb + wave) * TPW + lane / G;
  if constexpr (G == 64) t = __builtin_amdgcn_readfirstlane((int)t);
  if (t >= n_targets) return;
  helm_target<L, G, U>(v, t, lane % G);
}

// The batched Helmholtz kernel: resident waves work through a static
// schedule of units (runs of consecutive targets of one item), as the
// Laplace persistent kernel does.  LC: the layer mask shared by every item
// (1..7), or kLayersAny (a switch over the masks).
template <int LC, int G, int U>
__global__ void __launch_bounds__(256, 3) k_helm_persistent(HelmPersistentArgs a) {
  constexpr int TPW = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wpb = blockDim.x >> 6;
  const int w = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * wpb +
                                               (int)(threadIdx.x >> 6));
  if (w >= a.n_waves) return;
  const int ub = a.wave_begin[w], ue = a.wave_begin[w + 1];
  for (int u = ub; u < ue; ++u) {
    const int item = __builtin_amdgcn_readfirstlane(a.units[u].item);
    const int first = __builtin_amdgcn_readfirstlane(a.units[u].first);
    const int count = __builtin_amdgcn_readfirstlane(a.units[u].count);
    const HelmWorkItem v = a.items[item];
    for (int q = 0; q < count; q += TPW) {
      int slot = q + lane / G;
      if constexpr (G == 64) slot = __builtin_amdgcn_readfirstlane(slot);
      if (slot >= count) break;  // whole groups leave together
      const int64_t t = (int64_t)first + slot;
      if constexpr (LC != kLayersAny) {
        helm_target<LC, G, U>(v, t, lane % G);
      } else {
        switch (v.layers) {
          case 1: helm_target<1, G, U>(v, t, lane % G); break;
          case 2: helm_target<2, G, U>(v, t, lane % G); break;
          case 3: helm_target<3, G, U>(v, t, lane % G); break;
          case 4: helm_target<4, G, U>(v, t, lane % G); break;
          case 5: helm_target<5, G, U>(v, t, lane % G); break;
          case 6: helm_target<6, G, U>(v, t, lane % G); break;
          default: helm_target<7, G, U>(v, t, lane % G); break;
        }
      }
    }
  }
}

template <int L, int G, int U>
hipError_t launch_helm_lgu(const tsqbx_geometry *g, int p, double k, const HelmStage &st,
                           const Outputs &o, bool acc, const Tuning &tn, hipStream_t s) {
  constexpr int TPW = 64 / G;
  const int64_t per_block = (int64_t)tn.waves_per_block * TPW;
  const int64_t blocks = (g->n_targets + per_block - 1) / per_block;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  HelmWorkItem v{};
  v.tgt = g->tgt;
  v.tnrm = g->tgt_nrm;
  v.idx = g->idx;
  v.rec = st.rec;
  v.tab = st.tab;
  v.tabs = st.tabs;
  v.out_s = o.s;
  v.out_d = o.d;
  v.out_t = o.t;
  v.k = k;
  v.p = p;
  v.layers = L;
  v.accumulate = acc ? 1 : 0;
  v.n_src = (uint32_t)g->n_sources;
  hipLaunchKernelGGL((k_helm_eval<L, G, U>), dim3((unsigned)blocks),
                     dim3(64 * tn.waves_per_block), 0, s, v, g->n_targets, tn.xcd_remap);
  return hipGetLastError();
}

template <int G, int U>
hipError_t launch_helm_gu(const tsqbx_geometry *g, int p, unsigned layers, double k,
                          const HelmStage &st, const Outputs &o, bool acc, const Tuning &tn,
                          hipStream_t s) {
  switch (layers) {
    case 1: return launch_helm_lgu<1, G, U>(g, p, k, st, o, acc, tn, s);
    case 2: return launch_helm_lgu<2, G, U>(g, p, k, st, o, acc, tn, s);
    case 3: return launch_helm_lgu<3, G, U>(g, p, k, st, o, acc, tn, s);
    case 4: return launch_helm_lgu<4, G, U>(g, p, k, st, o, acc, tn, s);
    case 5: return launch_helm_lgu<5, G, U>(g, p, k, st, o, acc, tn, s);
    case 6: return launch_helm_lgu<6, G, U>(g, p, k, st, o, acc, tn, s);
    case 7: return launch_helm_lgu<7, G, U>(g, p, k, st, o, acc, tn, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_helm_prepare(const tsqbx_geometry *g, int p, unsigned layers, double k,
                               const double *d_sigma, const HelmStage &st, hipStream_t s) {
  // S' needs the target normals (none are stored when there are no targets)
  // and the S' table
  if ((layers & TSQBX_SPRIME) && ((g->n_targets > 0 && !g->tgt_nrm) || !st.tabs))
    return hipErrorInvalidValue;
  const int64_t n = g->n_sources, T = g->n_targets;
  {
    const int64_t blocks = std::min<int64_t>((n + 1 + 255) / 256, 65536);
    hipLaunchKernelGGL(k_helm_stage, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s,
                       n, g->src_pos, g->src_nrm, g->src_perm, d_sigma, st.rec);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (T <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_helm_table, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, g->tgt, T,
                     k, p, st.tab, (layers & TSQBX_SPRIME) ? st.tabs : nullptr);
  return hipGetLastError();
}

hipError_t launch_helmholtz(const tsqbx_geometry *g, int p, unsigned layers, double k,
                            const double *d_sigma, const HelmStage &st, const Outputs &out,
                            bool accumulate, const Tuning &tn, hipStream_t s) {
  if (!tuning_supported(tn)) return hipErrorInvalidValue;
  hipError_t e = launch_helm_prepare(g, p, layers, k, d_sigma, st, s);
  if (e != hipSuccess || g->n_targets <= 0) return e;
  // the pair kernel keeps at most two pairs in flight
  const int G = tn.group_lanes, U = std::min(tn.unroll, 2);
  if (G == 64 && U == 1) return launch_helm_gu<64, 1>(g, p, layers, k, st, out, accumulate, tn, s);
  if (G == 64) return launch_helm_gu<64, 2>(g, p, layers, k, st, out, accumulate, tn, s);
  if (G == 32) return launch_helm_gu<32, 2>(g, p, layers, k, st, out, accumulate, tn, s);
  return launch_helm_gu<16, 2>(g, p, layers, k, st, out, accumulate, tn, s);
}

namespace {
template <int LC>
hipError_t launch_helm_persistent_l(const HelmPersistentArgs &a, const Tuning &tn,
                                    hipStream_t s) {
  const dim3 block(64 * tn.waves_per_block);
  const int grid = (a.n_waves + tn.waves_per_block - 1) / tn.waves_per_block;
  // the same (group width, pairs in flight) choices as the plain kernel
  const int G = tn.group_lanes, U = std::min(tn.unroll, 2);
  if (G == 64 && U == 1)
    hipLaunchKernelGGL((k_helm_persistent<LC, 64, 1>), dim3(grid), block, 0, s, a);
  else if (G == 64)
    hipLaunchKernelGGL((k_helm_persistent<LC, 64, 2>), dim3(grid), block, 0, s, a);
  else if (G == 32)
    hipLaunchKernelGGL((k_helm_persistent<LC, 32, 2>), dim3(grid), block, 0, s, a);
  else
    hipLaunchKernelGGL((k_helm_persistent<LC, 16, 2>), dim3(grid), block, 0, s, a);
  return hipGetLastError();
}
}  // namespace

hipError_t launch_helm_prepare_multi(const HelmPrepItem *d_items, int n_items, int64_t max_n,
                                     int64_t max_t, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  if (n_items > 65535) return hipErrorInvalidValue;
  const unsigned bs = (unsigned)std::min<int64_t>(std::max<int64_t>((max_n + 1 + 255) / 256, 1), 4096);
  hipLaunchKernelGGL(k_helm_stage_multi, dim3(bs, (unsigned)n_items), dim3(256), 0, s, d_items);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || max_t <= 0) return e;
  const unsigned bt = (unsigned)std::min<int64_t>(std::max<int64_t>((max_t + 255) / 256, 1), 4096);
  hipLaunchKernelGGL(k_helm_table_multi, dim3(bt, (unsigned)n_items), dim3(256), 0, s, d_items);
  return hipGetLastError();
}

hipError_t launch_helm_persistent(const HelmPersistentArgs &a, unsigned layer_class,
                                  const Tuning &tn, hipStream_t s) {
  if (!tuning_supported(tn) || a.n_waves <= 0) return hipErrorInvalidValue;
  switch (layer_class) {
    case 1: return launch_helm_persistent_l<1>(a, tn, s);
    case 2: return launch_helm_persistent_l<2>(a, tn, s);
    case 3: return launch_helm_persistent_l<3>(a, tn, s);
    case 4: return launch_helm_persistent_l<4>(a, tn, s);
    case 5: return launch_helm_persistent_l<5>(a, tn, s);
    case 6: return launch_helm_persistent_l<6>(a, tn, s);
    case 7: return launch_helm_persistent_l<7>(a, tn, s);
    default: return launch_helm_persistent_l<kLayersAny>(a, tn, s);
  }
}

}  // namespace tsqbx
