// Conventional QBX on the device (Sec. 2.3; the first approach of Sec. 2.4),
// the comparator of the target-specific path: for every center that a
// target uses, the local coefficients
//   L_n^m = sum_{y in L(c)} q_y Y_n^{-m}(y - c) / ((2n+1) |y - c|^{n+1}),
// n = 0..p, 0 <= m <= n (eq. local-coeffs; real densities give
// L_n^{-m} = conj(L_n^m)), and the truncated local expansion at the targets
//   u(t) = sum_n [ L_n^0 rho^n Y_n^0 + 2 sum_{m>=1} Re(L_n^m rho^n Y_n^m) ]
// (eq. local-expansion), Y_n^m of eq. sph-harm with P_n^{|m|} taken without
// the Condon-Shortley factor.  Work per (source, center) is O((p+1)^2)
// against O(p+1) per (source, target) for the target-specific kernel.
//
// The solid harmonics come from Cartesian recurrences, with no angles:
//   irregular, d = y - c:  A_n^m = P_n^m(d_z/R) e^{-i m phi} / R^{n+1},
//     A_m^m = (2m-1)!! (d_x - i d_y)^m / R^{2m+1},
//     (n-m) A_n^m = (2n-1) (d_z/R^2) A_{n-1}^m - (n+m-1) (1/R^2) A_{n-2}^m;
//   regular, delta = t - c:  B_n^m = rho^n P_n^m(delta_z/rho) e^{i m phi},
//     B_m^m = (2m-1)!! (delta_x + i delta_y)^m,
//     (n-m) B_n^m = (2n-1) delta_z B_{n-1}^m - (n+m-1) rho^2 B_{n-2}^m
// (the associated-Legendre recurrence in the degree at fixed order, times
// the powers of R or rho).  Dividing both by s_n^m = (2n-1)!!/(n-m)!, the
// leading factor of P_n^m, leaves
//   a_n = zeta a_{n-1} - kappa_n^m eta a_{n-2},
//   kappa_n^m = ((n-1)^2 - m^2) / ((2n-1)(2n-3)),
// one multiply shared by the real and imaginary parts and two multiply-adds
// each (zeta, eta = d_z/R^2, 1/R^2 or delta_z, rho^2).
//
// Layout: one wave per center row.  For each order m the lanes stride over
// the row's list, two entries at a time; each recomputes the source's
// geometry and (d_x - i d_y)^m by a fixed chain of squarings, runs the
// degrees n = m..p and adds into registers; a xor butterfly then sums the
// lanes and lane 0 stores the scaled coefficients into LDS.  The evaluation reads them from LDS, one
// target per lane.  Coefficients in memory use the compact real layout:
// (p+1)^2 doubles per center, degree n at offset n^2, holding Re L_n^0 and
// then Re L_n^m, Im L_n^m for m = 1..n.
#include <algorithm>

#include "tsqbx_device.h"

namespace tsqbx {
namespace {

constexpr double kShPi = 3.14159265358979323846;

// Coefficients read back from LDS one by one as the evaluation uses them
// (volatile, so that the compiler does not hoist all of them into registers
// ahead of the loop over a row's targets).
#define TSQBX_LDS_RO volatile __attribute__((address_space(3)))

// Newton's iteration from above for the square root of x > 0 (compile time).
constexpr double sh_sqrt(double x) {
  double y = x > 1.0 ? x : 1.0;
  for (int i = 0; i < 400; ++i) {
    const double z = 0.5 * (y + x / y);
    if (!(z < y)) break;
    y = z;
  }
  return y;
}
constexpr double sh_dfact(int n) {  // (2n-1)!!
  double r = 1.0;
  for (int k = 1; k <= n; ++k) r *= double(2 * k - 1);
  return r;
}
constexpr double sh_fact(int n) {
  double r = 1.0;
  for (int k = 2; k <= n; ++k) r *= double(k);
  return r;
}
// N_n^m s_n^m with N_n^m = sqrt((2n+1)/(4 pi) (n-m)!/(n+m)!) (eq. sph-harm)
constexpr double sh_ns(int n, int m) {
  return sh_sqrt(double(2 * n + 1) / (4.0 * kShPi)) * sh_dfact(n) /
         sh_sqrt(sh_fact(n - m) * sh_fact(n + m));
}
constexpr double sh_kap(int n, int m) {
  return double((n - 1) * (n - 1) - m * m) / double((2 * n - 1) * (2 * n - 3));
}
// scale of the summed rescaled irregular harmonics into L_n^m
constexpr double sh_form_scale(int n, int m) { return sh_ns(n, m) / double(2 * n + 1); }
// weight of L_n^m times the rescaled regular harmonic in u (2 Re for m > 0)
constexpr double sh_eval_scale(int n, int m) { return (m ? 2.0 : 1.0) * sh_ns(n, m); }

// (wr + i wi)^M by squarings.
template <int M>
__device__ __forceinline__ void cpow(double wr, double wi, double &pr, double &pi) {
  if constexpr (M == 0) {
    pr = 1.0;
    pi = 0.0;
  } else if constexpr (M == 1) {
    pr = wr;
    pi = wi;
  } else if constexpr (M % 2 == 0) {
    double hr, hi;
    cpow<M / 2>(wr, wi, hr, hi);
    pr = fma(hr, hr, -(hi * hi));
    pi = (hr + hr) * hi;
  } else {
    double hr, hi;
    cpow<M - 1>(wr, wi, hr, hi);
    pr = fma(hr, wr, -(hi * wi));
    pi = fma(hr, wi, hi * wr);
  }
}

// Degrees n = N..PC of order M (stopping after p unless EXACT) for U list
// entries whose recurrences interleave; (r1, i1) and (r2, i2) hold the
// rescaled harmonics of degrees n-1 and n-2.  Adds each degree's values into
// (ar, ai)[n - M], entry 0 first.  REAL: order 0, imaginary parts zero.
template <int PC, bool EXACT, int M, int N, bool REAL, int U>
__device__ __forceinline__ void irr_steps(int p, const double (&zz)[U], const double (&ii)[U],
                                          const double (&r1)[U], const double (&i1)[U],
                                          const double (&r2)[U], const double (&i2)[U],
                                          double (&ar)[PC - M + 1], double (&ai)[PC - M + 1]) {
  if constexpr (N <= PC) {
    if constexpr (!EXACT)
      if (N > p) return;
    double r[U], i[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      i[u] = 0.0;
      if constexpr (N == M + 1) {
        r[u] = zz[u] * r1[u];
        if constexpr (!REAL) i[u] = zz[u] * i1[u];
      } else {
        constexpr double kap = sh_kap(N, M);
        const double t = kap * ii[u];
        r[u] = fma(zz[u], r1[u], -(t * r2[u]));
        if constexpr (!REAL) i[u] = fma(zz[u], i1[u], -(t * i2[u]));
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ar[N - M] += r[u];
      if constexpr (!REAL) ai[N - M] += i[u];
    }
    irr_steps<PC, EXACT, M, N + 1, REAL, U>(p, zz, ii, r, i, r1, i1, ar, ai);
  }
}

// The terms of order M of U list entries (sources s[u]), added into (ar, ai).
template <int PC, bool EXACT, int M, int U>
__device__ __forceinline__ void order_terms(int p, const uint32_t (&s)[U], double cx, double cy,
                                            double cz, const SrcView &src,
                                            double (&ar)[PC - M + 1], double (&ai)[PC - M + 1]) {
  double zz[U], ii[U], tr[U], ti[U], z0[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const double2 a = load2(src.xy, s[u]);
    const double2 aq = load2(src.zq, s[u]);  // (z, q)
    const double dx = a.x - cx, dy = a.y - cy, dz = aq.x - cz;
    const double R2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const double rinv = rsqrt_nr(R2);
    ii[u] = rinv * rinv;
    zz[u] = dz * ii[u];
    z0[u] = 0.0;
    const double qr = aq.y * rinv;  // q / R
    ti[u] = 0.0;                   // (tr, ti) = q (d_x - i d_y)^M / R^{2M+1}
    if constexpr (M == 0) {
      tr[u] = qr;
    } else {
      double pr, pi;
      cpow<M>(dx * ii[u], -(dy * ii[u]), pr, pi);
      tr[u] = qr * pr;
      ti[u] = qr * pi;
    }
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    ar[0] += tr[u];
    if constexpr (M > 0) ai[0] += ti[u];
  }
  irr_steps<PC, EXACT, M, M + 1, M == 0, U>(p, zz, ii, tr, ti, z0, z0, ar, ai);
}

// Lane 0 stores the summed degrees n = N..min(p, PC) of order M into coef.
template <int PC, bool EXACT, int M, int N>
__device__ __forceinline__ void store_order(int p, const double (&ar)[PC - M + 1],
                                            const double (&ai)[PC - M + 1], double *coef) {
  if constexpr (N <= PC) {
    if constexpr (!EXACT)
      if (N > p) return;
    constexpr double sc = sh_form_scale(N, M);
    if constexpr (M == 0) {
      coef[N * N] = ar[0 + N - M] * sc;
    } else {
      coef[N * N + 2 * M - 1] = ar[N - M] * sc;
      coef[N * N + 2 * M] = ai[N - M] * sc;
    }
    store_order<PC, EXACT, M, N + 1>(p, ar, ai, coef);
  }
}

// The coefficients of order M, then of the orders above it.
template <int PC, bool EXACT, int M>
__device__ __forceinline__ void form_orders(int p, int lane, const int32_t *__restrict__ row,
                                            int len, double cx, double cy, double cz,
                                            const SrcView &src, double *coef) {
  if constexpr (M <= PC) {
    if constexpr (!EXACT)
      if (M > p) return;
    constexpr int K = PC - M + 1;
    double ar[K], ai[K];
#pragma unroll
    for (int k = 0; k < K; ++k) ar[k] = ai[k] = 0.0;
    // lane l takes the entries l, l + 64, l + 128, ..., two at a time
    int j = lane;
    for (; j + 64 < len; j += 128) {
      const uint32_t s2[2] = {load_idx(row, (uint32_t)j), load_idx(row, (uint32_t)(j + 64))};
      order_terms<PC, EXACT, M, 2>(p, s2, cx, cy, cz, src, ar, ai);
    }
    if (j < len) {
      const uint32_t s1[1] = {load_idx(row, (uint32_t)j)};
      order_terms<PC, EXACT, M, 1>(p, s1, cx, cy, cz, src, ar, ai);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) {
      if (EXACT || M + k <= p) {
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
          ar[k] += __shfl_xor(ar[k], off, 64);
          if constexpr (M > 0) ai[k] += __shfl_xor(ai[k], off, 64);
        }
      }
    }
    if (lane == 0) store_order<PC, EXACT, M, M>(p, ar, ai, coef);
    form_orders<PC, EXACT, M + 1>(p, lane, row, len, cx, cy, cz, src, coef);
  }
}

// u += sum over degrees n = N..p of order M of the coefficient times the
// rescaled regular harmonic (b1, c1) = degree n-1, (b2, c2) = degree n-2.
template <int PC, bool EXACT, int M, int N>
__device__ __forceinline__ void reg_steps(int p, double zz, double rr, double b1, double c1,
                                          double b2, double c2, const TSQBX_LDS_RO double *coef,
                                          double &u) {
  if constexpr (N <= PC) {
    if constexpr (!EXACT)
      if (N > p) return;
    double b, c = 0.0;
    if constexpr (N == M + 1) {
      b = zz * b1;
      if constexpr (M > 0) c = zz * c1;
    } else {
      constexpr double kap = sh_kap(N, M);
      const double t = kap * rr;
      b = fma(zz, b1, -(t * b2));
      if constexpr (M > 0) c = fma(zz, c1, -(t * c2));
    }
    constexpr double es = sh_eval_scale(N, M);
    if constexpr (M == 0)
      u = fma(es * coef[N * N], b, u);
    else
      u = fma(es, fma(coef[N * N + 2 * M - 1], b, -(coef[N * N + 2 * M] * c)), u);
    reg_steps<PC, EXACT, M, N + 1>(p, zz, rr, b, c, b1, c1, coef, u);
  }
}

// Orders M..p at one target; (zr, zi) = (delta_x + i delta_y)^M.
template <int PC, bool EXACT, int M>
__device__ __forceinline__ void eval_orders(int p, double dx, double dy, double dz, double rr,
                                            double zr, double zi, const TSQBX_LDS_RO double *coef,
                                            double &u) {
  if constexpr (M <= PC) {
    if constexpr (!EXACT)
      if (M > p) return;
    constexpr double es = sh_eval_scale(M, M);
    if constexpr (M == 0)
      u = fma(es * coef[0], zr, u);
    else
      u = fma(es, fma(coef[M * M + 2 * M - 1], zr, -(coef[M * M + 2 * M] * zi)), u);
    reg_steps<PC, EXACT, M, M + 1>(p, dz, rr, zr, zi, 0.0, 0.0, coef, u);
    const double nr = fma(zr, dx, -(zi * dy));
    const double ni = fma(zr, dy, zi * dx);
    eval_orders<PC, EXACT, M + 1>(p, dx, dy, dz, rr, nr, ni, coef, u);
  }
}

constexpr int kModeForm = 1, kModeEval = 2;

// One wave (block of 64) per center row.  MODE & kModeForm: form the
// coefficients from the staged sources; else read them from
// coeffs_in.  MODE & kModeEval: evaluate at the row's targets into out;
// else write the coefficients to coeffs_out.
template <int PC, bool EXACT, int MODE>
__global__ void __launch_bounds__(64)
k_qbxl(const CenterRec *__restrict__ rows, int64_t n_rows, const int32_t *__restrict__ idx,
       SrcView src, const int32_t *__restrict__ row_tgts,
       const TargetRec *__restrict__ tgt, const double *__restrict__ coeffs_in,
       double *__restrict__ coeffs_out, double *__restrict__ out, int p_rt, int accumulate,
       int remap) {
  __shared__ double coef[(PC + 1) * (PC + 1)];
  const int p = EXACT ? PC : p_rt;
  const int nc = (p + 1) * (p + 1);
  const int lane = threadIdx.x;
  const int64_t r = remap ? xcd_remap(blockIdx.x, gridDim.x) : blockIdx.x;
  if (r >= n_rows) return;
  const TSQBX_GLOBAL CenterRec *cr = (const TSQBX_GLOBAL CenterRec *)rows + r;
  const double cx = cr->c[0], cy = cr->c[1], cz = cr->c[2];
  const int64_t center = cr->center;
  if constexpr ((MODE & kModeForm) != 0) {
    form_orders<PC, EXACT, 0>(p, lane, idx + cr->row_begin, cr->len, cx, cy, cz, src, coef);
  } else {
    for (int k = lane; k < nc; k += 64) coef[k] = coeffs_in[center * nc + k];
  }
  __syncthreads();
  if constexpr ((MODE & kModeEval) != 0) {
    const int tb = cr->tgt_begin, tn = cr->tgt_count;
    for (int k = lane; k < tn; k += 64) {
      const TSQBX_GLOBAL TargetRec *tr = (const TSQBX_GLOBAL TargetRec *)tgt + row_tgts[tb + k];
      const double dx = tr->d[0], dy = tr->d[1], dz = tr->d[2];
      const double rr = fma(dz, dz, fma(dy, dy, dx * dx));
      double u = 0.0;
      eval_orders<PC, EXACT, 0>(p, dx, dy, dz, rr, 1.0, 0.0,
                                (const TSQBX_LDS_RO double *)coef, u);
      const int o = tr->out_index;
      out[o] = accumulate ? out[o] + u : u;
    }
  } else {
    double *dst = coeffs_out + center * nc;
    for (int k = lane; k < nc; k += 64) dst[k] = accumulate ? dst[k] + coef[k] : coef[k];
  }
}

template <int PC, bool EXACT, int MODE>
hipError_t launch_mode(const tsqbx_geometry *g, int p, const SrcView &src, const double *cin,
                       double *cout, double *out, bool acc, hipStream_t s) {
  const int64_t blocks = g->n_rows;
  if (blocks <= 0) return hipSuccess;
  if (blocks > INT32_MAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_qbxl<PC, EXACT, MODE>), dim3((unsigned)blocks), dim3(64), 0, s, g->ctr,
                     g->n_rows, g->idx, src, g->row_tgts, g->tgt, cin, cout, out, p, acc ? 1 : 0,
                     1);
  return hipGetLastError();
}

template <int MODE>
hipError_t launch_p(const tsqbx_geometry *g, int p, const SrcView &src, const double *cin,
                    double *cout, double *out, bool acc, hipStream_t s) {
  switch (p) {
    case 5: return launch_mode<5, true, MODE>(g, p, src, cin, cout, out, acc, s);
    case 8: return launch_mode<8, true, MODE>(g, p, src, cin, cout, out, acc, s);
    case 16: return launch_mode<16, true, MODE>(g, p, src, cin, cout, out, acc, s);
    default:
      if (p <= 16) return launch_mode<16, false, MODE>(g, p, src, cin, cout, out, acc, s);
      return launch_mode<32, false, MODE>(g, p, src, cin, cout, out, acc, s);
  }
}

}  // namespace

hipError_t launch_qbxl(const tsqbx_geometry *g, int p, int mode, const SourceStage &st,
                       const double *coeffs_in, double *coeffs_out, double *out, bool accumulate,
                       hipStream_t s) {
  if (p < 0 || p > TSQBX_P_MAX) return hipErrorInvalidValue;
  const SrcView src{st.xy, st.zq, nullptr, nullptr};
  const SrcView none{nullptr, nullptr, nullptr, nullptr};
  switch (mode) {
    case kModeForm: return launch_p<kModeForm>(g, p, src, nullptr, coeffs_out, nullptr, accumulate, s);
    case kModeEval: return launch_p<kModeEval>(g, p, none, coeffs_in, nullptr, out, accumulate, s);
    case kModeForm | kModeEval:
      return launch_p<kModeForm | kModeEval>(g, p, src, nullptr, nullptr, out, accumulate, s);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tsqbx
