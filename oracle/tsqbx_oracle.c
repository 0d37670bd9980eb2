/*
 * Plain FP64 CPU oracle for TSQBX near-field evaluation.  TEST
 * INFRASTRUCTURE ONLY: see tsqbx_oracle.h for what is computed and where the
 * paper defines it.  Built with -O2 -fno-fast-math -ffp-contract=off so that
 * every operation below is one IEEE FP64 rounding, in the order written.
 */
#include "tsqbx_oracle.h"

#include <math.h>
#include <stddef.h>
#include <omp.h>

static const double PI = 3.14159265358979323846;

static double dot3(const double a[3], const double b[3]) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* One pair, following App. A term by term: x = cos(gamma), P_n(x) and
 * P_n'(x) by recurrence, running powers |t-c|^n and |s-c|^-(n+1). */
void tsqbx_oracle_pair(const double t[3], const double c[3], const double s[3],
                       const double *nu, const double *nu_t, int p, double k[6]) {
  double dt[3] = {t[0] - c[0], t[1] - c[1], t[2] - c[2]};
  double ds[3] = {s[0] - c[0], s[1] - c[1], s[2] - c[2]};
  double rho = sqrt(dot3(dt, dt));
  double R = sqrt(dot3(ds, ds));
  double that[3] = {0.0, 0.0, 0.0};
  if (rho > 0.0) {
    that[0] = dt[0] / rho;
    that[1] = dt[1] / rho;
    that[2] = dt[2] / rho;
  }
  double shat[3] = {ds[0] / R, ds[1] / R, ds[2] / R};
  double x = dot3(that, shat);
  double nu_sh = 0.0, nu_th = 0.0, nu_len = 0.0, perp = 0.0;
  if (nu) {
    nu_sh = dot3(nu, shat);
    nu_th = dot3(nu, that);
    nu_len = sqrt(dot3(nu, nu));
    /* |t_hat - s_hat x|: length of the P_n' direction of the source gradient */
    double w[3] = {that[0] - shat[0] * x, that[1] - shat[1] * x, that[2] - shat[2] * x};
    perp = sqrt(dot3(w, w));
  }
  double m_t = 0.0, m_s = 0.0, m_len = 0.0, m_perp = 0.0;
  if (nu_t) {
    m_t = dot3(nu_t, that);
    m_s = dot3(nu_t, shat);
    m_len = sqrt(dot3(nu_t, nu_t));
    /* |s_hat - t_hat x|: length of the P_n' direction of the target gradient */
    double w[3] = {shat[0] - that[0] * x, shat[1] - that[1] * x, shat[2] - that[2] * x};
    m_perp = sqrt(dot3(w, w));
  }
  double Rinv = 1.0 / R;

  double P_prev = 0.0; /* P_{n-1} */
  double P = 1.0;      /* P_n */
  double dP = 0.0;     /* P_n' */
  double rho_n = 1.0;  /* |t-c|^n */
  double rho_nm1 = 1.0;/* |t-c|^(n-1), used from n = 1 on */
  double Rpow = Rinv;  /* |s-c|^-(n+1) */
  double ks = 0.0, ks_abs = 0.0, kd = 0.0, kd_abs = 0.0, kt = 0.0, kt_abs = 0.0;
  for (int n = 0; n <= p; ++n) {
    double radial = rho_n * Rpow;
    double term_s = radial * P;
    ks += term_s;
    ks_abs += fabs(term_s);
    if (nu) {
      double radial_d = radial * Rinv;
      double a = -(double)(n + 1) * nu_sh * P;
      double b = (nu_th - nu_sh * x) * dP;
      kd += radial_d * (a + b);
      /* yardstick: |nu| times the size of the gradient term, which bounds
       * the rounding of its projection on nu */
      kd_abs += radial_d * nu_len * ((double)(n + 1) * fabs(P) + fabs(dP) * perp);
    }
    if (nu_t && n >= 1) {
      /* App. A's target gradient starts at n = 1 */
      double radial_t = rho_nm1 * Rpow;
      double a = (double)n * m_t * P;
      double b = (m_s - m_t * x) * dP;
      kt += radial_t * (a + b);
      kt_abs += radial_t * m_len * ((double)n * fabs(P) + fabs(dP) * m_perp);
      rho_nm1 *= rho;
    }
    /* Bonnet: (n+1) P_{n+1} = (2n+1) x P_n - n P_{n-1};  P_{n+1}' = x P_n' + (n+1) P_n */
    double P_next = ((double)(2 * n + 1) * x * P - (double)n * P_prev) / (double)(n + 1);
    double dP_next = x * dP + (double)(n + 1) * P;
    P_prev = P;
    P = P_next;
    dP = dP_next;
    rho_n *= rho;
    Rpow *= Rinv;
  }
  double inv4pi = 1.0 / (4.0 * PI);
  k[0] = ks * inv4pi;
  k[1] = kd * inv4pi;
  k[2] = ks_abs * inv4pi;
  k[3] = kd_abs * inv4pi;
  k[4] = kt * inv4pi;
  k[5] = kt_abs * inv4pi;
}

int tsqbx_oracle_max_threads(void) { return omp_get_max_threads(); }

int tsqbx_oracle_eval(const tsqbx_oracle_problem *prob, int p, unsigned layers,
                      const double *sigma, int64_t n_sel, const int64_t *sel,
                      double *const out[3], double *const abs[3], int n_threads) {
  if (!prob || p < 0 || !sigma || !out || !abs) return -1;
  if ((layers & TSQBX_ORACLE_DLP) && !prob->normals) return -1;
  if ((layers & TSQBX_ORACLE_SPRIME) && !prob->target_normals) return -1;
  int64_t n_out = sel ? n_sel : prob->n_targets;
  int want_s = (layers & TSQBX_ORACLE_SLP) != 0;
  int want_d = (layers & TSQBX_ORACLE_DLP) != 0;
  int want_t = (layers & TSQBX_ORACLE_SPRIME) != 0;
  if (n_threads <= 0) n_threads = omp_get_max_threads();

#pragma omp parallel for schedule(dynamic, 16) num_threads(n_threads)
  for (int64_t i = 0; i < n_out; ++i) {
    int64_t ti = sel ? sel[i] : i;
    int64_t ci = prob->target_center ? (int64_t)prob->target_center[ti] : ti;
    const double *t = prob->targets + 3 * ti;
    const double *c = prob->centers + 3 * ci;
    const double *nu_t = want_t ? prob->target_normals + 3 * ti : NULL;
    double sum[3] = {0.0, 0.0, 0.0}, sum_abs[3] = {0.0, 0.0, 0.0};
    for (int64_t j = prob->list_offsets[ci]; j < prob->list_offsets[ci + 1]; ++j) {
      int64_t y = prob->list_sources[j];
      double q = prob->weights[y] * sigma[y];
      double k[6];
      tsqbx_oracle_pair(t, c, prob->sources + 3 * y,
                        want_d ? prob->normals + 3 * y : NULL, nu_t, p, k);
      if (want_s) {
        sum[0] += q * k[0];
        sum_abs[0] += fabs(q) * k[2];
      }
      if (want_d) {
        sum[1] += q * k[1];
        sum_abs[1] += fabs(q) * k[3];
      }
      if (want_t) {
        sum[2] += q * k[4];
        sum_abs[2] += fabs(q) * k[5];
      }
    }
    const int want[3] = {want_s, want_d, want_t};
    for (int l = 0; l < 3; ++l) {
      if (!want[l]) continue;
      if (out[l]) out[l][i] = sum[l];
      if (abs[l]) abs[l][i] = sum_abs[l];
    }
  }
  return 0;
}
