/*
 * Plain FP64 CPU oracle for target-specific QBX (TSQBX) near-field evaluation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include,
 * link or call this code; only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg use it.  It shares no source with the GPU path.
 *
 * What it computes (Wala & Kloeckner, "Optimization of fast algorithms for
 * global quadrature by expansion using target-specific expansions"):
 *
 *   single layer, eq. (tsqbx) of Sec. 2.7 and the first formula of App. A:
 *     G^(p)(t, s) = 1/(4 pi) sum_{n=0..p} |t-c|^n / |s-c|^{n+1} P_n(cos gamma),
 *     gamma the angle between t-c and s-c about the QBX center c;
 *
 *   double layer, App. A (gradient of G^(p) with respect to the source s),
 *   dotted with the outward unit normal nu at s:
 *     nu . grad_s G^(p)(t, s) = 1/(4 pi) sum_{n=0..p} |t-c|^n / |s-c|^{n+2}
 *        [ -(n+1) (nu . s_hat) P_n(x) + (nu . t_hat - (nu . s_hat) x) P_n'(x) ],
 *     x = cos gamma, s_hat = (s-c)/|s-c|, t_hat = (t-c)/|t-c|;
 *
 *   potentials at each target t with center c = c(t), summed over the sources
 *   y of the center's near-field list L(c) (the QBX near field of
 *   Algorithm 1, stages 3, 5(a) and 6(a)) with strengths q_y = w_y sigma_y
 *   (the point potential of eq. (pt-pot)):
 *     out_slp[t] = sum_{y in L(c)} w_y sigma_y G^(p)(t, y)
 *     out_dlp[t] = sum_{y in L(c)} w_y sigma_y nu_y . grad_y G^(p)(t, y)
 *
 * P_n comes from Bonnet's three-term recurrence and P_n' from
 * P_{n+1}' = x P_n' + (n+1) P_n (the recurrences the paper cites from the
 * DLMF).  Sums run sequentially in list order in plain IEEE FP64, so results do
 * not depend on the thread count.
 *
 * Readings where the paper is silent: when t = c the angle is undefined and
 * only the n = 0 term survives (t_hat is taken as 0); an empty list gives 0;
 * a repeated index is summed as often as it is listed.  |s - c| = 0 is not a
 * valid input.
 *
 * abs_* receive rounding-error yardsticks: for the single layer
 * 1/(4 pi) sum_y |w_y sigma_y| sum_n |term_n|; for the double layer the same
 * sum with each term replaced by |nu| times the length of the gradient term
 * |t-c|^n/|s-c|^{n+2} [ (n+1) |P_n| + |P_n'| |t_hat - s_hat x| ], since the
 * rounding of a projection nu . g scales with |nu| |g| and not with |nu . g|.
 */
#ifndef TSQBX_ORACLE_H
#define TSQBX_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int64_t n_sources;
  const double *sources;       /* [n_sources][3] */
  const double *weights;       /* [n_sources] */
  const double *normals;       /* [n_sources][3], may be NULL for single layer only */
  int64_t n_centers;
  const double *centers;       /* [n_centers][3] */
  const int64_t *list_offsets; /* [n_centers + 1] */
  const int32_t *list_sources; /* [list_offsets[n_centers]] */
  int64_t n_targets;
  const double *targets;       /* [n_targets][3] */
  const int32_t *target_center;/* [n_targets], NULL: target i uses center i */
} tsqbx_oracle_problem;

enum { TSQBX_ORACLE_SLP = 1u, TSQBX_ORACLE_DLP = 2u };

/* One source/target pair: k[0] = G^(p), k[1] = nu . grad_s G^(p),
 * k[2], k[3] = the matching sums of absolute term values (all including
 * the 1/(4 pi) factor).  nu may be NULL (k[1] = k[3] = 0). */
void tsqbx_oracle_pair(const double t[3], const double c[3], const double s[3],
                       const double *nu, int p, double k[4]);

/* Potentials at every target (sel == NULL) or at the n_sel targets listed in
 * sel (outputs then have n_sel entries).  Any output pointer may be NULL.
 * Returns 0, or -1 on invalid arguments.  n_threads <= 0: OpenMP default. */
int tsqbx_oracle_eval(const tsqbx_oracle_problem *prob, int p, unsigned layers,
                      const double *sigma, int64_t n_sel, const int64_t *sel,
                      double *out_slp, double *out_dlp, double *abs_slp,
                      double *abs_dlp, int n_threads);

/* Threads OpenMP would use for n_threads <= 0. */
int tsqbx_oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
