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
 *   normal derivative of the single layer at the target (S', App. A,
 *   gradient of G^(p) with respect to the target t), dotted with the unit
 *   normal nu_t at t:
 *     nu_t . grad_t G^(p)(t, s) = 1/(4 pi) sum_{n=1..p} |t-c|^(n-1) / |s-c|^{n+1}
 *        [ n (nu_t . t_hat) P_n(x) + (nu_t . s_hat - (nu_t . t_hat) x) P_n'(x) ];
 *
 *   potentials at each target t with center c = c(t), summed over the sources
 *   y of the center's near-field list L(c) (the QBX near field of
 *   Algorithm 1, stages 3, 5(a) and 6(a)) with strengths q_y = w_y sigma_y
 *   (the point potential of eq. (pt-pot)):
 *     out_slp[t] = sum_{y in L(c)} w_y sigma_y G^(p)(t, y)
 *     out_dlp[t] = sum_{y in L(c)} w_y sigma_y nu_y . grad_y G^(p)(t, y)
 *     out_sp[t]  = sum_{y in L(c)} w_y sigma_y nu_t . grad_t G^(p)(t, y)
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
 * rounding of a projection nu . g scales with |nu| |g| and not with |nu . g|;
 * for S' likewise |nu_t| |t-c|^(n-1)/|s-c|^{n+1} [ n |P_n| + |P_n'| |s_hat - t_hat x| ].
 * At t = c the reading t_hat = 0 leaves S' its n = 1 term, nu_t . s_hat / |s-c|^2,
 * which is the limit of App. A's sum.
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
  const double *target_normals;/* [n_targets][3], may be NULL unless S' is asked for */
} tsqbx_oracle_problem;

enum { TSQBX_ORACLE_SLP = 1u, TSQBX_ORACLE_DLP = 2u, TSQBX_ORACLE_SPRIME = 4u };

/* One source/target pair: k[0] = G^(p), k[1] = nu . grad_s G^(p),
 * k[2], k[3] = the matching sums of absolute term values, k[4] =
 * nu_t . grad_t G^(p), k[5] its yardstick (all including the 1/(4 pi)
 * factor).  nu may be NULL (k[1] = k[3] = 0), nu_t may be NULL
 * (k[4] = k[5] = 0). */
void tsqbx_oracle_pair(const double t[3], const double c[3], const double s[3],
                       const double *nu, const double *nu_t, int p, double k[6]);

/* Potentials at every target (sel == NULL) or at the n_sel targets listed in
 * sel (outputs then have n_sel entries).  out[0..2] receive the single layer,
 * double layer and S', abs[0..2] their yardsticks; any entry may be NULL.
 * Returns 0, or -1 on invalid arguments (DLP without source normals, S'
 * without target normals).  n_threads <= 0: OpenMP default. */
int tsqbx_oracle_eval(const tsqbx_oracle_problem *prob, int p, unsigned layers,
                      const double *sigma, int64_t n_sel, const int64_t *sel,
                      double *const out[3], double *const abs[3], int n_threads);

/* Threads OpenMP would use for n_threads <= 0. */
int tsqbx_oracle_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
