/* Test driver: runs the C oracle on a problem read from a binary file, so
 * that a build with AddressSanitizer and UndefinedBehaviorSanitizer can
 * check the oracle's memory accesses (tests/test_oracle_sanitize.py).
 *
 * Input (little-endian): int64 N, M, T, nnz, p, layers, n_threads, then
 * sources[N*3], weights[N], normals[N*3], centers[M*3], offsets[M+1] (int64),
 * lists[nnz] (int32), targets[T*3], target_center[T] (int32),
 * target_normals[T*3], sigma[N] (doubles unless stated).
 * Output: out_slp, out_dlp, out_sprime, abs_slp, abs_dlp, abs_sprime, [T]
 * doubles each. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "tsqbx_oracle.h"

static void *read_n(FILE *f, size_t n, size_t sz) {
  void *p = malloc(n * sz > 0 ? n * sz : 1);
  if (!p || fread(p, sz, n, f) != n) {
    fprintf(stderr, "short read\n");
    exit(2);
  }
  return p;
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t h[7];
  if (fread(h, sizeof h[0], 7, f) != 7) return 2;
  const int64_t N = h[0], M = h[1], T = h[2], nnz = h[3];
  const int p = (int)h[4], n_threads = (int)h[6];
  const unsigned layers = (unsigned)h[5];
  double *src = read_n(f, 3 * N, 8), *w = read_n(f, N, 8), *nrm = read_n(f, 3 * N, 8);
  double *ctr = read_n(f, 3 * M, 8);
  int64_t *off = read_n(f, M + 1, 8);
  int32_t *lst = read_n(f, nnz, 4);
  double *tgt = read_n(f, 3 * T, 8);
  int32_t *tc = read_n(f, T, 4);
  double *tn = read_n(f, 3 * T, 8), *sigma = read_n(f, N, 8);
  fclose(f);
  tsqbx_oracle_problem pr = {N, src, w, nrm, M, ctr, off, lst, T, tgt, tc, tn};
  double *res = calloc(6 * (size_t)(T > 0 ? T : 1), sizeof(double));
  double *const out[3] = {res, res + T, res + 2 * T};
  double *const abs_[3] = {res + 3 * T, res + 4 * T, res + 5 * T};
  const int rc = tsqbx_oracle_eval(&pr, p, layers, sigma, 0, NULL, out, abs_, n_threads);
  if (rc != 0) return 3;
  FILE *o = fopen(argv[2], "wb");
  if (!o || fwrite(res, sizeof(double), 6 * (size_t)T, o) != 6 * (size_t)T) return 4;
  fclose(o);
  free(src); free(w); free(nrm); free(ctr); free(off); free(lst); free(tgt); free(tc); free(tn);
  free(sigma); free(res);
  return 0;
}
