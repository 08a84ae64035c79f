/* Drives the oracle through every operator, function, base scheme and the
 * shuffle under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only;
 * built and run by test_oracle_sanitized.py).  Exit status 0 = clean. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../oracle/oracle.h"

static int run_case(int64_t N, int64_t D, int xo, int fn, int dtype, int base, int shuffle,
                    double CR, int gens) {
  double* rot = NULL;
  if (fn == OR_FN_ELLIPSOID_ROT) { /* a permutation matrix is orthogonal */
    rot = (double*)calloc((size_t)(D * D), sizeof(double));
    for (int64_t k = 0; k < D; ++k) rot[k * D + (k * 7 + 3) % D] = 1.0;
  }
  oracle_desc d = {0};
  d.N = N; d.D = D; d.F = 0.6; d.CR = CR; d.xo = xo; d.fn = fn; d.dtype = dtype; d.run = 2;
  d.lo = -5.0; d.hi = 5.0; d.olo = -1.0; d.ohi = 1.0; d.seed = 12345u; d.rot = rot;
  d.base = base; d.shuffle = shuffle;
  oracle_state* s = oracle_create(&d);
  if (!s) { free(rot); return 1; }
  int64_t* ti = (int64_t*)malloc(sizeof(int64_t) * 6 * N);
  uint8_t* tm = (uint8_t*)malloc((size_t)(N * D));
  double* tt = (double*)malloc(sizeof(double) * N * D);
  double* tf = (double*)malloc(sizeof(double) * N);
  double* pop = (double*)malloc(sizeof(double) * N * D);
  double* fit = (double*)malloc(sizeof(double) * N);
  int bad = oracle_generation(s, gens, ti, tm, tt, tf);
  int64_t g = 0;
  oracle_get_state(s, pop, fit, &g);
  int64_t idx6[6];
  oracle_individual(s, pop, g + 1, N - 1, idx6, tm, tt, tf);
  double bf; int64_t bi, bg;
  oracle_get_best(s, &bf, &bi, &bg, tt);
  oracle_set_state(s, pop, fit, g, bf, bi, bg);
  bad |= oracle_generation(s, 2, NULL, NULL, NULL, NULL);
  oracle_destroy(s);
  free(ti); free(tm); free(tt); free(tf); free(pop); free(fit); free(rot);
  return bad;
}

int main(void) {
  int bad = 0;
  const int64_t Ds[] = {1, 2, 7, 33};
  for (int xo = 0; xo <= 2; ++xo)
    for (int fn = 0; fn <= 5; ++fn)
      for (int k = 0; k < 4; ++k) {
        const int64_t D = (fn == OR_FN_ELLIPSOID_ROT && Ds[k] < 2) ? 2 : Ds[k];
        bad |= run_case(9, D, xo, fn, k % 2, k, k >= 2, k == 3 ? 1.0 : 0.7, 3);
      }
  for (int base = 0; base <= 3; ++base) bad |= run_case(4, 5, 2, 1, 0, base, 1, 0.0, 4);
  /* building blocks on their own */
  uint8_t m[40];
  for (int64_t L = 0; L <= 10; ++L) {
    oracle_alg9_mask(10, 7, L, m);
    oracle_alg10_mask(10, 7, L, m);
  }
  for (int64_t n = 4; n < 70; ++n)
    for (int64_t k = 0; k < n; ++k) bad |= oracle_permute(1, 0, OR_TAG_PERM, 3, n, k) >= n;
  bad |= oracle_nec_length(0.5, 0.0, 10) != 1;
  printf("%s\n", bad ? "FAIL" : "ok");
  return bad;
}
