/*
 * Driver that runs the oracle (test infrastructure) under AddressSanitizer and
 * UndefinedBehaviorSanitizer on the CPU: every stage of the force pass on
 * small random and degenerate inputs (coincident bodies, zero masses, a
 * single body, deep single-child chains), the direct sum with and without
 * compensation, and the operator building blocks up to the largest order of
 * the tables.  Built and run by the CPU test suite; exits non-zero (or the
 * sanitizer aborts) on any failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "fmm_oracle.h"

static uint64_t rng_state = 0x9e3779b97f4a7c15ull;
static double urand(void) { /* splitmix64 -> [0, 1) */
  uint64_t z = (rng_state += 0x9e3779b97f4a7c15ull);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
  z ^= z >> 31;
  return (double)(z >> 11) * (1.0 / 9007199254740992.0);
}

static int run_case(int64_t n, int p, double eps_tol, int n_leaf, int mac, int m2l_kind,
                    double soft, int kind) {
  double* pos = malloc(sizeof(double) * 3 * n);
  double* mass = malloc(sizeof(double) * n);
  double* acc = malloc(sizeof(double) * 3 * n);
  double* pot = malloc(sizeof(double) * n);
  uint8_t* mask = malloc(n);
  for (int64_t i = 0; i < n; i++) {
    for (int d = 0; d < 3; d++) pos[3 * i + d] = 2.0 * urand() - 1.0;
    mass[i] = urand();
    mask[i] = (uint8_t)(i % 5 == 0);
    if (kind == 1 && i % 3 == 0) { /* coincident with the previous body */
      if (i > 0)
        for (int d = 0; d < 3; d++) pos[3 * i + d] = pos[3 * (i - 1) + d];
    }
    if (kind == 2 && i % 4 == 0) mass[i] = 0.0;
    if (kind == 3) { /* clustered on a tiny scale: long single-child chains */
      for (int d = 0; d < 3; d++) pos[3 * i + d] = 1e-9 * pos[3 * i + d];
      if (i == 0) pos[0] = 1.0;
    }
  }
  orc_ctx* c = orc_new();
  int rc = 0;
  for (int stage = ORC_STAGE_TREE; stage <= ORC_STAGE_EVAL && !rc; stage++)
    rc |= orc_run(c, n, pos, mass, soft, p, eps_tol, 1.0, 1.0, n_leaf, mac, m2l_kind, stage, NULL,
                  acc, pot);
  for (int64_t i = 0; i < n && !rc; i++) /* every output finite (coincident pairs skipped) */
    if (!(isfinite(acc[3 * i]) && isfinite(acc[3 * i + 1]) && isfinite(acc[3 * i + 2]) && isfinite(pot[i])))
      rc = 1;
  if (!rc) rc |= orc_run(c, n, pos, mass, soft, p, eps_tol, 1.0, 1.0, n_leaf, mac, m2l_kind,
                         ORC_STAGE_EVAL, mask, acc, pot);
  for (int what = ORC_KEYS; what <= ORC_SORTED_POS; what++) {
    const void* ptr = NULL;
    (void)orc_get(c, what, &ptr);
  }
  orc_free(c);
  int64_t nout = n > 3 ? n : 3;
  double* dacc = malloc(sizeof(double) * 3 * nout);
  double* dpot = malloc(sizeof(double) * nout);
  int64_t sinks[3] = {0, n / 2, n - 1};
  rc |= orc_direct(n, pos, mass, soft, n, NULL, 0, dacc, dpot);
  rc |= orc_direct(n, pos, mass, soft, 3, sinks, 1, dacc, dpot);
  free(pos); free(mass); free(acc); free(pot); free(mask); free(dacc); free(dpot);
  if (rc) fprintf(stderr, "case n=%lld p=%d kind=%d failed\n", (long long)n, p, kind);
  return rc;
}

int main(void) {
  int rc = 0;
  rc |= run_case(1, 4, 1e-6, 64, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 0);
  rc |= run_case(2, 4, 1e-6, 1, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 0);
  rc |= run_case(700, 6, 1e-6, 8, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 0);
  rc |= run_case(700, 5, 1e-4, 4, ORC_MAC_GEOMETRIC, ORC_M2L_DIRECT, 1e-3, 0);
  rc |= run_case(500, 6, 1e-6, 4, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 1);
  rc |= run_case(500, 6, 1e-6, 4, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 2);
  rc |= run_case(300, 8, 1e-7, 2, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 3);
  rc |= run_case(400, 30, 1e-9, 16, ORC_MAC_ERROR, ORC_M2L_ROTATION, 0.0, 0);
  /* building blocks at the largest order of the tables */
  int p = 30, nc = (p + 1) * (p + 2) / 2;
  double *re = malloc(sizeof(double) * nc), *im = malloc(sizeof(double) * nc);
  double *lre = malloc(sizeof(double) * nc), *lim = malloc(sizeof(double) * nc);
  double *ore = malloc(sizeof(double) * nc), *oim = malloc(sizeof(double) * nc);
  double pk[31], R[3] = {0.3, -1.2, 2.1}, d[3] = {0.01, 0.02, -0.03}, X[3] = {0.1, 0.1, -0.05};
  double pt[6] = {0.1, 0.2, 0.3, -0.1, 0.05, 0.0}, ms[2] = {1.0, 0.5}, ctr[3] = {0, 0, 0}, ph, a[3];
  orc_regular(p, 0.3, -0.2, 0.5, re, im);
  orc_irregular(p, 0.3, -0.2, 0.5, re, im);
  orc_p2m(p, 2, pt, ms, ctr, re, im);
  orc_pk(p, re, im, pk);
  orc_m2m(p, re, im, d, ore, oim);
  orc_m2l_direct(p, re, im, R, lre, lim);
  orc_m2l_rotated(p, re, im, R, lre, lim);
  orc_l2l(p, lre, lim, d, ore, oim);
  orc_l2p(p, ore, oim, X, &ph, a);
  for (int n = 0; n <= p; n++) (void)orc_swap_table(n);
  (void)orc_factorials();
  free(re); free(im); free(lre); free(lim); free(ore); free(oim);
  if (rc) fprintf(stderr, "oracle sanitizer run: a call returned an error\n");
  else printf("oracle sanitizer run: ok\n");
  return rc ? 1 : 0;
}
