/*
 * Runs the FP64 oracle on a few small problems, for a build under the
 * address and undefined-behaviour sanitizers (tests/test_oracle_sanitize.py).
 * Each problem must launch and terminate every photon and satisfy the
 * ledger identity launched + roulette gain = absorbed + escaped + timed out
 * + roulette loss + capped.  Prints "ok" and exits 0, or reports and exits 1.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../oracle/mcx_oracle.h"

static int check(const char *name, const orc_problem *p, uint64_t n, uint64_t seed) {
  const size_t nvox = (size_t)p->nx * p->ny * p->nz;
  double *tally = calloc(nvox * p->ngates, sizeof(double));
  int64_t *dep = calloc(nvox * p->ngates, sizeof(int64_t));
  const uint64_t cap = 64;
  float *rec = calloc(cap * (size_t)(4 + p->nmedia - 1), sizeof(float));
  uint64_t *rec_ph = calloc(cap, sizeof(uint64_t));
  double *dig = calloc(16 * ORC_DG_N, sizeof(double));
  orc_output o;
  memset(&o, 0, sizeof o);
  o.tally = tally;
  o.deposits = dep;
  o.det_rec = rec;
  o.det_photon = rec_ph;
  o.det_cap = cap;
  o.digest = dig;
  o.ndigest = 16;
  int bad = 0;
  if (orc_run(p, 0, n, seed, 2, &o) != ORC_OK) {
    printf("%s: orc_run failed\n", name);
    bad = 1;
  } else {
    const int64_t *c = o.counts;
    const double *L = o.ledger;
    const int64_t ended = c[ORC_CNT_ESCAPED] + c[ORC_CNT_TIMEOUT] + c[ORC_CNT_RR_DEAD] +
                          c[ORC_CNT_CAPPED];
    const double lhs = L[ORC_LEDGER_LAUNCHED] + L[ORC_LEDGER_RR_GAIN];
    const double rhs = L[ORC_LEDGER_ABSORBED] + L[ORC_LEDGER_ESCAPED] + L[ORC_LEDGER_TIMEOUT] +
                       L[ORC_LEDGER_RR_LOSS] + L[ORC_LEDGER_CAPPED];
    if (c[ORC_CNT_LAUNCHED] != (int64_t)n || ended != (int64_t)n) {
      printf("%s: launched %lld ended %lld of %llu\n", name, (long long)c[ORC_CNT_LAUNCHED],
             (long long)ended, (unsigned long long)n);
      bad = 1;
    }
    if (fabs(lhs - rhs) > 1e-9 * (double)n) {
      printf("%s: ledger %.17g != %.17g\n", name, lhs, rhs);
      bad = 1;
    }
  }
  free(tally);
  free(dep);
  free(rec);
  free(rec_ph);
  free(dig);
  return bad;
}

int main(void) {
  int bad = 0;
  /* 8^3 cube with a 2^3 inclusion of a different index, reflection on,
   * two detectors, five gates */
  {
    uint8_t lab[512];
    for (int i = 0; i < 512; ++i) lab[i] = 1;
    for (int k = 3; k < 5; ++k)
      for (int j = 3; j < 5; ++j)
        for (int i = 3; i < 5; ++i) lab[i + 8 * (j + 8 * k)] = 2;
    const double media[] = {0, 0, 1, 1, 0.01, 1.0, 0.5, 1.37, 0.05, 5.0, 0.9, 1.5};
    const double det[] = {2.0, 4.0, 0.0, 1.0, 6.0, 4.0, 0.0, 1.0};
    orc_problem p = {8, 8, 8, 1.0, lab, 3, media, {3.5, 3.5, 0.0}, {0, 0, 1}, 2, det,
                     0.0, 0.2, 5, 1, 1.0, 1e-4, 10.0, 0};
    bad |= check("inclusion", &p, 3000, 1);
  }
  /* strongly absorbing slab: roulette, a short gate and an event cap */
  {
    uint8_t lab[5 * 5 * 3];
    for (int i = 0; i < 75; ++i) lab[i] = 1;
    const double media[] = {0, 0, 1, 1, 2.0, 20.0, 0.8, 1.37};
    orc_problem p = {5, 5, 3, 0.5, lab, 2, media, {1.25, 1.25, 0.0}, {0, 0, 1}, 0, NULL,
                     0.0, 0.01, 3, 1, 1.0, 1e-4, 10.0, 200};
    bad |= check("roulette", &p, 2000, 7);
  }
  /* one voxel, index matched, no reflection */
  {
    uint8_t lab[1] = {1};
    const double media[] = {0, 0, 1, 1, 0.1, 1.0, 0.0, 1.0};
    orc_problem p = {1, 1, 1, 1.0, lab, 2, media, {0.5, 0.5, 0.0}, {0, 0, 1}, 0, NULL,
                     0.0, 5.0, 1, 0, 1.0, 1e-4, 10.0, 0};
    bad |= check("voxel", &p, 1000, 3);
  }
  if (!bad) printf("ok\n");
  return bad;
}
