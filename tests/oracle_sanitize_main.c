/* Driver for the sanitizer build of the oracle: every entry point of
 * oracle/pfr_oracle.h on small inputs, including the degenerate ones (empty
 * and one-element vectors, zero, negative and non-finite weights, bad
 * offspring counts, out-of-range ancestors, a trial cap).  Built with
 * AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py;
 * any report aborts the run.  Returns 0 when every call returned. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pfr_oracle.h"

#define N_MAX 600

static double w[N_MAX], r[N_MAX], p[N_MAX], u[N_MAX], wout[N_MAX];
static int32_t a[N_MAX], c[N_MAX], d[N_MAX], o[N_MAX], B[8], segs[8];
static uint32_t trials[N_MAX];

static void fill_weights(int64_t n, int kind) {
  for (int64_t i = 0; i < n; ++i) {
    const double x = (double)((i * 7919) % 1000) / 250.0 - 2.0;
    w[i] = exp(-0.5 * (x - 1.0) * (x - 1.0));
    if (kind == 1) w[i] = 0.0;                       /* all zero */
    if (kind == 2 && i == n / 2) w[i] = NAN;          /* non-finite */
    if (kind == 3 && i == n / 3) w[i] = -1.0;         /* negative */
    if (kind == 4) w[i] = (double)(i % 5) * 0x1p-1074; /* subnormal */
  }
}

static void resamplers(int64_t n) {
  uint32_t fl = 0;
  orc_resample_metropolis(w, n, 17, 3, 1, 2, a);
  orc_resample_rejection(w, n, 1.0, 64, 3, 1, 2, a, trials, &fl);
  orc_resample_rejection(w, n, 1e6, 4, 3, 1, 2, a, NULL, &fl); /* trial cap */
  orc_resample_partial_rejection(w, n, 0.5, 64, 3, 1, 2, a, wout, &fl);
  orc_resample_stratified(w, n, 3, 1, 2, a, r, &fl);
  orc_stratum_offsets(n, 3, 1, 2, u);
  orc_stratified_u(w, n, u, a, r, &fl);
  orc_resample_systematic(w, n, 3, 1, 2, a, r, &fl);
  orc_resample_multinomial(w, n, 3, 1, 2, a, r, p, &fl);
  orc_resample_multinomial_iid(w, n, 3, 1, 2, a, r, p, &fl);
  for (int64_t i = 0; i < n; ++i) p[i] = (double)i;
  orc_multinomial_points(w, n, p, a, &fl);
  orc_resample_metropolis_mt(w, n, 9, 3, 1, 2, a, 3);
  orc_resample_rejection_mt(w, n, 1.0, 64, 3, 1, 2, a, trials, &fl, 3);
  double ess = 0.0;
  orc_ess(w, n, &ess, &fl);
}

int main(void) {
  uint32_t fl = 0;
  /* Philox at several round counts */
  const uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  for (int k = 1; k <= 16; ++k) orc_philox4x32_r(ctr, key, k, out);
  orc_set_philox_rounds(7);
  orc_set_philox_rounds(10);
  (void)orc_u_accept(0xFFFFFFFFu);
  (void)orc_index(0xFFFFFFFFu, 0xFFFFFFFFu, 1000);
  (void)orc_accept(1.0, 0x1p-1074, 0.0);
  (void)orc_systematic_offset(1, 2, 3);
  (void)orc_threads(2);

  const int64_t sizes[] = {0, 1, 2, 5, 257, N_MAX};
  for (size_t s = 0; s < sizeof(sizes) / sizeof(sizes[0]); ++s)
    for (int kind = 0; kind <= 4; ++kind) {
      fill_weights(sizes[s], kind);
      resamplers(sizes[s]);
    }

  /* ragged batch of three vectors, every operation */
  fill_weights(N_MAX, 0);
  const int64_t off[4] = {0, 1, 300, N_MAX};
  for (int f = 0; f < 3; ++f) B[f] = 5 + f, segs[f] = f;
  for (int op = 0; op <= 4; ++op)
    orc_batch_mt(op, w, off, segs, 3, B, 1.0, 7, 2, 1, a, r, p, &fl, 2);

  /* offspring <-> ancestors, with counts that do not sum to n */
  for (int64_t n = 0; n <= 9; ++n) {
    for (int64_t i = 0; i < n; ++i) o[i] = (int32_t)((i * 3) % 4);
    orc_offspring_to_ancestors(o, n, a, &fl);
    orc_ancestors_to_offspring(a, n, o, &fl);
  }
  /* permutation, with out-of-range ancestors */
  for (int64_t n = 0; n <= 64; ++n) {
    for (int64_t i = 0; i < n; ++i) a[i] = (int32_t)((i * 5 + 3) % (n + 2)) - 1;
    orc_permute(a, n, c, d, &fl);
    orc_permute(a, n, c, NULL, &fl);
    memcpy(d, a, (size_t)n * sizeof(int32_t));
    for (int64_t i = 0; i < n; ++i)
      if (d[i] < 0 || d[i] >= n) d[i] = (int32_t)i;
    orc_permute_serial(d, n);
    double x_in[64 * 3], x_out[64 * 3];
    for (int64_t i = 0; i < 3 * n; ++i) x_in[i] = (double)i;
    orc_copy_rows(c, n, 3, x_in, x_out, &fl);
  }

  /* the bootstrap filter and the Kalman value */
  enum { F = 3, NP = 50 };
  float x[F * NP], wf[F * NP];
  double lz[F] = {0, 0, 0}, y[4] = {0.1, -0.3, 0.7, 1.2};
  int32_t Bf[F], cf[F * NP];
  orc_lgssm_init(F, NP, 2.3, 1, 0, 0, x);
  for (int i = 0; i < F * NP; ++i) cf[i] = i % NP;
  for (uint32_t t = 1; t <= 4; ++t)
    orc_lgssm_move(F, NP, 0.9, 1.0, 0.5, t, y[t - 1], 1, 0, 0, cf, x, wf, lz, Bf);
  (void)orc_normal(1, 2, ORC_DOM_INIT, 0, 0, 0);
  (void)orc_kalman_loglik(y, 4, 0.9, 1.0, 0.5, 2.3);
  printf("oracle sanitizer driver: done\n");
  return 0;
}
