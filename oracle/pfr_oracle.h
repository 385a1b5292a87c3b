/*
 * pfr_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded CPU reference for the particle-filter
 * resampling step of Murray, Lee & Jacob, "Parallel resampling in the
 * particle filter" (arXiv:1301.4019).  It exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the HIP library
 * against the paper.  Nothing in the product path may link, load or call it.
 * It shares no code with the HIP library (own Philox, own sums, own
 * comparisons).
 *
 * Conventions (0-based, see the paper's section 1.1 for the 1-based form):
 *   weights    w[0..n)  doubles (FP32 inputs are widened exactly)
 *   ancestors  a[0..n)  int32, a[i] = index of the parent of particle i
 *   offspring  o[0..n)  int32
 * Random numbers come from Philox4x32-10 with the counter layout
 *   ctr = (index, (domain << 28) | step, filter, offset), key = seed.
 *
 * Every function that has a flags argument ORs the ORC_FLAG_* bits into it
 * (it may be NULL).  Return value is 0, or -1 for invalid arguments.
 */
#ifndef PFR_ORACLE_H
#define PFR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_FLAG_ZERO_TOTAL   1u  /* total weight is zero                          */
#define ORC_FLAG_TRIAL_CAP    2u  /* a rejection lane used all its trials          */
#define ORC_FLAG_BAD_COUNTS   4u  /* offspring negative or not summing to n        */
#define ORC_FLAG_BAD_WEIGHTS  8u  /* a weight is negative, NaN or infinite         */
#define ORC_FLAG_BAD_ANCESTOR 16u /* an ancestor index lies outside [0, n)         */

#define ORC_DOM_STRATA 0u /* stratified / systematic offsets  */
#define ORC_DOM_EXP    1u /* exponential spacings (multinomial) */
#define ORC_DOM_TRIAL  2u /* Metropolis steps, rejection trials */
#define ORC_DOM_NOISE  3u /* state-space model propagation     */
#define ORC_DOM_INIT   4u /* state-space model initial state   */
#define ORC_DOM_UNIFORM 5u /* independent uniforms (Code 5)     */

/* Philox4x32 with 10 rounds (Salmon et al., SC'11). */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Philox4x32 with `rounds` rounds (1..16); 10 gives the function above. */
void orc_philox4x32_r(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4]);
/* Round count used by every draw of the oracle (default 10); -1 if out of
 * range.  For the round-count study only. */
int orc_set_philox_rounds(int rounds);

/* Canonical draws shared by definition with the HIP library.                  */
/* u in (0,1]: ((x + 1) * 2^-32); index in [0,n): floor(((x1<<32)|x0) * n / 2^64) */
double orc_u_accept(uint32_t x);
int64_t orc_index(uint32_t x0, uint32_t x1, int64_t n);
/* Exact decision u * w_k <= w_j (Metropolis, Code 2; rejection, Code 3). */
int orc_accept(double u, double w_k, double w_j);

/* Code 2 (Metropolis-Ancestors), B steps per lane. */
int orc_resample_metropolis(const double* w, int64_t n, int32_t B, uint64_t seed,
                            uint32_t filter, uint32_t offset, int32_t* a);

/* Code 3 (Rejection-Ancestors) with first proposal j = i.  trials[i] (may be
 * NULL) receives the number of trials lane i used. */
int orc_resample_rejection(const double* w, int64_t n, double w_max, uint32_t max_trials,
                           uint64_t seed, uint32_t filter, uint32_t offset, int32_t* a,
                           uint32_t* trials, uint32_t* flags);

/* Partial rejection control (section 2.2, after Liu et al. 1998): for a bound
 * v_max, the clipped weights v_i = min(w_i, v_max) are resampled by Code 3
 * with bound v_max, and particle i receives the importance weight
 * w_out[i] = w_{a_i} / v_{a_i} (computed in binary64).  Reading: v_i keeps a
 * NaN or negative w_i (which Code 3 never accepts); a lane that reaches the
 * trial cap keeps a_i = i and gets w_i / v_i, or 0 when v_i is not positive. */
int orc_resample_partial_rejection(const double* w, int64_t n, double v_max, uint32_t max_trials,
                                   uint64_t seed, uint32_t filter, uint32_t offset, int32_t* a,
                                   double* w_out, uint32_t* flags);

/* Code 7 (stratified) with explicit stratum offsets u[0..n) in [0,1).
 * r_out (may be NULL) receives the scaled prefix r_i = n W_i / W_n (rounded
 * to double from the oracle's binary128 value). */
int orc_stratified_u(const double* w, int64_t n, const double* u, int32_t* a,
                     double* r_out, uint32_t* flags);
/* Code 7 with Philox offsets (stratum m uses word m&3 of call m>>2, domain 0). */
int orc_resample_stratified(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                            uint32_t offset, int32_t* a, double* r_out, uint32_t* flags);
/* Code 8 (systematic): one offset, word 0 of call 0, domain 0. */
int orc_resample_systematic(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                            uint32_t offset, int32_t* a, double* r_out, uint32_t* flags);
/* The systematic offset the canonical draw produces (for tests). */
double orc_systematic_offset(uint64_t seed, uint32_t filter, uint32_t offset);
/* The stratum offsets the canonical draw produces (for tests). */
void orc_stratum_offsets(int64_t n, uint64_t seed, uint32_t filter, uint32_t offset, double* u);

/* Code 5 (multinomial) driven by sorted uniforms from exponential spacings:
 * E_k (k = 0..n) from word k&3 of call k>>2, domain 1; p_k = n S_k / S_n for
 * k < n; a[k] = #{ i < n-1 : r_i <= p_k }.  p_out (may be NULL) gets p. */
int orc_resample_multinomial(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                             uint32_t offset, int32_t* a, double* r_out, double* p_out,
                             uint32_t* flags);
/* Code 5 as printed: particle i draws its own uniform and searches the
 * prefix.  u_i = m 2^-53 with m = (word 0 >> 11) 2^32 + word 1 of Philox call
 * (i, UNIFORM<<28, filter, offset), p_i = n u_i rounded to binary64, and
 * a[i] = #{k < n-1 : r_k <= p_i}.  The output is not sorted.  p_out (may be
 * NULL) gets p. */
int orc_resample_multinomial_iid(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                                 uint32_t offset, int32_t* a, double* r_out, double* p_out,
                                 uint32_t* flags);
/* The same search with caller-given sorted points p[0..n) in [0,n]. */
int orc_multinomial_points(const double* w, int64_t n, const double* p, int32_t* a,
                           uint32_t* flags);

/* Code 11 (Cumulative-Offspring-to-Ancestors) on offspring counts. */
int orc_offspring_to_ancestors(const int32_t* o, int64_t n, int32_t* a, uint32_t* flags);
/* Code 12 (Ancestors-to-Offspring). */
int orc_ancestors_to_offspring(const int32_t* a, int64_t n, int32_t* o, uint32_t* flags);

/* Effective sample size Sum(w)^2 / w^T w (section 3.4, after Liu 1995),
 * both sums in binary128.  An empty or all-zero vector gives 0 (all-zero
 * raises ORC_FLAG_ZERO_TOTAL); a negative or non-finite weight gives NaN and
 * ORC_FLAG_BAD_WEIGHTS. */
int orc_ess(const double* w, int64_t n, double* ess, uint32_t* flags);

/* The copy step of section 2.3 written out of place: x_out row i is x_in row
 * c_i when c_i != i, else x_in row i (rows of `dim` doubles).  It reads only
 * slots that are not written when c satisfies the in-place predicate of
 * section 2.3 (c_{c_i} = c_i for every copied i).  Reading for other input: a
 * particle whose c_i lies outside [0, n), or whose source slot is itself
 * overwritten (c_{c_i} != c_i), keeps its own row and ORC_FLAG_BAD_ANCESTOR is
 * raised. */
int orc_copy_rows(const int32_t* c, int64_t n, int64_t dim, const double* x_in, double* x_out,
                  uint32_t* flags);

/* All-cores legs: the serial functions above run over disjoint lane ranges
 * (or vectors) on `nthreads` host threads (<= 0: every core OpenMP sees),
 * with the serial result bit for bit.  For timing the oracle on the host's
 * cores and for large test cases. */
int orc_threads(int requested);
int orc_resample_metropolis_mt(const double* w, int64_t n, int32_t B, uint64_t seed,
                               uint32_t filter, uint32_t offset, int32_t* a, int nthreads);
int orc_resample_rejection_mt(const double* w, int64_t n, double w_max, uint32_t max_trials,
                              uint64_t seed, uint32_t filter, uint32_t offset, int32_t* a,
                              uint32_t* trials, uint32_t* flags, int nthreads);
/* One resampler per listed vector of a ragged batch (vector f = positions
 * [off[f], off[f+1]), filter id filter_base + f, local ancestors); op 0..4 =
 * multinomial, stratified, systematic, Metropolis (B[f]), rejection (w_max,
 * trial cap 2^20).  r_out / p_out (may be NULL) as for the single calls. */
int orc_batch_mt(int op, const double* w, const int64_t* off, const int32_t* segs, int32_t n_segs,
                 const int32_t* B, double w_max, uint64_t seed, uint32_t filter_base,
                 uint32_t offset, int32_t* a, double* r_out, double* p_out, uint32_t* flags,
                 int nthreads);

/* Code 10 (Prepermute + Permute); c receives the permuted ancestry, d (may be
 * NULL) the final claim vector (n = unclaimed). */
int orc_permute(const int32_t* a, int64_t n, int32_t* c, int32_t* d, uint32_t* flags);
/* Code 9 (serial in-place Permute), used only as an invariant cross-check. */
int orc_permute_serial(int32_t* a, int64_t n);

/* ---------------------------------------------------------------------- */
/* Bootstrap filter on the 1-D linear-Gaussian model (Code 1 with K_t the   */
/* transition density and G_t the observation density):                   */
/*   x_0 ~ N(0, s0^2),  x_t = phi x_{t-1} + q e_t,  y_t = x_t + r v_t.      */
/* Filter f holds particles [f n, (f+1) n).  Normals come from Philox words */
/* 0 and 1 by the Box-Muller transform (u1 = (x0+1) 2^-32, u2 = x1 2^-32).  */
/* ---------------------------------------------------------------------- */

/* Standard normal of the canonical draw (index, domain, step, filter, offset). */
double orc_normal(uint64_t seed, uint32_t index, uint32_t domain, uint32_t step,
                  uint32_t filter, uint32_t offset);

/* x_0 of every particle (binary32, as the state is stored). */
void orc_lgssm_init(int32_t n_filters, int32_t n, double s0, uint64_t seed, uint32_t offset,
                    uint32_t filter_base, float* x);

/* One step t after resampling, for every filter: the in-place copy
 * x_i <- x_{c_i} (c the permuted ancestry), propagation with noise
 * (i, NOISE<<28 | t, filter_base + f, offset), the log-weights
 * lw_i = log N(y_t; x_i, r^2), log_z[f] += m + log(mean exp(lw - m)) with
 * m = max lw, w_i = exp(lw_i - m) (binary32) and
 * B[f] = ceil(log(1/100) / log(1 - mean w)) clamped to [1, 65536]. */
void orc_lgssm_move(int32_t n_filters, int32_t n, double phi, double q, double r, uint32_t t,
                    double y_t, uint64_t seed, uint32_t offset, uint32_t filter_base,
                    const int32_t* c, float* x, float* w, double* log_z, int32_t* B);

/* Exact log p(y_1..y_T) of the model by the Kalman filter (binary64). */
double orc_kalman_loglik(const double* y, int64_t T, double phi, double q, double r, double s0);

#ifdef __cplusplus
}
#endif
#endif
