/*
 * pfr_oracle.c -- TEST INFRASTRUCTURE ONLY (see pfr_oracle.h).
 *
 * Plain CPU reference for the resampling step of Murray, Lee & Jacob,
 * "Parallel resampling in the particle filter" (arXiv:1301.4019).  Each
 * function follows one of the paper's Code listings in its own order and
 * notation, translated to 0-based indices.  Readings of the places where the
 * paper is silent or ambiguous are noted at each function.
 *
 * Precision.  Sums that the paper writes as Inclusive-Prefix-Sum (appendix A,
 * Code 4) are accumulated sequentially in IEEE binary128 (__float128), which is
 * monotone for non-negative terms and accurate to ~2^-113 relative, so that
 * the oracle stands in for the exact real-number definition.  Accept/reject
 * decisions u*w_k <= w_j are made on exact binary128 products (a 32-bit u times
 * a 53-bit weight needs 85 bits).  Nothing here is tuned for speed.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fPIC -shared (no -ffast-math).
 */
#include "pfr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef __float128 q128;

/* ------------------------------------------------------------------------ */
/* Philox4x32-10.  Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as  */
/* easy as 1, 2, 3", SC'11: each round multiplies counter words 0 and 2 by    */
/* fixed odd constants, takes the 64-bit products apart into high and low     */
/* halves, and mixes the high halves with the other two counter words and the */
/* round key; the key is bumped by two Weyl constants between rounds.         */
/* ------------------------------------------------------------------------ */
void orc_philox4x32_r(const uint32_t ctr[4], const uint32_t key[2], int rounds, uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    int round;
    for (round = 0; round < rounds; ++round) {
        uint64_t p0, p1;
        uint32_t y0, y1, y2, y3;
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        p0 = (uint64_t)M0 * (uint64_t)x0;
        p1 = (uint64_t)M1 * (uint64_t)x2;
        y0 = (uint32_t)(p1 >> 32) ^ x1 ^ k0;
        y1 = (uint32_t)p1;
        y2 = (uint32_t)(p0 >> 32) ^ x3 ^ k1;
        y3 = (uint32_t)p0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    orc_philox4x32_r(ctr, key, 10, out);
}

/* Round count of every draw below: 10 (Philox4x32-10) unless a round-count
 * study sets another. */
static int g_rounds = 10;

int orc_set_philox_rounds(int rounds)
{
    if (rounds < 1 || rounds > 16) return -1;
    g_rounds = rounds;
    return 0;
}

static void draw(uint64_t seed, uint32_t index, uint32_t domain, uint32_t step,
                 uint32_t filter, uint32_t offset, uint32_t out[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = index;
    ctr[1] = (domain << 28) | (step & 0x0FFFFFFFu);
    ctr[2] = filter;
    ctr[3] = offset;
    key[0] = (uint32_t)seed;
    key[1] = (uint32_t)(seed >> 32);
    orc_philox4x32_r(ctr, key, g_rounds, out);
}

/* u in (0, 1]: the paper draws u ~ U[0,1] in Codes 2 and 3; the 32-bit
 * lattice excludes 0 so that a zero weight is never accepted by chance. */
double orc_u_accept(uint32_t x) { return ldexp((double)x + 1.0, -32); }

/* offsets in [0, 1) for Codes 7 and 8. */
static double u_offset(uint32_t x) { return ldexp((double)x, -32); }

/* j ~ U{0..n-1}: the high 64 bits of a 64-bit uniform times n. */
int64_t orc_index(uint32_t x0, uint32_t x1, int64_t n)
{
    unsigned __int128 r = ((unsigned __int128)(((uint64_t)x1 << 32) | x0)) * (uint64_t)n;
    return (int64_t)(r >> 64);
}

/* u * w_k <= w_j evaluated exactly: both products fit in binary128. */
int orc_accept(double u, double w_k, double w_j)
{
    q128 lhs = (q128)u * (q128)w_k;
    return lhs <= (q128)w_j;
}

/* The 32-bit words of lane i's stream in a domain: word k is word k & 3 of   */
/* the call with step k >> 2.  A one-call cache keeps the oracle from calling  */
/* Philox again for the next word of the same block.                          */
typedef struct {
    uint64_t seed;
    uint32_t index, domain, filter, offset;
    int64_t call;
    uint32_t x[4];
} word_stream;

static void ws_init(word_stream* s, uint64_t seed, uint32_t index, uint32_t domain,
                    uint32_t filter, uint32_t offset)
{
    s->seed = seed;
    s->index = index;
    s->domain = domain;
    s->filter = filter;
    s->offset = offset;
    s->call = -1;
}

static uint32_t ws_word(word_stream* s, int64_t k)
{
    if ((k >> 2) != s->call) {
        s->call = k >> 2;
        draw(s->seed, s->index, s->domain, (uint32_t)s->call, s->filter, s->offset, s->x);
    }
    return s->x[k & 3];
}

/* ------------------------------------------------------------------------ */
/* Code 2: Metropolis-Ancestors.  Each lane i runs an independent Metropolis */
/* chain started at k = i for B steps; step n proposes j uniformly and moves */
/* when u <= w_j / w_k (read as u w_k <= w_j, so a chain sitting on a zero   */
/* weight always moves).  Random numbers: step n takes words 3n, 3n+1 (for  */
/* j) and 3n+2 (for u) of lane i's stream in the trial domain, so four steps */
/* use three Philox calls.                                                   */
/* ------------------------------------------------------------------------ */
/* Lanes [i0, i1) of Code 2 on the n weights (every lane reads all of w). */
static void metropolis_lanes(const double* w, int64_t n, int32_t B, uint64_t seed,
                             uint32_t filter, uint32_t offset, int64_t i0, int64_t i1, int32_t* a)
{
    int64_t i;
    for (i = i0; i < i1; ++i) {
        int64_t k = i;
        int32_t step;
        word_stream s;
        ws_init(&s, seed, (uint32_t)i, ORC_DOM_TRIAL, filter, offset);
        for (step = 0; step < B; ++step) {
            const int64_t w0 = 3 * (int64_t)step;
            const uint32_t x0 = ws_word(&s, w0), x1 = ws_word(&s, w0 + 1);
            const uint32_t x2 = ws_word(&s, w0 + 2);
            const int64_t j = orc_index(x0, x1, n);
            const double u = orc_u_accept(x2);
            if (orc_accept(u, w[k], w[j])) k = j;
        }
        a[i] = (int32_t)k;
    }
}

int orc_resample_metropolis(const double* w, int64_t n, int32_t B, uint64_t seed,
                            uint32_t filter, uint32_t offset, int32_t* a)
{
    if (n < 0 || B < 0 || (n > 0 && (!w || !a))) return -1;
    metropolis_lanes(w, n, B, seed, filter, offset, 0, n, a);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Code 3: Rejection-Ancestors.  The first proposal is j = i; while the      */
/* proposal is rejected (u > w_j / w_max, i.e. not u w_max <= w_j) a new j   */
/* and u are drawn.  Trial t of lane i uses call (i, trial domain, t); trial */
/* 0 uses only that call's u.  A lane that rejects max_trials proposals ends */
/* with a_i = i and raises ORC_FLAG_TRIAL_CAP (the paper's loop has no cap). */
/* ------------------------------------------------------------------------ */
/* Lanes [i0, i1) of Code 3; returns the flags they raise. */
static uint32_t rejection_lanes(const double* w, int64_t n, double w_max, uint32_t max_trials,
                                uint64_t seed, uint32_t filter, uint32_t offset, int64_t i0,
                                int64_t i1, int32_t* a, uint32_t* trials)
{
    int64_t i;
    uint32_t fl = 0;
    for (i = i0; i < i1; ++i) {
        uint32_t x[4], t = 0;
        int64_t j = i;
        double u;
        int accepted;
        draw(seed, (uint32_t)i, ORC_DOM_TRIAL, 0, filter, offset, x);
        u = orc_u_accept(x[2]);
        accepted = orc_accept(u, w_max, w[j]);
        while (!accepted) {
            ++t;
            if (t >= max_trials) break;
            draw(seed, (uint32_t)i, ORC_DOM_TRIAL, t, filter, offset, x);
            j = orc_index(x[0], x[1], n);
            u = orc_u_accept(x[2]);
            accepted = orc_accept(u, w_max, w[j]);
        }
        if (!accepted) {
            j = i;
            fl |= ORC_FLAG_TRIAL_CAP;
            t = max_trials - 1;
        }
        a[i] = (int32_t)j;
        if (trials) trials[i] = t + 1;
    }
    return fl;
}

int orc_resample_rejection(const double* w, int64_t n, double w_max, uint32_t max_trials,
                           uint64_t seed, uint32_t filter, uint32_t offset, int32_t* a,
                           uint32_t* trials, uint32_t* flags)
{
    uint32_t fl;
    if (n < 0 || max_trials == 0 || (n > 0 && (!w || !a))) return -1;
    fl = rejection_lanes(w, n, w_max, max_trials, seed, filter, offset, 0, n, a, trials);
    if (flags) *flags |= fl;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Partial rejection control: Code 3 on the clipped weights, then the        */
/* importance weight of each particle's ancestor.                            */
/* ------------------------------------------------------------------------ */
int orc_resample_partial_rejection(const double* w, int64_t n, double v_max, uint32_t max_trials,
                                   uint64_t seed, uint32_t filter, uint32_t offset, int32_t* a,
                                   double* w_out, uint32_t* flags)
{
    int64_t i;
    double* v;
    int rc;
    if (n < 0 || max_trials == 0 || !(v_max > 0.0) || (n > 0 && (!w || !a || !w_out))) return -1;
    if (n == 0) return 0;
    v = (double*)malloc((size_t)n * sizeof(double));
    if (!v) return -1;
    for (i = 0; i < n; ++i) v[i] = (w[i] > v_max) ? v_max : w[i];
    rc = orc_resample_rejection(v, n, v_max, max_trials, seed, filter, offset, a, NULL, flags);
    if (rc == 0) {
        for (i = 0; i < n; ++i) {
            const double va = v[a[i]];
            w_out[i] = (va > 0.0) ? w[a[i]] / va : 0.0;
        }
    }
    free(v);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Shared pieces of the collective schemes (appendix B).                     */
/* ------------------------------------------------------------------------ */

/* Inclusive-Prefix-Sum (Code 4), sequential in binary128.  Returns the
 * weight-validity flag: any negative, NaN or infinite weight. */
static uint32_t inclusive_prefix_sum(const double* w, int64_t n, q128* W)
{
    q128 s = 0;
    int64_t i;
    uint32_t fl = 0;
    for (i = 0; i < n; ++i) {
        double x = w[i];
        if (!(x >= 0.0) || isinf(x)) fl |= ORC_FLAG_BAD_WEIGHTS;
        s += (q128)x;
        W[i] = s;
    }
    return fl;
}

/* Identity ancestry: the defined output when the weights cannot be used. */
static void identity(int64_t n, int32_t* a)
{
    int64_t i;
    for (i = 0; i < n; ++i) a[i] = (int32_t)i;
}

/* r_i = n W_i / W_n.  The quotient is formed first so that r_{n-1} = n
 * exactly and particles after the last non-zero weight also get r = n. */
static q128 scaled(q128 Wi, q128 Wn, int64_t n) { return (q128)n * (Wi / Wn); }

/* Code 11: Cumulative-Offspring-to-Ancestors with O given as int64 values
 * already clipped to [0, n] and non-decreasing. */
static void cumulative_offspring_to_ancestors(const int64_t* O, int64_t n, int32_t* a)
{
    int64_t i, j;
    for (i = 0; i < n; ++i) {
        int64_t start = (i == 0) ? 0 : O[i - 1];
        int64_t o = O[i] - start;
        for (j = 0; j < o; ++j) a[start + j] = (int32_t)i;
    }
}

/* ------------------------------------------------------------------------ */
/* Code 7: Stratified-Cumulative-Offspring, then Code 11.                    */
/*   r_i = n W_i / W_n;  m = floor(r_i) is the (0-based) stratum holding    */
/*   r_i;  O_i = min(n, floor(r_i + u_m)).                                  */
/* floor(r + u) is evaluated exactly as m + [frac(r) >= 1 - u] (frac and     */
/* 1 - u are exact in binary128), which avoids the loss of u against r that  */
/* the paper warns about for single precision.                               */
/* ------------------------------------------------------------------------ */
int orc_stratified_u(const double* w, int64_t n, const double* u, int32_t* a,
                     double* r_out, uint32_t* flags)
{
    q128* W;
    int64_t* O;
    int64_t i;
    uint32_t fl;
    if (n < 0 || (n > 0 && (!w || !u || !a))) return -1;
    if (n == 0) return 0;
    W = (q128*)malloc(sizeof(q128) * (size_t)n);
    O = (int64_t*)malloc(sizeof(int64_t) * (size_t)n);
    if (!W || !O) { free(W); free(O); return -1; }
    fl = inclusive_prefix_sum(w, n, W);
    if (!fl && !(W[n - 1] > 0)) fl |= ORC_FLAG_ZERO_TOTAL;
    if (fl) {
        identity(n, a);
        if (r_out) for (i = 0; i < n; ++i) r_out[i] = NAN;
    } else {
        for (i = 0; i < n; ++i) {
            q128 r = scaled(W[i], W[n - 1], n);
            int64_t m = (int64_t)r; /* r >= 0: truncation is floor */
            int64_t Oi;
            if (m >= n) {
                Oi = n;
            } else {
                q128 frac = r - (q128)m;
                q128 one_minus_u = (q128)1 - (q128)u[m];
                Oi = m + (frac >= one_minus_u ? 1 : 0);
                if (Oi > n) Oi = n;
            }
            O[i] = Oi;
            if (r_out) r_out[i] = (double)r;
        }
        cumulative_offspring_to_ancestors(O, n, a);
    }
    if (flags) *flags |= fl;
    free(W);
    free(O);
    return 0;
}

void orc_stratum_offsets(int64_t n, uint64_t seed, uint32_t filter, uint32_t offset, double* u)
{
    int64_t m;
    for (m = 0; m < n; ++m) {
        uint32_t x[4];
        draw(seed, (uint32_t)(m >> 2), ORC_DOM_STRATA, 0, filter, offset, x);
        u[m] = u_offset(x[m & 3]);
    }
}

int orc_resample_stratified(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                            uint32_t offset, int32_t* a, double* r_out, uint32_t* flags)
{
    double* u;
    int rc;
    if (n < 0) return -1;
    if (n == 0) return 0;
    u = (double*)malloc(sizeof(double) * (size_t)n);
    if (!u) return -1;
    orc_stratum_offsets(n, seed, filter, offset, u);
    rc = orc_stratified_u(w, n, u, a, r_out, flags);
    free(u);
    return rc;
}

/* Code 8: the systematic scheme is Code 7 with one offset shared by all
 * strata. */
double orc_systematic_offset(uint64_t seed, uint32_t filter, uint32_t offset)
{
    uint32_t x[4];
    draw(seed, 0, ORC_DOM_STRATA, 0, filter, offset, x);
    return u_offset(x[0]);
}

int orc_resample_systematic(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                            uint32_t offset, int32_t* a, double* r_out, uint32_t* flags)
{
    double* u;
    double u0;
    int64_t m;
    int rc;
    if (n < 0) return -1;
    if (n == 0) return 0;
    u = (double*)malloc(sizeof(double) * (size_t)n);
    if (!u) return -1;
    u0 = orc_systematic_offset(seed, filter, offset);
    for (m = 0; m < n; ++m) u[m] = u0;
    rc = orc_stratified_u(w, n, u, a, r_out, flags);
    free(u);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Code 5: Multinomial-Ancestors.  W = Inclusive-Prefix-Sum(w); every draw   */
/* u^k ~ U[0, W_n) is located in W.  Two readings: (1) the draws are the     */
/* order statistics of n uniforms, produced from exponential spacings, so    */
/* the ancestry comes out sorted (same law as independent draws, cf. the     */
/* sorted-uniform idea of Code 6); (2) the search returns the number of      */
/* prefix values <= the draw (upper bound) instead of Lower-Bound, so that a */
/* zero-weight particle is never selected; the count is capped at n - 1.     */
/* Both are expressed in units of r = n W / W_n.                             */
/* ------------------------------------------------------------------------ */
static int multinomial_core(const q128* W, int64_t n, const q128* p, int32_t* a)
{
    int64_t k;
    for (k = 0; k < n; ++k) {
        /* upper bound of p_k in r_0 <= ... <= r_{n-2} by bisection */
        int64_t lo = 0, hi = n - 1; /* answer in [0, n-1] */
        while (lo < hi) {
            int64_t mid = lo + (hi - lo) / 2;
            if (scaled(W[mid], W[n - 1], n) <= p[k]) lo = mid + 1;
            else hi = mid;
        }
        a[k] = (int32_t)lo;
    }
    return 0;
}

int orc_multinomial_points(const double* w, int64_t n, const double* p, int32_t* a,
                           uint32_t* flags)
{
    q128 *W, *pq;
    int64_t k;
    uint32_t fl;
    if (n < 0 || (n > 0 && (!w || !p || !a))) return -1;
    if (n == 0) return 0;
    W = (q128*)malloc(sizeof(q128) * (size_t)n);
    pq = (q128*)malloc(sizeof(q128) * (size_t)n);
    if (!W || !pq) { free(W); free(pq); return -1; }
    fl = inclusive_prefix_sum(w, n, W);
    if (!fl && !(W[n - 1] > 0)) fl |= ORC_FLAG_ZERO_TOTAL;
    if (fl) {
        identity(n, a);
    } else {
        for (k = 0; k < n; ++k) pq[k] = (q128)p[k];
        multinomial_core(W, n, pq, a);
    }
    if (flags) *flags |= fl;
    free(W);
    free(pq);
    return 0;
}

int orc_resample_multinomial(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                             uint32_t offset, int32_t* a, double* r_out, double* p_out,
                             uint32_t* flags)
{
    q128 *W, *S, *p;
    int64_t k, i;
    uint32_t fl;
    if (n < 0 || (n > 0 && (!w || !a))) return -1;
    if (n == 0) return 0;
    W = (q128*)malloc(sizeof(q128) * (size_t)n);
    S = (q128*)malloc(sizeof(q128) * (size_t)(n + 1));
    p = (q128*)malloc(sizeof(q128) * (size_t)n);
    if (!W || !S || !p) { free(W); free(S); free(p); return -1; }
    fl = inclusive_prefix_sum(w, n, W);
    if (!fl && !(W[n - 1] > 0)) fl |= ORC_FLAG_ZERO_TOTAL;
    if (fl) {
        identity(n, a);
        if (r_out) for (i = 0; i < n; ++i) r_out[i] = NAN;
        if (p_out) for (k = 0; k < n; ++k) p_out[k] = NAN;
    } else {
        /* exponential spacings E_0..E_n and their running sums S_k */
        q128 s = 0;
        for (k = 0; k <= n; ++k) {
            uint32_t x[4];
            double e;
            draw(seed, (uint32_t)(k >> 2), ORC_DOM_EXP, 0, filter, offset, x);
            e = -log(ldexp((double)x[k & 3] + 0.5, -32));
            s += (q128)e;
            S[k] = s;
        }
        /* p_k = n S_k / S_n, k = 0..n-1: order statistics of n uniforms on [0, n) */
        for (k = 0; k < n; ++k) p[k] = (q128)n * (S[k] / S[n]);
        multinomial_core(W, n, p, a);
        if (r_out) for (i = 0; i < n; ++i) r_out[i] = (double)scaled(W[i], W[n - 1], n);
        if (p_out) for (k = 0; k < n; ++k) p_out[k] = (double)p[k];
    }
    if (flags) *flags |= fl;
    free(W);
    free(S);
    free(p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Code 5 with independent uniforms: each particle draws u on [0, 1) and    */
/* takes the upper bound of n u among the scaled prefix r.                   */
/* ------------------------------------------------------------------------ */
int orc_resample_multinomial_iid(const double* w, int64_t n, uint64_t seed, uint32_t filter,
                                 uint32_t offset, int32_t* a, double* r_out, double* p_out,
                                 uint32_t* flags)
{
    q128 *W, *p;
    int64_t i;
    uint32_t fl;
    if (n < 0 || (n > 0 && (!w || !a))) return -1;
    if (n == 0) return 0;
    W = (q128*)malloc(sizeof(q128) * (size_t)n);
    p = (q128*)malloc(sizeof(q128) * (size_t)n);
    if (!W || !p) { free(W); free(p); return -1; }
    fl = inclusive_prefix_sum(w, n, W);
    if (!fl && !(W[n - 1] > 0)) fl |= ORC_FLAG_ZERO_TOTAL;
    if (fl) {
        identity(n, a);
        if (r_out) for (i = 0; i < n; ++i) r_out[i] = NAN;
        if (p_out) for (i = 0; i < n; ++i) p_out[i] = NAN;
    } else {
        for (i = 0; i < n; ++i) {
            uint32_t x[4];
            uint64_t m;
            double u, pi;
            draw(seed, (uint32_t)i, ORC_DOM_UNIFORM, 0, filter, offset, x);
            m = ((uint64_t)(x[0] >> 11) << 32) | (uint64_t)x[1]; /* 53 random bits */
            u = ldexp((double)m, -53);                            /* exact */
            pi = (double)n * u;                                   /* one rounding */
            p[i] = (q128)pi;
            if (p_out) p_out[i] = pi;
        }
        multinomial_core(W, n, p, a);
        if (r_out) for (i = 0; i < n; ++i) r_out[i] = (double)scaled(W[i], W[n - 1], n);
    }
    if (flags) *flags |= fl;
    free(W);
    free(p);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Code 11 from offspring counts: O = Inclusive-Prefix-Sum(o), then          */
/* a[O_{i-1} .. O_i) = i.  Readings for invalid input: a negative count is   */
/* used as 0; positions at or beyond n are dropped; if the counts sum to     */
/* less than n the remaining positions s keep a[s] = s.  All three raise     */
/* ORC_FLAG_BAD_COUNTS.                                                      */
/* ------------------------------------------------------------------------ */
int orc_offspring_to_ancestors(const int32_t* o, int64_t n, int32_t* a, uint32_t* flags)
{
    int64_t i, j, O = 0;
    uint32_t fl = 0;
    if (n < 0 || (n > 0 && (!o || !a))) return -1;
    for (i = 0; i < n; ++i) {
        int64_t oi = o[i];
        int64_t start = O;
        if (oi < 0) { fl |= ORC_FLAG_BAD_COUNTS; oi = 0; }
        O += oi;
        for (j = start; j < O && j < n; ++j) a[j] = (int32_t)i;
    }
    if (O != n) fl |= ORC_FLAG_BAD_COUNTS;
    for (j = O; j < n; ++j) a[j] = (int32_t)j;
    if (flags) *flags |= fl;
    return 0;
}

/* Code 12: o_{a_i} += 1 for every i (out-of-range ancestors are skipped and
 * flagged). */
int orc_ancestors_to_offspring(const int32_t* a, int64_t n, int32_t* o, uint32_t* flags)
{
    int64_t i;
    uint32_t fl = 0;
    if (n < 0 || (n > 0 && (!a || !o))) return -1;
    for (i = 0; i < n; ++i) o[i] = 0;
    for (i = 0; i < n; ++i) {
        if (a[i] < 0 || a[i] >= n) { fl |= ORC_FLAG_BAD_ANCESTOR; continue; }
        o[a[i]] += 1;
    }
    if (flags) *flags |= fl;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Effective sample size (section 3.4): the square of the weight sum over    */
/* the sum of squared weights.  Sums in binary128, so neither the squares of */
/* large binary64 weights nor the rounding of a long sum matter here.        */
/* ------------------------------------------------------------------------ */
int orc_ess(const double* w, int64_t n, double* ess, uint32_t* flags)
{
    int64_t i;
    q128 s1 = 0, s2 = 0;
    if (n < 0 || !ess || (n > 0 && !w)) return -1;
    for (i = 0; i < n; ++i) {
        if (!(w[i] >= 0.0) || isinf(w[i])) {
            if (flags) *flags |= ORC_FLAG_BAD_WEIGHTS;
            *ess = NAN;
            return 0;
        }
        s1 += (q128)w[i];
        s2 += (q128)w[i] * (q128)w[i];
    }
    if (s2 == 0) {
        if (n > 0 && flags) *flags |= ORC_FLAG_ZERO_TOTAL;
        *ess = 0.0;
        return 0;
    }
    *ess = (double)(s1 * s1 / s2);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Copy step of section 2.3, out of place (see the header for the reading of */
/* an ancestry that breaks the in-place predicate).                          */
/* ------------------------------------------------------------------------ */
int orc_copy_rows(const int32_t* c, int64_t n, int64_t dim, const double* x_in, double* x_out,
                  uint32_t* flags)
{
    int64_t i, k;
    uint32_t fl = 0;
    if (n < 0 || dim < 1 || (n > 0 && (!c || !x_in || !x_out))) return -1;
    for (i = 0; i < n; ++i) {
        int64_t src = i;
        if (c[i] != i) {
            if (c[i] < 0 || c[i] >= n || c[c[i]] != c[i]) fl |= ORC_FLAG_BAD_ANCESTOR;
            else src = c[i];
        }
        for (k = 0; k < dim; ++k) x_out[i * dim + k] = x_in[src * dim + k];
    }
    if (flags) *flags |= fl;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Code 10: Prepermute then Permute.                                         */
/*   Prepermute: d_j = n (unclaimed) for all j; then every i claims slot a_i */
/*   and the lowest index wins, d_{a_i} = min(d_{a_i}, i).                   */
/*   Permute: an i whose claim failed (d_{a_i} != i) follows x <- d_x from   */
/*   x = i until it reaches an unclaimed slot, and claims it (d_x = i).      */
/*   Finally c_i = a_{d_i}.                                                  */
/* The paper's loops are "for each" loops; the chains are disjoint (the      */
/* appendix's termination argument), so the serial order used here gives the */
/* same d as any parallel order.  Reading for invalid input: an ancestor     */
/* outside [0, n) is replaced by i itself and ORC_FLAG_BAD_ANCESTOR is set.  */
/* ------------------------------------------------------------------------ */
int orc_permute(const int32_t* a_in, int64_t n, int32_t* c, int32_t* d_out, uint32_t* flags)
{
    int32_t *a, *d;
    int64_t i;
    uint32_t fl = 0;
    if (n < 0 || (n > 0 && (!a_in || !c))) return -1;
    if (n == 0) return 0;
    a = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    d = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    if (!a || !d) { free(a); free(d); return -1; }
    for (i = 0; i < n; ++i) {
        if (a_in[i] < 0 || a_in[i] >= n) { a[i] = (int32_t)i; fl |= ORC_FLAG_BAD_ANCESTOR; }
        else a[i] = a_in[i];
    }
    /* Prepermute */
    for (i = 0; i < n; ++i) d[i] = (int32_t)n;
    for (i = 0; i < n; ++i)
        if (i < d[a[i]]) d[a[i]] = (int32_t)i;
    /* Permute */
    for (i = 0; i < n; ++i) {
        int64_t x = d[a[i]];
        if (x != i) {
            x = i;
            while (d[x] < n) x = d[x];
            d[x] = (int32_t)i;
        }
    }
    for (i = 0; i < n; ++i) c[i] = a[d[i]];
    if (d_out) memcpy(d_out, d, sizeof(int32_t) * (size_t)n);
    if (flags) *flags |= fl;
    free(a);
    free(d);
    return 0;
}

/* Code 9: serial in-place permutation by pairwise swaps.  The paper's loop
 * revisits position i after a swap; a while loop expresses that. */
int orc_permute_serial(int32_t* a, int64_t n)
{
    int64_t i = 0;
    if (n < 0 || (n > 0 && !a)) return -1;
    for (i = 0; i < n; ++i)
        if (a[i] < 0 || a[i] >= n) return -1;
    i = 0;
    while (i < n) {
        int64_t ai = a[i];
        if (ai != i && a[ai] != ai) {
            int32_t t = a[i];
            a[i] = a[ai];
            a[ai] = t;
            continue; /* repeat for the new value at i */
        }
        ++i;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Bootstrap particle filter, Code 1, on the linear-Gaussian model.          */
/* ------------------------------------------------------------------------ */

/* Box & Muller (1958): for u1 in (0, 1] and u2 in [0, 1),
 * sqrt(-2 log u1) cos(2 pi u2) is a standard normal. */
double orc_normal(uint64_t seed, uint32_t index, uint32_t domain, uint32_t step,
                  uint32_t filter, uint32_t offset)
{
    uint32_t x[4];
    double u1, u2;
    draw(seed, index, domain, step, filter, offset, x);
    u1 = ldexp((double)x[0] + 1.0, -32);
    u2 = ldexp((double)x[1], -32);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

void orc_lgssm_init(int32_t n_filters, int32_t n, double s0, uint64_t seed, uint32_t offset,
                    uint32_t filter_base, float* x)
{
    int32_t f, i;
    for (f = 0; f < n_filters; ++f)
        for (i = 0; i < n; ++i)
            x[(int64_t)f * n + i] = (float)(s0 * orc_normal(seed, (uint32_t)i, ORC_DOM_INIT, 0,
                                                             filter_base + (uint32_t)f, offset));
}

void orc_lgssm_move(int32_t n_filters, int32_t n, double phi, double q, double r, uint32_t t,
                    double y_t, uint64_t seed, uint32_t offset, uint32_t filter_base,
                    const int32_t* c, float* x, float* w, double* log_z, int32_t* B)
{
    /* log of the observation density's normalising constant 1 / (r sqrt(2 pi)) */
    const double log_norm = -log(r) - 0.5 * log(6.283185307179586);
    int32_t f, i;
    for (f = 0; f < n_filters; ++f) {
        float* xf = x + (int64_t)f * n;
        float* wf = w + (int64_t)f * n;
        const int32_t* cf = c + (int64_t)f * n;
        double m = -HUGE_VAL, sum = 0.0, beta, b;
        /* copy step before propagation (section 2.3): slots with offspring
         * keep their particle, the others receive their ancestor's */
        for (i = 0; i < n; ++i)
            if (cf[i] != i) xf[i] = xf[cf[i]];
        /* propagate with the transition density, weight with G_t */
        for (i = 0; i < n; ++i) {
            const double e = orc_normal(seed, (uint32_t)i, ORC_DOM_NOISE, t,
                                        filter_base + (uint32_t)f, offset);
            double d, lw;
            xf[i] = (float)(phi * (double)xf[i] + q * e);
            d = (y_t - (double)xf[i]) / r;
            lw = -0.5 * d * d + log_norm;
            if (lw > m) m = lw;
        }
        /* renormalisation by the maximum log-weight (appendix E) */
        for (i = 0; i < n; ++i) {
            const double d = (y_t - (double)xf[i]) / r;
            const double e = exp((-0.5 * d * d + log_norm) - m);
            wf[i] = (float)e;
            sum += e;
        }
        beta = sum / (double)n;
        log_z[f] += m + log(beta);
        /* eq. (B) with epsilon = 1/100 and beta = mean(w) / max(w), max(w) = 1 */
        b = beta >= 1.0 ? 1.0 : ceil(log(0.01) / log1p(-beta));
        if (b < 1.0) b = 1.0;
        if (b > 65536.0) b = 65536.0;
        B[f] = (int32_t)b;
    }
}

/* Kalman (1960) filter for the scalar model: predictive mean m and variance P
 * of x_t given y_1..y_{t-1}; y_t ~ N(m, P + r^2) contributes its log-density
 * and the update conditions x_t on y_t. */
double orc_kalman_loglik(const double* y, int64_t T, double phi, double q, double r, double s0)
{
    double m = 0.0, P = s0 * s0, ll = 0.0;
    int64_t t;
    for (t = 0; t < T; ++t) {
        double S, K, v;
        m = phi * m;
        P = phi * phi * P + q * q;
        S = P + r * r;
        v = y[t] - m;
        ll += -0.5 * (log(6.283185307179586 * S) + v * v / S);
        K = P / S;
        m = m + K * v;
        P = (1.0 - K) * P;
    }
    return ll;
}

/* ------------------------------------------------------------------------ */
/* All-cores legs.  The lanes of Codes 2 and 3 and the vectors of a batch    */
/* are independent and every random number is keyed on (lane, filter), so    */
/* running the serial functions above over disjoint ranges on several host    */
/* threads gives the serial result bit for bit.  Used to time the oracle on  */
/* every host core and to check large cases; the arithmetic is the serial    */
/* code's.                                                                   */
/* ------------------------------------------------------------------------ */
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MT_CHUNK 2048

int orc_threads(int requested)
{
#ifdef _OPENMP
    return requested > 0 ? requested : omp_get_max_threads();
#else
    (void)requested;
    return 1;
#endif
}

int orc_resample_metropolis_mt(const double* w, int64_t n, int32_t B, uint64_t seed,
                               uint32_t filter, uint32_t offset, int32_t* a, int nthreads)
{
    int64_t c, nc;
    if (n < 0 || B < 0 || (n > 0 && (!w || !a))) return -1;
    nc = (n + ORC_MT_CHUNK - 1) / ORC_MT_CHUNK;
#pragma omp parallel for schedule(dynamic, 1) num_threads(orc_threads(nthreads))
    for (c = 0; c < nc; ++c) {
        const int64_t i0 = c * ORC_MT_CHUNK;
        const int64_t i1 = (i0 + ORC_MT_CHUNK < n) ? i0 + ORC_MT_CHUNK : n;
        metropolis_lanes(w, n, B, seed, filter, offset, i0, i1, a);
    }
    return 0;
}

int orc_resample_rejection_mt(const double* w, int64_t n, double w_max, uint32_t max_trials,
                              uint64_t seed, uint32_t filter, uint32_t offset, int32_t* a,
                              uint32_t* trials, uint32_t* flags, int nthreads)
{
    int64_t c, nc;
    uint32_t fl = 0;
    if (n < 0 || max_trials == 0 || (n > 0 && (!w || !a))) return -1;
    nc = (n + ORC_MT_CHUNK - 1) / ORC_MT_CHUNK;
#pragma omp parallel for schedule(dynamic, 1) reduction(|:fl) num_threads(orc_threads(nthreads))
    for (c = 0; c < nc; ++c) {
        const int64_t i0 = c * ORC_MT_CHUNK;
        const int64_t i1 = (i0 + ORC_MT_CHUNK < n) ? i0 + ORC_MT_CHUNK : n;
        fl |= rejection_lanes(w, n, w_max, max_trials, seed, filter, offset, i0, i1, a, trials);
    }
    if (flags) *flags |= fl;
    return 0;
}

/* One resampler per vector of a ragged batch: vector f holds positions
 * [off[f], off[f+1]) and is resampled as a call on it alone with filter id
 * filter_base + f, ancestors local to the vector.  Only the vectors listed
 * in segs[0..n_segs) are computed (their outputs a, and r_out / p_out when
 * not NULL, at the vector's positions).  op: 0 multinomial, 1 stratified,
 * 2 systematic, 3 Metropolis (B[f] steps), 4 rejection (bound w_max). */
int orc_batch_mt(int op, const double* w, const int64_t* off, const int32_t* segs, int32_t n_segs,
                 const int32_t* B, double w_max, uint64_t seed, uint32_t filter_base,
                 uint32_t offset, int32_t* a, double* r_out, double* p_out, uint32_t* flags,
                 int nthreads)
{
    int32_t k;
    int bad = 0;
    uint32_t fl = 0;
    if (op < 0 || op > 4 || !w || !off || !segs || n_segs < 0 || !a) return -1;
    if (op == 3 && !B) return -1;
#pragma omp parallel for schedule(dynamic, 1) reduction(|:fl) reduction(|:bad) \
    num_threads(orc_threads(nthreads))
    for (k = 0; k < n_segs; ++k) {
        const int32_t f = segs[k];
        const int64_t o = off[f], m = off[f + 1] - off[f];
        const uint32_t filt = filter_base + (uint32_t)f;
        uint32_t sfl = 0;
        int rc = 0;
        double* r = r_out ? r_out + o : NULL;
        switch (op) {
        case 0:
            rc = orc_resample_multinomial(w + o, m, seed, filt, offset, a + o, r,
                                          p_out ? p_out + o : NULL, &sfl);
            break;
        case 1:
            rc = orc_resample_stratified(w + o, m, seed, filt, offset, a + o, r, &sfl);
            break;
        case 2:
            rc = orc_resample_systematic(w + o, m, seed, filt, offset, a + o, r, &sfl);
            break;
        case 3:
            rc = orc_resample_metropolis(w + o, m, B[f], seed, filt, offset, a + o);
            break;
        default:
            rc = orc_resample_rejection(w + o, m, w_max, 1u << 20, seed, filt, offset, a + o,
                                        NULL, &sfl);
            break;
        }
        fl |= sfl;
        bad |= (rc != 0);
    }
    if (flags) *flags |= fl;
    return bad ? -1 : 0;
}
