/*
 * pfresample.h -- C ABI of libpfresample, the particle-filter resampling step
 * of Murray, Lee & Jacob, "Parallel resampling in the particle filter"
 * (arXiv:1301.4019), for AMD Instinct MI355X (gfx950).
 *
 * The resampling step maps a weight vector w in [0, inf)^n to an ancestry
 * vector a in {0..n-1}^n, a_i being the index of the parent of particle i
 * (section 1.1 of the paper, 0-based here).  The library provides the five
 * resamplers the paper studies, the conversion of offspring counts to
 * ancestors and the ancestor permutation that makes in-place propagation safe.
 *
 * Conventions for every entry point
 *   - All arrays are DEVICE pointers owned by the caller.  The library never
 *     allocates, frees or synchronises: a call only enqueues kernels on
 *     `stream` (a hipStream_t; NULL = the default stream) and returns.
 *   - Return value: a pfr_status, reporting only argument and launch errors,
 *     detected synchronously on the host.  Problems in the data (zero total
 *     weight, non-finite weights, bad counts, ...) are reported
 *     asynchronously by OR-ing PFR_FLAG_* bits into *dev_flags (a device
 *     uint32, may be NULL); each has a defined output (see the flags below).
 *   - n is the particle count of one vector, below 2^31.  Ragged batches of
 *     independent vectors are described by pfr_segments (see below); every
 *     index in a batched output is local to its segment.
 *   - Weights are float32 or float64 (pfr_dtype), contiguous.  The collective
 *     resamplers read them with 16-byte vector loads when the segment start
 *     is 16-byte aligned and fall back to scalar loads otherwise.
 *   - Workspaces are caller-provided device buffers of at least
 *     pfr_workspace_bytes() bytes, 256-byte aligned, and must be set to zero
 *     once (pfr_workspace_init) before their first use; the library keeps
 *     them in a reusable state after every call.  Calls that share a
 *     workspace must be ordered (same stream, or synchronised).
 *   - Outputs must not alias inputs.
 *   - Random numbers come from Philox4x32-10 (Salmon et al., SC'11) with
 *     counter (index, domain << 28 | step, filter, offset) and key = seed, so
 *     results are bit-reproducible and independent of the launch shape.
 */
#ifndef PFRESAMPLE_H
#define PFRESAMPLE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define PFR_API __attribute__((visibility("default")))
#else
#define PFR_API
#endif

typedef enum {
    PFR_OK = 0,
    PFR_EINVAL = 1,     /* invalid argument (null pointer, size, alias, ...) */
    PFR_EWORKSPACE = 2, /* workspace missing, too small or misaligned */
    PFR_ELAUNCH = 3,    /* a kernel launch failed */
    PFR_ENOTSUP = 4,    /* combination not supported */
    PFR_ETOOBIG = 5     /* input beyond the fixed scratch of a no-allocation entry point */
} pfr_status;

typedef enum { PFR_F32 = 0, PFR_F64 = 1 } pfr_dtype;

/* Arithmetic of the prefix sum of the collective resamplers.
 *   PFR_SCAN_EXACT      fixed-point sums, exact for the quantised weights
 *                       (default; see below): every float32 weight within
 *                       2^29 of its block maximum, and every binary64 weight
 *                       whose bits lie within 53 bits of the block maximum's
 *                       exponent, is summed without error; smaller ones are
 *                       truncated to that grid (error below max(w) 2^-52)
 *   PFR_SCAN_F64        binary64 sums and scaling
 *   PFR_SCAN_COMP_F32   compensated (two-sum) binary32 sums, binary64 scaling
 *   PFR_SCAN_NAIVE_F32  binary32 sums and the literal binary32 floor(r + u) of
 *                       Codes 7 and 8 (reproduces the bias the paper reports)
 * In the floating-point modes a zero weight may be selected when rounding
 * puts a point exactly on its empty interval. */
typedef enum {
    PFR_SCAN_EXACT = 0,
    PFR_SCAN_F64 = 1,
    PFR_SCAN_COMP_F32 = 2,
    PFR_SCAN_NAIVE_F32 = 3
} pfr_precision;

/* Asynchronous data flags (OR-ed into *dev_flags). */
#define PFR_FLAG_ZERO_TOTAL 1u   /* all weights zero: output is the identity a_i = i */
#define PFR_FLAG_TRIAL_CAP 2u    /* rejection: a particle rejected max_trials proposals; it keeps a_i = i */
#define PFR_FLAG_BAD_COUNTS 4u   /* offspring negative or not summing to n (see offspring_to_ancestors);
                                    also raised by a batched collective call whose segment exceeds
                                    PFR_MAX_BATCH_SEGMENT (that segment gets the identity) */
#define PFR_FLAG_BAD_WEIGHTS 8u  /* a weight is negative, NaN or infinite: output is the identity */
#define PFR_FLAG_BAD_ANCESTOR 16u /* permute: an ancestor outside [0, n) is replaced by its own index */
#define PFR_FLAG_BAD_STEP 32u    /* lgssm_step: step index t outside [1, T]; the state is left unchanged */
#define PFR_FLAG_WMAX_BELOW 64u  /* checks on (pfr_set_checks): a weight exceeds rejection's w_max */
#define PFR_FLAG_NOT_SORTED 128u /* checks on: sorted_hint given with a decreasing ancestry */

/* Longest segment a batched collective call (n_filters > 1) accepts. */
#define PFR_MAX_BATCH_SEGMENT (256 * 1024 - 1)

/* A ragged batch of independent vectors stored back to back: segment f holds
 * global positions [offsets[f], offsets[f+1]).  offsets is a DEVICE int64
 * array of n_filters + 1 non-decreasing values with offsets[0] = 0 and
 * offsets[n_filters] = n_total; it may be NULL when n_filters == 1.
 * max_len is a host-side upper bound on the segment lengths (0 = unknown). */
typedef struct {
    int64_t n_total;
    int32_t n_filters;
    const int64_t* offsets;
    int64_t max_len;
} pfr_segments;

/* Philox key and counter words: seed is the 64-bit key, offset the last
 * counter word (e.g. the time step of a filter), filter_base the filter id of
 * segment 0 (segment f uses filter_base + f).  offset_dev, if not NULL, is a
 * DEVICE uint32 read by the kernels when they run, in place of offset: a
 * captured graph can then advance the offset between replays. */
typedef struct {
    uint64_t seed;
    uint32_t offset;
    uint32_t filter_base;
    const uint32_t* offset_dev;
} pfr_rng;

typedef enum {
    PFR_OP_MULTINOMIAL = 0,
    PFR_OP_STRATIFIED = 1,
    PFR_OP_SYSTEMATIC = 2,
    PFR_OP_METROPOLIS = 3,
    PFR_OP_REJECTION = 4,
    PFR_OP_OFFSPRING_TO_ANCESTORS = 5,
    PFR_OP_PERMUTE = 6,
    PFR_OP_ANCESTORS_TO_OFFSPRING = 7,
    PFR_OP_ESS = 8,
    PFR_OP_MULTINOMIAL_IID = 9,
    PFR_OP_SCALED_PREFIX = 10
} pfr_op;

/* Bytes of workspace the operation needs for these segments (0 if none). */
PFR_API size_t pfr_workspace_bytes(pfr_op op, const pfr_segments* seg, pfr_dtype dtype);

/* Zero a workspace (enqueued on stream; no hipMemset, so it may be captured
 * in a graph).  Needed once per workspace, before its first use. */
PFR_API int pfr_workspace_init(void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------- resamplers
 * Collective resamplers (appendix B of the paper).  They need the total
 * weight, which the library forms as an exact fixed-point prefix sum: each
 * block of 1024 weights is quantised to integers below 2^53 relative to the
 * block maximum and summed exactly, so the result is deterministic and the
 * only rounding is the final scaling r_i = n W_i / W_n to binary64.  Zero
 * weights are never selected.  Output ancestry is sorted (non-decreasing).
 * Workspace: a single vector longer than the tuned single-workgroup length
 * needs one (PFR_EWORKSPACE without); a batch (n_filters > 1) runs
 * block-parallel with one and one workgroup per segment without one (a NULL
 * workspace), with identical results.  The floating-point precision modes
 * ignore a batch workspace.
 */

/* The scaled prefix r_i = n W_i / W_n (binary64, r_{n-1} = n) that the
 * collective resamplers of a single vector compare their points against in
 * the given precision mode (sections 3.1 and 3.2: it carries the whole effect
 * of the prefix sum's arithmetic).  Given r, the stratified and systematic
 * schemes give particle i r_i - r_{i-1} offspring in expectation (also the
 * multinomial scheme, up to its cap at n - 1), so
 * sum_i (r_i - r_{i-1} - n w_i / W)^2 is the deterministic bias of the mode.
 * For analysis and tests; single vectors (n_filters = 1) only.  Workspace:
 * pfr_workspace_bytes(PFR_OP_SCALED_PREFIX, ...).  Zero or invalid weights
 * leave r_out unwritten and raise the flags of the resamplers. */
PFR_API int pfr_scaled_prefix(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                              pfr_precision precision, double* r_out, void* ws, size_t ws_bytes,
                              uint32_t* dev_flags, void* stream);

/* Multinomial resampling (Code 5): draws the order statistics of n uniforms
 * from exponential spacings E_k = -log((x + 1/2) 2^-32), k = 0..n, taken from
 * word k&3 of Philox call k>>2 (domain 1), p_k = n S_k / S_n, and sets
 * a_k = #{i < n-1 : r_i <= p_k}. */
PFR_API int resample_multinomial(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                         pfr_precision precision, pfr_rng rng,
                         int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                         void* stream);

/* Multinomial resampling as Code 5 prints it, with one independent uniform
 * per particle: u_i = m 2^-53, m = (word 0 >> 11) 2^32 + word 1 of Philox call
 * (i, 5<<28, filter, offset), p_i = n u_i (binary64), and
 * a_i = #{k < n-1 : r_k <= p_i} over the same exact prefix r as
 * resample_multinomial.  Same law as resample_multinomial, but the output is
 * NOT sorted (permute it with sorted_hint = 0), and each particle pays a
 * search over r.  Single vectors only (PFR_ENOTSUP for n_filters > 1);
 * workspace required (the scan records plus r, 8 bytes per particle). */
PFR_API int resample_multinomial_iid(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                                     pfr_rng rng, int32_t* ancestors, void* ws, size_t ws_bytes,
                                     uint32_t* dev_flags, void* stream);

/* Stratified resampling (Code 7 then Code 11): stratum s takes the point
 * s + 1 - u_s with u_s = word s&3 of Philox call s>>2 (domain 0) times 2^-32,
 * and a_s = min{i : r_i >= s + 1 - u_s}. */
PFR_API int resample_stratified(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                        pfr_precision precision, pfr_rng rng,
                        int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                        void* stream);

/* Systematic resampling (Code 8): as stratified with the single offset
 * u = word 0 of Philox call 0 (domain 0) times 2^-32 for every stratum. */
PFR_API int resample_systematic(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                        pfr_precision precision, pfr_rng rng,
                        int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                        void* stream);

/* Metropolis resampling (Code 2): lane i starts at k = i and runs B steps.
 * Lane i's words come from Philox calls (i, 2<<28 | c), word m being word
 * m&3 of call m>>2; step s takes words x0, x1, x2 = 3s, 3s+1, 3s+2 (four steps
 * per three calls), proposes j = floor(((x1<<32)|x0) n / 2^64) with
 * u = (x2 + 1) 2^-32, and moves to j when u w_k <= w_j, decided exactly for
 * every weight, subnormal binary64 weights included (one fused multiply-add,
 * rounded once, keeps the sign of u w_k - w_j whenever the weights lie on the
 * 2^-1042 lattice; a zero result with w_k below 2^-900 is re-decided on both
 * weights scaled by 2^200).  B_dev (device int32[n_filters], may be NULL) overrides B per segment.
 * No collective operation: the chains are independent, so the output does
 * not depend on the launch shape.  Segments of up to 16K (float32) or 8K
 * (float64) weights, and with pfr_segments.max_len set up to 32K / 16K, are
 * staged in LDS.  The workspace (may be NULL, ws_bytes 0) holds, for a single
 * long vector of less than 2^31 bytes of weights, a table of power-of-two
 * weight bounds per bucket of particles that lets most rejected proposals
 * skip the load of w_j; it changes the speed, never the result. */
PFR_API int resample_metropolis(const void* w, pfr_dtype dtype, const pfr_segments* seg, int32_t B,
                        const int32_t* B_dev, pfr_rng rng, int32_t* ancestors, void* ws,
                        size_t ws_bytes, void* stream);

/* Rejection resampling (Code 3): particle i first proposes j = i, then draws
 * j as above from Philox call (i, 2<<28 | t) for trial t >= 1 (every trial
 * takes u from its own call), and keeps the first j with u w_max <= w_j
 * (decided exactly as for resample_metropolis, for any w_max).  w_max must bound the weights (else the output is
 * biased); w_max_dev (device double[n_filters], may be NULL) overrides it per
 * segment.  After max_trials trials (>= 1) a particle keeps a_i = i and
 * PFR_FLAG_TRIAL_CAP is raised.  No collective operation; LDS staging and
 * the optional workspace (weight-bound table) as for resample_metropolis. */
PFR_API int resample_rejection(const void* w, pfr_dtype dtype, const pfr_segments* seg, double w_max,
                       const double* w_max_dev, uint32_t max_trials, pfr_rng rng,
                       int32_t* ancestors, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                       void* stream);

/* Partial rejection control (section 2.2, after Liu et al. 1998): with a
 * bound v_max that need not bound the weights, the clipped weights
 * v_i = min(w_i, v_max) are resampled as by resample_rejection with bound
 * v_max -- which accepts exactly when u v_max <= w_j, so the ancestors are
 * those of resample_rejection(w, v_max) -- and the outcome is weighted:
 * weights_out[i] (same type as w) = w_{a_i} / v_{a_i}, i.e. w_{a_i} / v_max
 * where w_{a_i} > v_max and 1 elsewhere (binary64 quotient, rounded); a lane
 * that hits max_trials keeps a_i = i, gets w_i / v_i (0 if w_i is not
 * positive) and raises PFR_FLAG_TRIAL_CAP.  v_max_dev (device
 * double[n_filters], may be NULL) overrides v_max per segment.  Workspace as
 * for resample_rejection.  weights_out must not alias w or ancestors. */
PFR_API int resample_partial_rejection(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                                       double v_max, const double* v_max_dev,
                                       uint32_t max_trials, pfr_rng rng, int32_t* ancestors,
                                       void* weights_out, void* ws, size_t ws_bytes,
                                       uint32_t* dev_flags, void* stream);

/* Scheme parameters of resample_permuted (the fields of other schemes are
 * ignored). */
typedef struct {
    pfr_precision precision;  /* multinomial, stratified, systematic */
    int32_t B;                /* Metropolis steps; B_dev (device int32[n_filters]) may override */
    const int32_t* B_dev;
    double w_max;             /* rejection bound; w_max_dev (device double[n_filters]) may override */
    const double* w_max_dev;
    uint32_t max_trials;      /* rejection trial cap (>= 1) */
} pfr_scheme_params;

/* Bytes of workspace for resample_permuted (256-byte aligned; zero it once
 * with pfr_workspace_init). */
PFR_API size_t pfr_resample_permuted_workspace_bytes(pfr_op scheme, const pfr_segments* seg,
                                                     pfr_dtype dtype);

/* Resampling and the ancestor permutation in one call (the paper times
 * resampling until an ancestry satisfying eq. (predicate) is delivered,
 * section 3.4, and appends Prepermute to every kernel that produces an
 * ancestry, appendix E).  scheme is one of PFR_OP_MULTINOMIAL ..
 * PFR_OP_REJECTION.  Writes the scheme's ancestry to `ancestors` and its
 * Code 10 permutation to `permuted`, bit for bit what resample_<scheme>
 * followed by permute_ancestors (sorted_hint set for the collective schemes)
 * would write, with the same flags.  For a long single vector of an exact
 * collective scheme (multinomial, stratified, systematic: sorted ancestries)
 * the emission writes the claim vector and the marked ancestry itself, so
 * only the resolve pass follows; the other
 * cases run the two steps one after the other (claiming inside Metropolis and
 * rejection, with atomics beside their random weight loads, measured slower
 * than the separate claim pass on MI355X). */
PFR_API int resample_permuted(pfr_op scheme, const void* w, pfr_dtype dtype,
                              const pfr_segments* seg, const pfr_scheme_params* params,
                              pfr_rng rng, int32_t* ancestors, int32_t* permuted, void* ws,
                              size_t ws_bytes, uint32_t* dev_flags, void* stream);

/* ---------------------------------------------------------------- auxiliaries */

/* Offspring counts to ancestors (appendix D, Code 11 after an inclusive prefix
 * sum): a[O_{i-1} .. O_i) = i.  A negative count is used as 0; positions at
 * or beyond n are dropped; if the counts sum to less than n the remaining
 * positions s get a_s = s.  Each of these raises PFR_FLAG_BAD_COUNTS. */
PFR_API int offspring_to_ancestors(const int32_t* offspring, const pfr_segments* seg, int32_t* ancestors,
                           void* ws, size_t ws_bytes, uint32_t* dev_flags, void* stream);

/* Ancestor permutation (section 2.3 and appendix C, Code 10): returns in
 * `permuted` a permutation c of `ancestors` with c_j = j for every j that
 * appears in the ancestry (a particle with offspring is its own first
 * descendant), so that the copy x_i <- x_{c_i} for c_i != i followed by
 * in-place propagation never reads a slot that is written.  Slot j is claimed by the lowest i with
 * a_i = j; unsuccessful claimers follow x <- d_x to a free slot.  With
 * sorted_hint != 0 the input must be non-decreasing (as produced by the
 * collective resamplers) and the claim needs no atomics; otherwise any
 * ancestry is accepted.  An ancestor outside [0, n) is treated as its own
 * index and raises PFR_FLAG_BAD_ANCESTOR.  The workspace holds the claim
 * vector and the marked ancestry (8 bytes per particle at least); with the
 * size pfr_workspace_bytes(PFR_OP_PERMUTE, ...) reports, a single unsorted
 * vector is claimed by buckets of slots in LDS instead of global atomics
 * (8 more bytes per particle and the bucket counts).  Either claim gives the
 * same result. */
PFR_API int permute_ancestors(const int32_t* ancestors, const pfr_segments* seg, int32_t sorted_hint,
                      int32_t* permuted, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                      void* stream);

/* permute_ancestors without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, result and flags as
 * permute_ancestors with the workspace removed; the claim vector, the
 * marked ancestry and (when they fit) the bucket counts and pairs live in a
 * static device array of
 * PFR_NOALLOC_SCRATCH_BYTES inside the library (one per GPU, held until the
 * process ends), so n_total is limited to PFR_NOALLOC_MAX_N: a longer input
 * returns PFR_ETOOBIG and enqueues nothing.  Every call on one GPU uses that
 * GPU's one array: calls that overlap in time on the same GPU (different
 * streams, or host threads without ordering) race and give undefined
 * results; order them.  The call allocates nothing (no hipMalloc, no library
 * allocation); its first call on a device looks up the array's address. */
#define PFR_NOALLOC_MAX_N (1 << 22)
#define PFR_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
PFR_API int permute_ancestors_noalloc(const int32_t* ancestors, const pfr_segments* seg,
                                      int32_t sorted_hint, int32_t* permuted,
                                      uint32_t* dev_flags, void* stream);

/* Ancestors to offspring counts (appendix D, Code 12): o_j = #{i : a_i = j}.
 * With sorted_hint != 0 the ancestry must be non-decreasing (as produced by
 * the collective resamplers; otherwise the counts are unspecified) and the
 * counts are formed without atomics, from the first and last position of each
 * run; otherwise any ancestry is counted (atomic additions, as in Code 12).
 * An ancestor outside [0, n) is not counted and raises PFR_FLAG_BAD_ANCESTOR.
 * No workspace. */
PFR_API int ancestors_to_offspring(const int32_t* ancestors, const pfr_segments* seg,
                                   int32_t sorted_hint, int32_t* offspring, uint32_t* dev_flags,
                                   void* stream);

/* Effective sample size (section 3.4): ess[f] = (sum w)^2 / (w^T w) for every
 * segment f (ess: DEVICE double[n_filters]).  Binary64 sums of weights scaled
 * by powers of two (exact), in an order fixed by the segment length, so the
 * result is reproducible and free of overflow for any finite weights; its
 * relative error is below (3d + 8) 2^-53 with d = 31 + ceil(P / 64), P the
 * number of 4096-weight chunks of the segment.  An empty or all-zero segment
 * gives 0 (all-zero raises PFR_FLAG_ZERO_TOTAL); a negative or non-finite
 * weight gives NaN and PFR_FLAG_BAD_WEIGHTS.  Workspace required
 * (pfr_workspace_bytes(PFR_OP_ESS, ...); it needs no initialisation). */
PFR_API int effective_sample_size(const void* w, pfr_dtype dtype, const pfr_segments* seg,
                                  double* ess, void* ws, size_t ws_bytes, uint32_t* dev_flags,
                                  void* stream);

/* The copy step of section 2.3, in place: x_i <- x_{c_i} for every particle i
 * with c_i != i, c = `permuted` (the output of permute_ancestors, local to its
 * segment).  The state of particle g (global index) has `dim` components of
 * elem_bytes bytes each (1, 2, 4, 8 or 16), component k at element
 * g * particle_stride + k * component_stride of x (strides in elements, >= 1;
 * either component_stride == 1 and particle_stride >= dim, or particle_stride
 * == 1 and component_stride >= n_total, or dim == 1).  x must be aligned to
 * elem_bytes.  A particle whose c_i lies outside [0, n) or whose source is
 * itself overwritten (c_{c_i} != c_i, which the in-place predicate forbids)
 * keeps its state and raises PFR_FLAG_BAD_ANCESTOR, so the step never races.
 * No workspace. */
PFR_API int copy_particles(const int32_t* permuted, const pfr_segments* seg, void* x,
                           size_t elem_bytes, int32_t dim, int64_t particle_stride,
                           int64_t component_stride, uint32_t* dev_flags, void* stream);

/* ---------------------------------------------------------------- filter
 * The bootstrap particle filter of Code 1 (section 1: K_t the transition
 * and G_t the observation density) for the 1-D linear-Gaussian model
 *   x_0 ~ N(0, s0^2),  x_t = phi x_{t-1} + q e_t,  y_t = x_t + r v_t,
 * batched over n_filters independent filters of n particles each (filter f
 * holds positions [f n, (f+1) n) of x, w, ancestors and permuted).  State x
 * and weights w are binary32; log Z per filter is binary64.
 *
 * Random numbers: x_0 of particle i of filter f takes Philox counter
 * (i, 4<<28, filter_base + f, offset), its noise at step t the counter
 * (i, 3<<28 | t, filter_base + f, offset); a standard normal is
 * sqrt(-2 log u1) cos(2 pi u2) with u1 = (x0 + 1) 2^-32, u2 = x1 2^-32.  The
 * resampler at step t runs with counter offset t. */
typedef struct {
    double phi, q, r, s0;
} pfr_lgssm;

/* Workspace bytes of lgssm_init / lgssm_step (segment offsets + permutation). */
PFR_API size_t lgssm_workspace_bytes(int32_t n_filters, int32_t n);

/* x_0 ~ N(0, s0^2), w = 1, log_z = 0, B_dev = 1, *t_dev = 1; writes the
 * segment offsets into the workspace. */
PFR_API int lgssm_init(const pfr_lgssm* model, int32_t n_filters, int32_t n, pfr_rng rng,
                       float* x, float* w, double* log_z, int32_t* B_dev, uint32_t* t_dev,
                       void* ws, size_t ws_bytes, void* stream);

/* One step t = *t_dev (read on the device) of Code 1 for every filter:
 *   a = Ancestors(w) by `scheme` (a resampler op; Metropolis takes B_dev,
 *       rejection the bound 1, which the shifted weights never exceed),
 *   c = permute_ancestors(a), x_i <- x_{c_i} in place,
 *   x_i <- phi x_i + q e_i, lw_i = log N(y_t; x_i, r^2) (binary64),
 *   log_z[f] += m + log(mean exp(lw - m)) with m = max lw, w_i = exp(lw_i - m),
 *   B_dev[f] = ceil(log(1/100) / log(1 - mean w)) in [1, 65536] (eq. (B)),
 * then *t_dev += 1.  y is a DEVICE binary64 array of T observations with
 * y[t-1] = y_t; a step with t outside [1, T] leaves x, w and log_z unchanged
 * and raises PFR_FLAG_BAD_STEP.  Every argument is read when the kernels run,
 * so the step can be captured once and replayed T times.  `ancestors` and
 * `permuted` receive a and c. */
PFR_API int lgssm_step(const pfr_lgssm* model, pfr_op scheme, pfr_precision precision,
                       int32_t n_filters, int32_t n, const double* y, int32_t T, uint32_t* t_dev,
                       pfr_rng rng, float* x, float* w, double* log_z, int32_t* B_dev,
                       int32_t* ancestors, int32_t* permuted, void* ws, size_t ws_bytes,
                       uint32_t* dev_flags, void* stream);

/* ---------------------------------------------------------------- tuning
 * Launch parameters of the library, chosen per machine by the autotuner
 * (paper_1301_4019_amd/autotune.py) and loaded at start-up.  None of them
 * changes a result: random numbers are drawn per particle and the exact
 * prefix sums do not depend on how they are split, so every setting gives the
 * same bits.  Process-wide; set them before launching work. */
#define PFR_TUNING_VERSION 2
typedef struct {
    int32_t version;                /* PFR_TUNING_VERSION */
    int32_t single_wg_max;          /* collective: single vectors up to this length run in one
                                       workgroup, without workspace [0, PFR_MAX_BATCH_SEGMENT] */
    int32_t direct_max_blocks;      /* exact collective: up to this many 1024-weight blocks every
                                       emit workgroup forms its own carries [0, 2048] */
    int32_t metropolis_table_min_B; /* long single vectors: the bound-table Metropolis kernel
                                       from this many steps on (0 = never) */
    int32_t rejection_table;        /* long single vectors: rejection with the bound table (0/1) */
    int32_t rejection_per_wave;     /* particles per wave of the rejection schedule [64, 4096] */
    int32_t metropolis_chunk;       /* particles per workgroup of the global-memory Metropolis
                                       kernel, a multiple of 256 in [256, 8192] */
    /* ragged batches (n_filters > 1) */
    int32_t batch_scan_wg_max_len;  /* collective, exact prefix: a batch whose longest segment is
                                       at most this runs one workgroup per segment even with a
                                       workspace, longer ones block-parallel
                                       [0, PFR_MAX_BATCH_SEGMENT] */
    int32_t batch_stage_max_kb;     /* Metropolis / rejection: largest LDS tier for staging a
                                       segment's weights (16, 64 or 128 KB); longer segments
                                       gather from global memory in the same launch */
    int32_t batch_metropolis_chunk; /* particles per 1024-thread workgroup of the batched
                                       Metropolis kernel, a multiple of 1024 in [1024, 65536] */
    int32_t batch_rejection_per_wave; /* particles per wave of the batched rejection kernel
                                       [64, 4096] */
    int32_t batch_permute_lds_max;  /* segments up to this length are permuted in LDS, one
                                       workgroup each (4096, 8192 or 16384) */
} pfr_tuning;

PFR_API void pfr_tuning_defaults(pfr_tuning* t);
PFR_API int pfr_get_tuning(pfr_tuning* t);
/* PFR_EINVAL (nothing changed) if a field is out of range or the version differs. */
PFR_API int pfr_set_tuning(const pfr_tuning* t);
/* Loads a flat JSON object with the fields above (absent ones keep their
 * value); PFR_EINVAL if the file is unreadable or a value is invalid. */
PFR_API int pfr_load_tuning(const char* path);

/* ---------------------------------------------------------------- misc */
PFR_API const char* pfr_status_string(int status);
/* Library version, e.g. "0.1.0". */
PFR_API const char* pfr_version(void);

/* Precondition checks, for debugging (off by default).  The hot path does not
 * test what the operations assume: finite, non-negative weights for
 * resample_metropolis, resample_rejection and resample_partial_rejection (the
 * collective schemes test them anyway), a w_max (or w_max_dev entry) at least
 * every weight of its segment for resample_rejection (section 2.2: a smaller
 * bound biases the output), and a non-decreasing ancestry inside every
 * segment where sorted_hint != 0 (permute_ancestors,
 * permute_ancestors_noalloc, ancestors_to_offspring).  With the checks on,
 * these calls first enqueue one pass over their input that ORs each
 * violation (PFR_FLAG_BAD_WEIGHTS, PFR_FLAG_WMAX_BELOW, PFR_FLAG_NOT_SORTED)
 * into *dev_flags where the call has it and into a word the library keeps per
 * GPU, and a sorted_hint is not relied on: the call takes the path for any
 * ancestry, which gives the same result for sorted input and the defined
 * result for any other.  Outputs of valid inputs are unchanged; the extra
 * pass makes the calls slower.  The setting is process-wide. */
PFR_API int pfr_set_checks(int32_t on);
PFR_API int32_t pfr_get_checks(void);
/* Waits for the stream, stores in *flags the violations recorded on the
 * current GPU since the previous call (or since start-up) and clears them.
 * It synchronises, so it is not for use under graph capture. */
PFR_API int pfr_take_check_flags(void* stream, uint32_t* flags);

/* Rounds of the Philox4x32 generator this library was built with: 10 (the
 * generator named above) unless a study build chose another count. */
PFR_API int pfr_philox_rounds(void);

#ifdef __cplusplus
}
#endif
#endif /* PFRESAMPLE_H */
