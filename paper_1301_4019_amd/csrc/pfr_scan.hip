// pfr_scan.hip -- the collective resamplers: multinomial (Code 5 of the
// paper), stratified (Code 7) and systematic (Code 8).
//
// All three compute the scaled prefix r_i = n W_i / W_n of the weights and map
// sorted points onto it:
//   stratified   point q_s = s + 1 - u_s in (s, s+1], ancestor = min{i : r_i >= q_s}
//   systematic   the same with one offset u for all strata
//   multinomial  p_k = n S_k / S_n from exponential spacings (sorted uniforms),
//                ancestor = #{i < n-1 : r_i <= p_k}
// i.e. Code 7/8 followed by Code 11, and Code 5 with an upper-bound search.
//
// Exact prefix sums.  The paper shows that a float32 prefix sum biases these
// schemes for large n.  Here each block of 1024 weights is quantised to
// integers q = floor(w * 2^s_b) < 2^53 relative to the block maximum (every
// float32 weight within 2^29 of the block maximum is represented exactly),
// block sums are exact 64-bit integers, and the carries between blocks are
// exact 128-bit integers at one global scale.  Integer sums do not depend on
// the order of addition, so the prefix is deterministic, monotone, exactly
// flat across zero weights and consistent at every block boundary; the only
// rounding is the final map r = n * I / I_total to binary64, itself monotone
// with r = n at the end.
//
// One workgroup of 256 threads handles one block, 4 consecutive weights per
// thread (one 16-byte load each for float32), so that a 2^20 vector runs
// 1024 workgroups, 16 waves per CU.  Passes for one vector:
//   records one record per block (validity, block scale, quantised sum), and
//           one sum per exponential-spacing block of the multinomial scheme.
//   carries one workgroup turns the records into the global scale, the exact
//           carries C_b and the total, and scans the exponential-block sums.
//           With at most 2048 blocks and no exponential blocks this step is
//           folded into the emit kernel: every emit workgroup reduces all
//           records itself, which costs less than one more launch.
//   emit    each block rebuilds its exact prefix, I = C_b + local prefix, and
//           r = n I / Q.  Stratified / systematic: every particle computes its
//           cumulative offspring O_i = #{s : q_s <= r_i} in O(1) with the
//           stratum offsets from an LDS table, and the block's output range
//           [O(C_b), O(C_b+1)) is filled through LDS markers and a max-scan,
//           then written coalesced.  Multinomial: the workgroup rebuilds the
//           exponential blocks whose points fall in its r-range and locates
//           each point with interleaved binary searches in r (LDS).
// Ragged batches run the same steps inside one workgroup per filter.
#include "pfr_kernels.h"

namespace pfr {

namespace {
#include "pfr_scan_common.h"


// ---------------------------------------------------------------- records
// Record of the block at base: validity, reference exponent (block maximum),
// quantised sum.  Same value in every thread.
template <typename T>
__device__ BlockRec block_record(const T* __restrict__ w, int64_t n, int64_t base, WgScratch* s) {
  T x[kPer];
  load4(w, n, base, x);
  uint32_t bad = 0;
  uint32_t emax = 1;
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    if (!weight_ok(x[v])) bad = FLAG_BAD_WEIGHTS;
    else emax = max(emax, (uint32_t)exp_field(x[v]));
  }
  // pack (bad, emax) into one max-reduction: bad dominates
  const uint32_t key = (bad << 16) | emax;
  const uint32_t red = wg_reduce(key, OpMax(), (uint32_t*)s->i);
  BlockRec r;
  r.bad = red >> 16;
  const int e_ref = (int)(red & 0xFFFFu);
  uint64_t sum = 0;
  if (!r.bad) {
#pragma unroll
    for (int v = 0; v < kPer; ++v) sum += quantize(x[v], e_ref);
  }
  r.sum = wg_reduce(sum, OpAdd(), s->u);
  r.scale = scale_of<T>(e_ref);
  return r;
}


__device__ __forceinline__ u128 conv_rec(const BlockRec& r, int32_t gscale) {
  return shift_u128((u128)r.sum, gscale - r.scale);
}

// ---------------------------------------------------------------- carries
// From nb records: global scale, exact exclusive carries C[0..nb] (C[nb] is
// the total) and status.  Whole workgroup; records are read in chunks of
// kBlock, 4 consecutive per thread, all loads of a chunk issued together.
struct Totals {
  u128 Q;
  int32_t gscale;
  uint32_t status;
};

template <typename RecPtr, typename CPtr>
__device__ Totals carries_from_records(uint32_t nb, RecPtr recs, CPtr C, WgScratch* s) {
  const int tid = (int)threadIdx.x;
  uint32_t bad = 0;
  uint32_t smin_key = 0xFFFFFFFFu;  // scale + 2^31, min over non-empty blocks
  for (uint32_t base = 0; base < nb; base += kBlock) {
    BlockRec r[kPer];
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      if (b < nb) r[k] = recs[b];
      else r[k].sum = 0, r[k].scale = 0, r[k].bad = 0;
    }
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      bad |= r[k].bad;
      if (r[k].sum) smin_key = min(smin_key, (uint32_t)r[k].scale ^ 0x80000000u);
    }
  }
  bad = wg_reduce(bad, OpOr(), (uint32_t*)s->i);
  smin_key = wg_reduce(smin_key, OpMin(), (uint32_t*)s->i);
  Totals t;
  // every converted block sum is below 2^(63 + gscale - smin); nb of them stay
  // below 2^kCarryBits
  t.gscale = (smin_key == 0xFFFFFFFFu)
                 ? 0
                 : (int32_t)(smin_key ^ 0x80000000u) + (kCarryBits - 63) - ceil_log2(nb);
  u128 carry = 0;
  for (uint32_t base = 0; base < nb; base += kBlock) {
    u128 v[kPer];
    u128 mine = 0;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      v[k] = (b < nb) ? conv_rec(recs[b], t.gscale) : (u128)0;
      mine += v[k];
    }
    u128 tot;
    u128 run = carry + wg_exclusive(mine, s->v, &tot);
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const uint32_t b = base + (uint32_t)tid * kPer + k;
      if (b < nb) C[b] = run;
      run += v[k];
    }
    carry += tot;
  }
  if (tid == 0) C[nb] = carry;
  __syncthreads();
  t.Q = carry;
  t.status = bad;
  if (!bad && carry == 0) t.status |= FLAG_ZERO_TOTAL;
  return t;
}

// r of the thread's 4 particles of the block at base, given the block's
// exclusive carry Cb and record.
template <typename T>
__device__ void block_r(const T* __restrict__ w, int64_t n, int64_t base, const BlockRec rec,
                        u128 Cb, int32_t gscale, const RMap& rm, double (&r)[kPer],
                        WgScratch* s) {
  T x[kPer];
  load4(w, n, base, x);
  // the block's scale is the same in every lane: keep it scalar, so that the
  // 128-bit shifts below branch on it once instead of selecting per lane
  const int32_t scale = (int32_t)__builtin_amdgcn_readfirstlane(rec.scale);
  const int e_ref = 52 + WTraits<T>::BIAS - scale;
  uint64_t q[kPer];
  uint64_t acc = 0;
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    acc += quantize(x[v], e_ref);
    q[v] = acc;
  }
  uint64_t tot;
  const uint64_t off = wg_exclusive(acc, s->u, &tot);
  const int sh = (int32_t)__builtin_amdgcn_readfirstlane(gscale) - scale;
#pragma unroll
  for (int v = 0; v < kPer; ++v) r[v] = rm(Cb + shift_u128((u128)(off + q[v]), sh));
}

// Emission of block b of a vector (n weights at w, outputs at a_out).
template <typename T, int SCHEME, typename CEPtr>
__device__ void emit_block(const T* __restrict__ w, int64_t n, uint32_t b, const BlockRec rec,
                           u128 Cb, u128 Cb1, int32_t gscale, const RMap& rm, Key key,
                           uint32_t filter, uint32_t offset, CEPtr CE, uint32_t nbe,
                           int32_t* __restrict__ a_out, EmitLds* L, WgScratch* s,
                           int32_t* __restrict__ d_out = nullptr,
                           int32_t* __restrict__ e_out = nullptr,
                           const uint64_t* __restrict__ evals = nullptr) {
  const int64_t P0 = (int64_t)b * kBlock;
  const int cnt = (int)min((int64_t)kBlock, n - P0);
  const double r_lo = rm(Cb);
  const double r_hi = rm(Cb1);
  double r[kPer];
  block_r(w, n, P0, rec, Cb, gscale, rm, r, s);
  if (SCHEME == SCHEME_MULTINOMIAL) {
#pragma unroll
    for (int v = 0; v < kPer; ++v) L->mu.r[threadIdx.x * kPer + v] = r[v];
    __syncthreads();
    emit_multinomial(L->mu.r, cnt, r_lo, r_hi, P0 + cnt == n, n, P0, key, filter, offset, CE, nbe,
                     a_out, s, evals);
  } else {
    const uint32_t u_sys =
        SCHEME == SCHEME_SYSTEMATIC ? draw(key, 0, DOM_STRATA, 0, filter, offset).x : 0u;
    emit_strata<SCHEME == SCHEME_SYSTEMATIC, false>(r, cnt, r_lo, r_hi, n, P0, key, filter,
                                                    offset, u_sys, a_out, &L->st, s, d_out,
                                                    e_out);
  }
}

// ---------------------------------------------------------------- kernels
// One record per weight block (and, for the multinomial scheme, one sum per
// exponential block, whose quantised spacings are kept in `evals` for the
// emission).  No cross-workgroup communication: the kernel boundary makes the
// records visible to the next kernel.
template <typename T, bool MULTI>
__global__ __launch_bounds__(kT) void k_scan_records(const T* __restrict__ w, int64_t n,
                                                     uint32_t nb, Key key, uint32_t offset,
                                                     uint32_t filter,
                                                     BlockRec* __restrict__ recs,
                                                     uint64_t* __restrict__ esums,
                                                     uint64_t* __restrict__ evals) {
  offset = counter_offset(key, offset);
  __shared__ WgScratch s;
  if (blockIdx.x < nb) {
    const BlockRec r = block_record(w, n, (int64_t)blockIdx.x * kBlock, &s);
    if (threadIdx.x == 0) recs[blockIdx.x] = r;
  } else if (MULTI) {
    const uint32_t b = blockIdx.x - nb;
    uint64_t q[kPer];
    exp_values(key, filter, offset, n, b, q);
    store_exp_values(evals, b, q);
    const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
    if (threadIdx.x == 0) esums[b] = sum;
  }
}

// One workgroup: global scale, exact carries C[0..nb], total and status, and
// the exponential-block carries CE[0..nbe] of the multinomial scheme.
template <bool MULTI>
__global__ __launch_bounds__(kT) void k_scan_carries(uint32_t nb, uint32_t nbe,
                                                     ScanHeader* __restrict__ hdr,
                                                     const BlockRec* __restrict__ recs,
                                                     const uint64_t* __restrict__ esums,
                                                     u128* __restrict__ C, u128* __restrict__ CE) {
  __shared__ WgScratch s;
  const Totals t = carries_from_records(nb, recs, C, &s);
  if (MULTI) exp_carries(nbe, esums, CE, &s);
  if (threadIdx.x == 0) {
    hdr->status = t.status;
    hdr->gscale = t.gscale;
    hdr->Q = t.Q;
  }
}

// Direct carries: with few blocks every emit workgroup derives the global
// scale, its own exact carry and the total from all records itself (at most
// kDirectMax records, held in registers), which saves the carry kernel.
constexpr uint32_t kDirectMax = kT * 8;

struct Direct {
  u128 Cb, Cb1, Q;
  int32_t gscale;
  uint32_t status;
};

__device__ Direct direct_carries(uint32_t nb, uint32_t b, const BlockRec* __restrict__ recs,
                                 WgScratch* s) {
  const int tid = (int)threadIdx.x;
  BlockRec r[8];
  uint32_t bad = 0, smin_key = 0xFFFFFFFFu;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t j = (uint32_t)tid + (uint32_t)k * kT;
    if (j < nb) r[k] = recs[j];
    else r[k].sum = 0, r[k].scale = 0, r[k].bad = 0;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    bad |= r[k].bad;
    if (r[k].sum) smin_key = min(smin_key, (uint32_t)r[k].scale ^ 0x80000000u);
  }
  bad = wg_reduce(bad, OpOr(), (uint32_t*)s->i);
  smin_key = wg_reduce(smin_key, OpMin(), (uint32_t*)s->i);
  Direct d;
  d.gscale = (smin_key == 0xFFFFFFFFu)
                 ? 0
                 : (int32_t)(smin_key ^ 0x80000000u) + (kCarryBits - 63) - ceil_log2(nb);
  u128 before = 0, all = 0, own = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint32_t j = (uint32_t)tid + (uint32_t)k * kT;
    const u128 v = (j < nb) ? conv_rec(r[k], d.gscale) : (u128)0;
    all += v;
    if (j < b) before += v;
    if (j == b) own = v;
  }
  d.Cb = wg_reduce(before, OpAdd(), s->v);
  d.Q = wg_reduce(all, OpAdd(), s->v);
  own = wg_reduce(own, OpAdd(), s->v);
  d.Cb1 = d.Cb + own;
  d.status = bad;
  if (!bad && d.Q == 0) d.status |= FLAG_ZERO_TOTAL;
  return d;
}

template <typename T, int SCHEME, bool DIRECT>
__global__ __launch_bounds__(kT) void k_scan_emit(const T* __restrict__ w, int64_t n,
                                                  uint32_t nb, uint32_t nbe, Key key,
                                                  uint32_t offset, uint32_t filter,
                                                  const ScanHeader* __restrict__ hdr,
                                                  const BlockRec* __restrict__ recs,
                                                  const u128* __restrict__ C,
                                                  const u128* __restrict__ CE,
                                                  int32_t* __restrict__ a,
                                                  uint32_t* __restrict__ flags,
                                                  int32_t* __restrict__ d_out,
                                                  int32_t* __restrict__ e_out,
                                                  const uint64_t* __restrict__ evals) {
  offset = counter_offset(key, offset);
  __shared__ EmitLds L;
  __shared__ WgScratch s;
  const uint32_t b = blockIdx.x;
  uint32_t status;
  u128 Cb, Cb1, Q;
  int32_t gscale;
  if (DIRECT) {
    const Direct d = direct_carries(nb, b, recs, &s);
    status = d.status;
    Cb = d.Cb;
    Cb1 = d.Cb1;
    Q = d.Q;
    gscale = d.gscale;
  } else {
    status = hdr->status;
    Cb = C[b];
    Cb1 = C[b + 1];
    Q = hdr->Q;
    gscale = hdr->gscale;
  }
  if (flags && b == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    // identity: every position claims its own slot
    const int64_t P0 = (int64_t)b * kBlock;
    for (int64_t i = P0 + threadIdx.x; i < min(P0 + kBlock, n); i += kT) {
      a[i] = (int32_t)i;
      if (d_out) {
        d_out[i] = (int32_t)i;
        e_out[i] = (int32_t)i;
      }
    }
    return;
  }
  const RMap rm = make_rmap(Q, n);
  emit_block<T, SCHEME>(w, n, b, recs[b], Cb, Cb1, gscale, rm, key, filter, offset, CE, nbe, a,
                        &L, &s, d_out, e_out, evals);
}

// ---------------------------------------------------------------- Code 5
// Multinomial resampling with one independent uniform per particle, as Code 5
// prints it: the scaled prefix r_k = n W_k / W_n of the exact sums is written
// out (binary64, the same values the other schemes compare against), then
// particle i draws u_i = m 2^-53 (m: 21 bits of word 0 and 32 of word 1 of its
// uniform-domain Philox call), p_i = n u_i, and takes #{k < n-1 : r_k <= p_i}.
// The search is two-level: every workgroup holds up to kSplit splitters
// r_{(j+1) S - 1} (S a power of two) in LDS, which narrow each point to S
// candidates, and a bisection over those in global memory finishes it.
template <typename T>
__global__ __launch_bounds__(kT) void k_scan_r(const T* __restrict__ w, int64_t n,
                                               const ScanHeader* __restrict__ hdr,
                                               const BlockRec* __restrict__ recs,
                                               const u128* __restrict__ C,
                                               double* __restrict__ r_out) {
  __shared__ WgScratch s;
  if (hdr->status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) return;
  const uint32_t b = blockIdx.x;
  const RMap rm = make_rmap(hdr->Q, n);
  double r[kPer];
  const int64_t P0 = (int64_t)b * kBlock;
  block_r(w, n, P0, recs[b], C[b], hdr->gscale, rm, r, &s);
#pragma unroll
  for (int v = 0; v < kPer; ++v) {
    const int64_t i = P0 + (int64_t)threadIdx.x * kPer + v;
    if (i < n) r_out[i] = r[v];
  }
}

constexpr int kSplit = 4096;

__global__ __launch_bounds__(kT) void k_multinomial_iid(int64_t n,
                                                        const ScanHeader* __restrict__ hdr,
                                                        const double* __restrict__ r,
                                                        int stride_log2, Key key,
                                                        uint32_t offset, uint32_t filter,
                                                        int32_t* __restrict__ a,
                                                        uint32_t* __restrict__ flags) {
  __shared__ double sp[kSplit];
  offset = counter_offset(key, offset);
  const uint32_t status = hdr->status;
  if (flags && blockIdx.x == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  const bool identity = (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) != 0;
  const int64_t m = n - 1;                  // candidates r_0 .. r_{m-1}
  const int64_t S = (int64_t)1 << stride_log2;
  const int J = (int)(m >> stride_log2);  // splitters inside [0, m), J <= kSplit
  if (!identity)
    for (int j = (int)threadIdx.x; j < J; j += kT) sp[j] = r[((int64_t)(j + 1) << stride_log2) - 1];
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kT;
  for (int64_t i = (int64_t)blockIdx.x * kT + threadIdx.x; i < n; i += stride) {
    if (identity) {
      a[i] = (int32_t)i;
      continue;
    }
    const uint4 x = draw(key, (uint32_t)i, DOM_UNIFORM, 0, filter, offset);
    const uint64_t mb = ((uint64_t)(x.x >> 11) << 32) | (uint64_t)x.y;
    const double p = (double)n * ((double)mb * 0x1p-53);
    // splitters: every r_k with k < lo S is <= p; r_{(lo+1) S - 1} > p if lo < J
    int lo = 0, hi = J;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (sp[mid] <= p) lo = mid + 1;
      else hi = mid;
    }
    int64_t L = (int64_t)lo << stride_log2;
    int64_t H = lo < J ? L + S - 1 : m;  // the answer lies in [L, H]
    while (L < H) {
      const int64_t mid = (L + H) >> 1;
      if (r[mid] <= p) L = mid + 1;
      else H = mid;
    }
    a[i] = (int32_t)L;
  }
}

// Ragged batch: one workgroup per filter runs the reduce, the carries and the
// emission of its own segment, with the records and carries in LDS.
constexpr int kBatchMaxBlocks = 256;  // segments up to 2^18 particles

struct BatchLds {
  BlockRec recs[kBatchMaxBlocks];
  u128 C[kBatchMaxBlocks + 1];
  uint64_t esums[kBatchMaxBlocks];
  u128 CE[kBatchMaxBlocks + 1];
};

template <typename T, int SCHEME>
__global__ __launch_bounds__(kT) void k_scan_batched(const T* __restrict__ w, int64_t n_total,
                                                     const int64_t* __restrict__ offsets,
                                                     uint32_t n_filters, Key key, uint32_t offset,
                                                     uint32_t filter_base, int32_t* __restrict__ a,
                                                     uint32_t* __restrict__ flags) {
  offset = counter_offset(key, offset);
  __shared__ BatchLds B;
  __shared__ EmitLds L;
  __shared__ WgScratch s;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const int tid = (int)threadIdx.x;
  const int64_t base = offsets ? offsets[f] : 0;
  const int64_t n = offsets ? offsets[f + 1] - base : n_total;
  if (n <= 0) return;
  const T* __restrict__ ws = w + base;
  int32_t* __restrict__ as = a + base;
  const uint32_t filt = filter_base + f;
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = (uint32_t)((n + 1 + kBlock - 1) / kBlock);
  if (nbe > kBatchMaxBlocks) {  // segment too long for this path: identity + flag
    for (int64_t i = tid; i < n; i += kT) as[i] = (int32_t)i;
    if (tid == 0 && flags) atomicOr(flags, FLAG_BAD_COUNTS);
    return;
  }
  for (uint32_t b = 0; b < nb; ++b) {
    const BlockRec r = block_record(ws, n, (int64_t)b * kBlock, &s);
    if (tid == 0) B.recs[b] = r;
  }
  if (SCHEME == SCHEME_MULTINOMIAL) {
    for (uint32_t b = 0; b < nbe; ++b) {
      uint64_t q[kPer];
      exp_values(key, filt, offset, n, b, q);
      const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
      if (tid == 0) B.esums[b] = sum;
    }
  }
  __syncthreads();
  const Totals t = carries_from_records(nb, (const BlockRec*)B.recs, (u128*)B.C, &s);
  if (SCHEME == SCHEME_MULTINOMIAL) exp_carries(nbe, (const uint64_t*)B.esums, (u128*)B.CE, &s);
  if (flags && tid == 0 && t.status) atomicOr(flags, t.status);
  if (t.status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    for (int64_t i = tid; i < n; i += kT) as[i] = (int32_t)i;
    return;
  }
  const RMap rm = make_rmap(t.Q, n);
  for (uint32_t b = 0; b < nb; ++b) {
    emit_block<T, SCHEME>(ws, n, b, B.recs[b], B.C[b], B.C[b + 1], t.gscale, rm, key, filt,
                          offset, (const u128*)B.CE, nbe, as, &L, &s);
    __syncthreads();
  }
}

// ---------------------------------------------------------------- segmented batches
// A batch with a workspace runs block-parallel: every 1024-weight block of
// every segment is one workgroup of the records and of the emit kernel, so a
// long segment no longer runs through one workgroup.  Blocks start at each
// segment's first weight (the same blocks as a single call on the segment),
// and one workgroup per segment forms the segment's exact carries, so the
// result is that of one call per segment.

// Exclusive block prefixes over the segments: bstart[f] (weight blocks) and,
// for the multinomial scheme, estart[f] (exponential blocks).  One workgroup.
__global__ __launch_bounds__(kT) void k_seg_prefix(const int64_t* __restrict__ offsets,
                                                   uint32_t n_filters,
                                                   uint32_t* __restrict__ bstart,
                                                   uint32_t* __restrict__ estart) {
  __shared__ WgScratch s;
  uint64_t carry_b = 0, carry_e = 0;
  for (uint32_t base = 0; base < n_filters; base += kT) {
    const uint32_t f = base + threadIdx.x;
    uint64_t nb = 0, ne = 0;
    if (f < n_filters) {
      const int64_t n = offsets[f + 1] - offsets[f];
      nb = n > 0 ? (uint64_t)((n + kBlock - 1) / kBlock) : 0;
      ne = n > 0 ? (uint64_t)((n + 1 + kBlock - 1) / kBlock) : 0;
    }
    uint64_t tb, te;
    const uint64_t xb = wg_exclusive(nb, s.u, &tb);
    const uint64_t xe = wg_exclusive(ne, s.u, &te);
    if (f < n_filters) {
      bstart[f] = (uint32_t)(carry_b + xb);
      if (estart) estart[f] = (uint32_t)(carry_e + xe);
    }
    carry_b += tb;
    carry_e += te;
  }
  if (threadIdx.x == 0) {
    bstart[n_filters] = (uint32_t)carry_b;
    if (estart) estart[n_filters] = (uint32_t)carry_e;
  }
}

// segment f of global block g: the last f with start[f] <= g (start non-decreasing)
__device__ __forceinline__ uint32_t seg_of_block(const uint32_t* __restrict__ start,
                                                 uint32_t n_filters, uint32_t g) {
  uint32_t lo = 0, hi = n_filters;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (start[mid] <= g) lo = mid;
    else hi = mid;
  }
  return lo;
}

template <typename T, bool MULTI>
__global__ __launch_bounds__(kT) void k_seg_records(
    const T* __restrict__ w, const int64_t* __restrict__ offsets, uint32_t n_filters,
    uint32_t grid_b, Key key, uint32_t offset, uint32_t filter_base,
    const uint32_t* __restrict__ bstart, const uint32_t* __restrict__ estart,
    BlockRec* __restrict__ recs, uint64_t* __restrict__ esums, uint64_t* __restrict__ evals) {
  __shared__ WgScratch s;
  offset = counter_offset(key, offset);
  if (blockIdx.x < grid_b) {
    const uint32_t g = blockIdx.x;
    if (g >= bstart[n_filters]) return;
    const uint32_t f = seg_of_block(bstart, n_filters, g);
    const int64_t base = offsets[f];
    const int64_t n = offsets[f + 1] - base;
    const BlockRec r = block_record(w + base, n, (int64_t)(g - bstart[f]) * kBlock, &s);
    if (threadIdx.x == 0) recs[g] = r;
  } else if (MULTI) {
    const uint32_t g = blockIdx.x - grid_b;
    if (g >= estart[n_filters]) return;
    const uint32_t f = seg_of_block(estart, n_filters, g);
    const int64_t n = offsets[f + 1] - offsets[f];
    uint64_t q[kPer];
    exp_values(key, filter_base + f, offset, n, g - estart[f], q);
    store_exp_values(evals, g, q);  // global block g = segment block g - estart[f]
    const uint64_t sum = wg_reduce(q[0] + q[1] + q[2] + q[3], OpAdd(), s.u);
    if (threadIdx.x == 0) esums[g] = sum;
  }
}

// Per segment (one workgroup each): global scale, exact carries C (nb + 1 per
// segment, at cstart = bstart[f] + f), total and status, and the
// exponential-block carries of the multinomial scheme (at estart[f] + f).
struct SegHdr {
  u128 Q;
  int32_t gscale;
  uint32_t status;
  uint64_t pad;
};

template <bool MULTI>
__global__ __launch_bounds__(kT) void k_seg_carries(uint32_t n_filters,
                                                    const uint32_t* __restrict__ bstart,
                                                    const uint32_t* __restrict__ estart,
                                                    const BlockRec* __restrict__ recs,
                                                    const uint64_t* __restrict__ esums,
                                                    u128* __restrict__ C, u128* __restrict__ CE,
                                                    SegHdr* __restrict__ hdr) {
  __shared__ WgScratch s;
  const uint32_t f = blockIdx.x;
  if (f >= n_filters) return;
  const uint32_t b0 = bstart[f], nb = bstart[f + 1] - b0;
  if (nb == 0) return;
  const Totals t = carries_from_records(nb, recs + b0, C + b0 + f, &s);
  if (MULTI) {
    const uint32_t e0 = estart[f];
    exp_carries(estart[f + 1] - e0, esums + e0, CE + e0 + f, &s);
  }
  if (threadIdx.x == 0) {
    hdr[f].Q = t.Q;
    hdr[f].gscale = t.gscale;
    hdr[f].status = t.status;
  }
}

template <typename T, int SCHEME>
__global__ __launch_bounds__(kT) void k_seg_emit(
    const T* __restrict__ w, const int64_t* __restrict__ offsets, uint32_t n_filters, Key key,
    uint32_t offset, uint32_t filter_base, const uint32_t* __restrict__ bstart,
    const uint32_t* __restrict__ estart, const BlockRec* __restrict__ recs,
    const u128* __restrict__ C, const u128* __restrict__ CE, const SegHdr* __restrict__ hdr,
    int32_t* __restrict__ a, uint32_t* __restrict__ flags, const uint64_t* __restrict__ evals) {
  __shared__ EmitLds L;
  __shared__ WgScratch s;
  offset = counter_offset(key, offset);
  const uint32_t g = blockIdx.x;
  if (g >= bstart[n_filters]) return;
  const uint32_t f = seg_of_block(bstart, n_filters, g);
  const int64_t base = offsets[f];
  const int64_t n = offsets[f + 1] - base;
  const uint32_t b = g - bstart[f];
  int32_t* __restrict__ as = a + base;
  const uint32_t status = hdr[f].status;
  if (flags && b == 0 && threadIdx.x == 0 && status) atomicOr(flags, status);
  if (status & (FLAG_BAD_WEIGHTS | FLAG_ZERO_TOTAL)) {
    const int64_t P0 = (int64_t)b * kBlock;
    for (int64_t i = P0 + threadIdx.x; i < min(P0 + kBlock, n); i += kT) as[i] = (int32_t)i;
    return;
  }
  const u128* Cs = C + bstart[f] + f;
  const uint32_t nbe = SCHEME == SCHEME_MULTINOMIAL ? estart[f + 1] - estart[f] : 0u;
  const u128* CEs = SCHEME == SCHEME_MULTINOMIAL ? CE + estart[f] + f : CE;
  const RMap rm = make_rmap(hdr[f].Q, n);
  const uint64_t* evs =
      SCHEME == SCHEME_MULTINOMIAL ? evals + (size_t)estart[f] * kBlock : nullptr;
  emit_block<T, SCHEME>(w + base, n, b, recs[g], Cs[b], Cs[b + 1], hdr[f].gscale, rm, key,
                        filter_base + f, offset, CEs, nbe, as, &L, &s, nullptr, nullptr, evs);
}

template <typename T, int SCHEME>
hipError_t launch_scan_t(const void* wv, int64_t n, Key key, uint32_t offset, uint32_t filter,
                         int32_t* a, void* ws, uint32_t* flags, hipStream_t stream,
                         int32_t* d_out = nullptr, int32_t* e_out = nullptr) {
  const T* w = (const T*)wv;
  constexpr bool multi = SCHEME == SCHEME_MULTINOMIAL;
  const ScanLayout L = scan_layout(n, multi);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  u128* C = (u128*)(base + L.carries);
  uint64_t* esums = (uint64_t*)(base + L.erecs);
  u128* CE = (u128*)(base + L.ecarries);
  uint64_t* evals = multi ? (uint64_t*)(base + L.evals) : nullptr;
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  const uint32_t nbe = multi ? (uint32_t)((n + 1 + kBlock - 1) / kBlock) : 0u;
  hipLaunchKernelGGL((k_scan_records<T, multi>), dim3(nb + nbe), dim3(kT), 0, stream, w, n, nb,
                     key, offset, filter, recs, esums, evals);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (!multi && nb <= (uint32_t)tuning().direct_max_blocks && nb <= kDirectMax) {
    hipLaunchKernelGGL((k_scan_emit<T, SCHEME, true>), dim3(nb), dim3(kT), 0, stream, w, n, nb,
                       nbe, key, offset, filter, hdr, recs, C, CE, a, flags, d_out, e_out,
                       (const uint64_t*)evals);
    return hipGetLastError();
  }
  hipLaunchKernelGGL((k_scan_carries<multi>), dim3(1), dim3(kT), 0, stream, nb, nbe, hdr, recs,
                     esums, C, CE);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_scan_emit<T, SCHEME, false>), dim3(nb), dim3(kT), 0, stream, w, n, nb,
                     nbe, key, offset, filter, hdr, recs, C, CE, a, flags, d_out, e_out,
                     (const uint64_t*)evals);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_scan_scheme(int scheme, const void* w, int64_t n, Key key, uint32_t offset,
                              uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                              hipStream_t stream) {
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      return launch_scan_t<T, SCHEME_MULTINOMIAL>(w, n, key, offset, filter, a, ws, flags, stream);
    case SCHEME_STRATIFIED:
      return launch_scan_t<T, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags, stream);
    default:
      return launch_scan_t<T, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags, stream);
  }
}

template <typename T>
hipError_t launch_batched_scheme(int scheme, const void* w, int64_t n_total,
                                 const int64_t* offsets, uint32_t n_filters, Key key,
                                 uint32_t offset, uint32_t filter_base, int32_t* a,
                                 uint32_t* flags, hipStream_t stream) {
  const T* wt = (const T*)w;
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_MULTINOMIAL>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
    case SCHEME_STRATIFIED:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_STRATIFIED>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
    default:
      hipLaunchKernelGGL((k_scan_batched<T, SCHEME_SYSTEMATIC>), dim3(n_filters), dim3(kT), 0,
                         stream, wt, n_total, offsets, n_filters, key, offset, filter_base, a,
                         flags);
      break;
  }
  return hipGetLastError();
}

template <typename T, int SCHEME>
hipError_t launch_segmented_t(const T* w, int64_t n_total, const int64_t* offsets,
                              uint32_t n_filters, Key key, uint32_t offset, uint32_t filter_base,
                              int32_t* a, void* ws, uint32_t* flags, hipStream_t stream) {
  constexpr bool multi = SCHEME == SCHEME_MULTINOMIAL;
  const SegLayout L = seg_layout(n_total, n_filters, multi);
  char* base = (char*)ws;
  uint32_t* bstart = (uint32_t*)(base + L.bstart);
  uint32_t* estart = multi ? (uint32_t*)(base + L.estart) : nullptr;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  uint64_t* esums = (uint64_t*)(base + L.esums);
  uint64_t* evals = multi ? (uint64_t*)(base + L.evals) : nullptr;
  hipLaunchKernelGGL(k_seg_prefix, dim3(1), dim3(kT), 0, stream, offsets, n_filters, bstart,
                     estart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_seg_records<T, multi>), dim3(L.grid_b + (multi ? L.grid_e : 0u)),
                     dim3(kT), 0, stream, w, offsets, n_filters, L.grid_b, key, offset,
                     filter_base, bstart, estart, recs, esums, evals);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  u128* C = (u128*)(base + L.carries);
  u128* CE = (u128*)(base + L.ecarries);
  SegHdr* hdr = (SegHdr*)(base + L.hdr);
  hipLaunchKernelGGL((k_seg_carries<multi>), dim3(n_filters), dim3(kT), 0, stream, n_filters,
                     bstart, estart, recs, esums, C, CE, hdr);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_seg_emit<T, SCHEME>), dim3(L.grid_b), dim3(kT), 0, stream, w, offsets,
                     n_filters, key, offset, filter_base, bstart, estart, recs, C, CE, hdr, a,
                     flags, (const uint64_t*)evals);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_segmented_scheme(int scheme, const void* w, int64_t n_total,
                                   const int64_t* offsets, uint32_t n_filters, Key key,
                                   uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                                   uint32_t* flags, hipStream_t stream) {
  const T* wt = (const T*)w;
  switch (scheme) {
    case SCHEME_MULTINOMIAL:
      return launch_segmented_t<T, SCHEME_MULTINOMIAL>(wt, n_total, offsets, n_filters, key,
                                                       offset, filter_base, a, ws, flags, stream);
    case SCHEME_STRATIFIED:
      return launch_segmented_t<T, SCHEME_STRATIFIED>(wt, n_total, offsets, n_filters, key,
                                                      offset, filter_base, a, ws, flags, stream);
    default:
      return launch_segmented_t<T, SCHEME_SYSTEMATIC>(wt, n_total, offsets, n_filters, key,
                                                      offset, filter_base, a, ws, flags, stream);
  }
}

}  // namespace

SegLayout seg_layout(int64_t n_total, uint32_t n_filters, bool multinomial) {
  SegLayout L;
  // upper bounds of the block counts: each segment adds at most one partial block
  L.grid_b = (uint32_t)(n_total / kBlock + n_filters);
  L.grid_e = multinomial ? (uint32_t)((n_total + n_filters) / kBlock + n_filters) : 0u;
  L.bstart = 0;
  L.estart = align256(((size_t)n_filters + 1) * sizeof(uint32_t));
  L.recs = L.estart + (multinomial ? align256(((size_t)n_filters + 1) * sizeof(uint32_t)) : 0);
  L.esums = L.recs + align256((size_t)L.grid_b * sizeof(BlockRec));
  L.carries = L.esums + align256((size_t)L.grid_e * sizeof(uint64_t));
  L.ecarries = L.carries + align256(((size_t)L.grid_b + n_filters) * sizeof(u128));
  L.hdr = L.ecarries +
          (multinomial ? align256(((size_t)L.grid_e + n_filters) * sizeof(u128)) : 0);
  L.evals = L.hdr + align256((size_t)n_filters * sizeof(SegHdr));
  L.total = L.evals + (multinomial ? align256((size_t)L.grid_e * kBlock * sizeof(uint64_t)) : 0);
  return L;
}

hipError_t launch_scan_segmented(int scheme, bool f64, const void* w, int64_t n_total,
                                 const int64_t* offsets, uint32_t n_filters, Key key,
                                 uint32_t offset, uint32_t filter_base, int32_t* a, void* ws,
                                 uint32_t* flags, hipStream_t stream) {
  return f64 ? launch_segmented_scheme<double>(scheme, w, n_total, offsets, n_filters, key,
                                               offset, filter_base, a, ws, flags, stream)
             : launch_segmented_scheme<float>(scheme, w, n_total, offsets, n_filters, key,
                                              offset, filter_base, a, ws, flags, stream);
}

ScanLayout scan_layout(int64_t n, bool multinomial) {
  const size_t nb = (size_t)((n + kBlock - 1) / kBlock);
  const size_t nbe = multinomial ? (size_t)((n + 1 + kBlock - 1) / kBlock) : 0;
  ScanLayout L;
  L.recs = 256;
  L.carries = L.recs + align256(nb * sizeof(BlockRec));
  L.erecs = L.carries + align256((nb + 1) * sizeof(u128));
  L.ecarries = L.erecs + align256(nbe * sizeof(uint64_t));
  L.evals = L.ecarries + align256((nbe + 1) * sizeof(u128));
  L.total = L.evals + align256(nbe * kBlock * sizeof(uint64_t));
  return L;
}

size_t batch_scan_lds_bytes() { return sizeof(BatchLds) + sizeof(EmitLds); }

hipError_t launch_scan(int scheme, bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                       uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                       hipStream_t stream) {
  return f64 ? launch_scan_scheme<double>(scheme, w, n, key, offset, filter, a, ws, flags, stream)
             : launch_scan_scheme<float>(scheme, w, n, key, offset, filter, a, ws, flags, stream);
}

size_t multinomial_iid_workspace_bytes(int64_t n) {
  return scan_layout(n, false).total + align256((size_t)n * sizeof(double));
}

template <typename T>
hipError_t launch_multinomial_iid_t(const T* w, int64_t n, Key key, uint32_t offset,
                                    uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                                    hipStream_t stream) {
  const ScanLayout L = scan_layout(n, false);
  char* base = (char*)ws;
  ScanHeader* hdr = (ScanHeader*)base;
  BlockRec* recs = (BlockRec*)(base + L.recs);
  u128* C = (u128*)(base + L.carries);
  double* r = (double*)(base + L.total);
  const uint32_t nb = (uint32_t)((n + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_scan_records<T, false>), dim3(nb), dim3(kT), 0, stream, w, n, nb, key,
                     offset, filter, recs, (uint64_t*)nullptr, (uint64_t*)nullptr);
  hipLaunchKernelGGL((k_scan_carries<false>), dim3(1), dim3(kT), 0, stream, nb, 0u, hdr, recs,
                     (const uint64_t*)nullptr, C, (u128*)nullptr);
  hipLaunchKernelGGL((k_scan_r<T>), dim3(nb), dim3(kT), 0, stream, w, n, hdr, recs, C, r);
  // splitter stride: the smallest power of two leaving at most kSplit splitters
  int sl = 0;
  while (((n - 1) >> sl) > kSplit) ++sl;
  int64_t grid = (n + kT - 1) / kT;
  if (grid > 1024) grid = 1024;
  hipLaunchKernelGGL(k_multinomial_iid, dim3((unsigned)grid), dim3(kT), 0, stream, n, hdr, r, sl,
                     key, offset, filter, a, flags);
  return hipGetLastError();
}

hipError_t launch_multinomial_iid(bool f64, const void* w, int64_t n, Key key, uint32_t offset,
                                  uint32_t filter, int32_t* a, void* ws, uint32_t* flags,
                                  hipStream_t stream) {
  return f64 ? launch_multinomial_iid_t((const double*)w, n, key, offset, filter, a, ws, flags,
                                        stream)
             : launch_multinomial_iid_t((const float*)w, n, key, offset, filter, a, ws, flags,
                                        stream);
}

hipError_t launch_scan_claimed(int scheme, bool f64, const void* w, int64_t n, Key key,
                               uint32_t offset, uint32_t filter, int32_t* a, void* ws,
                               uint32_t* flags, int32_t* d, int32_t* e, hipStream_t stream) {
  if (scheme == SCHEME_STRATIFIED)
    return f64 ? launch_scan_t<double, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags,
                                                          stream, d, e)
               : launch_scan_t<float, SCHEME_STRATIFIED>(w, n, key, offset, filter, a, ws, flags,
                                                         stream, d, e);
  if (scheme == SCHEME_SYSTEMATIC)
    return f64 ? launch_scan_t<double, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags,
                                                          stream, d, e)
               : launch_scan_t<float, SCHEME_SYSTEMATIC>(w, n, key, offset, filter, a, ws, flags,
                                                         stream, d, e);
  return hipErrorInvalidValue;
}

hipError_t launch_scan_batched(int scheme, bool f64, const void* w, int64_t n_total,
                               const int64_t* offsets, uint32_t n_filters, Key key,
                               uint32_t offset, uint32_t filter_base, int32_t* a, uint32_t* flags,
                               hipStream_t stream) {
  return f64 ? launch_batched_scheme<double>(scheme, w, n_total, offsets, n_filters, key, offset,
                                             filter_base, a, flags, stream)
             : launch_batched_scheme<float>(scheme, w, n_total, offsets, n_filters, key, offset,
                                            filter_base, a, flags, stream);
}

}  // namespace pfr
